"""Tucker-ALS (HOOI) on MI355X: Python binding of libtucker_mi355x.so.

Argument marshalling only: every step of the decomposition runs in the library's HIP
kernels.  PyTorch provides device memory and the stream.  Sec. III-B of arXiv 2104.04726
defines the computation:

    X ~ G x_1 U_1 ... x_N U_N,   T-HOSVD start, HOOI sweeps via mode-n Gram eigenvectors.

Example::

    import torch, paper_2104_04726_amd as tk
    x = torch.randn(64, 48, 3, 6, device="cuda")
    res = tk.decompose(x, ranks=(16, 12, 3, 4), max_iters=10)
    xhat = tk.reconstruct(res.core, res.factors)
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

from . import _lib
from ._lib import FP32, BF16, FP16, FP8_E4M3  # noqa: F401

__all__ = ["Context", "TuckerError", "Result", "decompose", "reconstruct", "default_context", "validate",
           "workspace_size", "Server", "Served"]

_PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp16": FP16, "fp8": FP8_E4M3, "fp8_e4m3": FP8_E4M3}


class TuckerError(RuntimeError):
    def __init__(self, code: int, message: str):
        self.code = int(code)
        super().__init__(f"{_lib.status_name(code)}: {message}")


@dataclass
class Result:
    core: "object"                  # torch.Tensor (R_1, ..., R_N), float32, on the device
    factors: List["object"]         # torch.Tensor (s_n, R_n), float32, orthonormal columns
    fit: float                      # 1 - ||X - Xhat|| / ||X|| from the explicit residual
    fit_history: List[float] = field(default_factory=list)   # fit_0 .. fit_sweeps (||G||-based)
    sweeps: int = 0
    stats: dict = field(default_factory=dict)


def _check(code: int, ctx=None):
    if code != _lib.OK:
        msg = ""
        if ctx is not None:
            raw = _lib.lib().tucker_last_error(ctx)
            msg = raw.decode() if raw else ""
        raise TuckerError(code, msg)


def _f32_device(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    return t.contiguous()


def validate(dims: Sequence[int], ranks: Sequence[int], max_iters: int = 0, tol: float = 0.0) -> int:
    """Host-only validation; returns the status code (0 = ok)."""
    n = len(dims)
    if len(ranks) != n:
        return _lib.ERR_INVALID_ARG
    return int(_lib.lib().tucker_validate(n, _lib.i64(dims), _lib.i64(ranks), int(max_iters), float(tol)))


def workspace_size(dims: Sequence[int], ranks: Sequence[int], precision: str = "fp32") -> int:
    out = C.c_size_t(0)
    _check(_lib.lib().tucker_workspace_size(len(dims), _lib.i64(dims), _lib.i64(ranks),
                                            _PRECISIONS[precision], C.byref(out)))
    return int(out.value)


class Context:
    """A library context bound to one device and one stream (torch's current stream by default)."""

    def __init__(self, device: int = 0, stream=None, inner_iters: int = 1, init_iters: int = 20,
                 seed: int = 0x5EED, hbm_budget_bytes: int = 0, precision: str = "fp32",
                 refine_sweeps: int = 1, timing: bool = False, use_graphs: bool = False, inner_tol: float = 0.0,
                 wait_spin_limit: int = 0, start: str = "thosvd", autotune: bool = False, pp_tol: float = 0.0,
                 oversample: int = 0, timing_stages=None):
        import torch
        lib = _lib.lib()
        opts = _lib.Options()
        lib.tucker_default_options(C.byref(opts))
        opts.device = int(device)
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.torch_stream = stream
        opts.stream = C.c_void_p(int(stream.cuda_stream)) if hasattr(stream, "cuda_stream") else C.c_void_p(stream)
        opts.inner_iters = int(inner_iters)
        opts.init_iters = int(init_iters)
        opts.seed = int(seed)
        opts.hbm_budget_bytes = int(hbm_budget_bytes)
        opts.precision = _PRECISIONS[precision]
        opts.refine_sweeps = int(refine_sweeps)
        opts.timing = 1 if timing else 0
        opts.use_graphs = 1 if use_graphs else 0
        opts.inner_tol = float(inner_tol)
        opts.wait_spin_limit = int(wait_spin_limit)
        opts.start = {"thosvd": _lib.START_THOSVD, "sthosvd": _lib.START_STHOSVD}[start]
        opts.autotune = 1 if autotune else 0
        opts.pp_tol = float(pp_tol)
        opts.oversample = int(oversample)
        opts.timing_stages = sum(1 << _lib.STAGES.index(n) for n in (timing_stages or ()))
        self.device = int(device)
        self._h = C.c_void_p()
        _check(lib.tucker_create(C.byref(opts), C.byref(self._h)))

    def close(self):
        if self._h:
            _lib.lib().tucker_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---------------------------------------------------------------- decomposition
    def decompose(self, x, ranks: Sequence[int], max_iters: int = 10, tol: float = 0.0,
                  init_factors: Optional[Sequence] = None) -> Result:
        import torch
        x = _f32_device(x, "x")
        dims = list(x.shape)
        ranks = [int(r) for r in ranks]
        n = len(dims)
        if len(ranks) != n:
            raise TuckerError(_lib.ERR_INVALID_ARG, "len(ranks) != x.dim()")
        dev = x.device
        core = torch.empty(ranks, dtype=torch.float32, device=dev)
        factors = [torch.empty((dims[i], ranks[i]), dtype=torch.float32, device=dev) for i in range(n)]
        fptrs = (C.c_void_p * n)(*[f.data_ptr() for f in factors])
        iptrs = None
        keep = []
        if init_factors is not None:
            init = [_f32_device(u, "init_factors") for u in init_factors]
            keep = init
            iptrs = (C.c_void_p * n)(*[u.data_ptr() for u in init])
        fit = C.c_double(0.0)
        hist = (C.c_double * (max_iters + 1))()
        sweeps = C.c_int(0)
        code = _lib.lib().tucker_decompose_ex(
            self._h, C.c_void_p(x.data_ptr()), n, _lib.i64(dims), _lib.i64(ranks), int(max_iters), float(tol),
            iptrs, C.c_void_p(core.data_ptr()), fptrs, C.byref(fit), hist, C.byref(sweeps))
        del keep
        _check(code, self._h)
        return Result(core, factors, float(fit.value), [float(hist[i]) for i in range(sweeps.value + 1)],
                      int(sweeps.value), self.stats())

    def reconstruct(self, core, factors):
        import torch
        core = _f32_device(core, "core")
        factors = [_f32_device(u, "factor") for u in factors]
        dims = [int(u.shape[0]) for u in factors]
        ranks = list(core.shape)
        out = torch.empty(dims, dtype=torch.float32, device=core.device)
        fptrs = (C.c_void_p * len(factors))(*[u.data_ptr() for u in factors])
        _check(_lib.lib().tucker_reconstruct(self._h, C.c_void_p(core.data_ptr()), fptrs, len(dims),
                                             _lib.i64(dims), _lib.i64(ranks), C.c_void_p(out.data_ptr())), self._h)
        return out

    # ---------------------------------------------------------------- codec hand-off
    def order_core(self, core, factors):
        """All-orthogonal, energy-ordered core: returns (core, factors, sigma list per mode)."""
        import torch
        core = _f32_device(core, "core")
        factors = [_f32_device(u, "factor") for u in factors]
        dims = [int(u.shape[0]) for u in factors]
        ranks = list(core.shape)
        out = torch.empty_like(core)
        fout = [torch.empty_like(u) for u in factors]
        sig = torch.empty(sum(ranks), dtype=torch.float64, device=core.device)
        fin = (C.c_void_p * len(factors))(*[u.data_ptr() for u in factors])
        fo = (C.c_void_p * len(factors))(*[u.data_ptr() for u in fout])
        _check(_lib.lib().tucker_order_core(self._h, C.c_void_p(core.data_ptr()), fin, len(dims), _lib.i64(dims),
                                            _lib.i64(ranks), C.c_void_p(out.data_ptr()), fo,
                                            C.c_void_p(sig.data_ptr())), self._h)
        return out, fout, list(torch.split(sig, ranks))

    def quantize_core(self, core, keep, bits: int):
        """Leading block `keep` of the core, uniformly quantised: returns (codes int32, dequantised, step)."""
        import torch
        core = _f32_device(core, "core")
        ranks = list(core.shape)
        keep = [int(k) for k in keep]
        codes = torch.empty(keep, dtype=torch.int32, device=core.device)
        deq = torch.empty(keep, dtype=torch.float32, device=core.device)
        step = C.c_float(0.0)
        _check(_lib.lib().tucker_quantize_core(self._h, C.c_void_p(core.data_ptr()), len(ranks), _lib.i64(ranks),
                                               _lib.i64(keep), int(bits), C.c_void_p(codes.data_ptr()),
                                               C.c_void_p(deq.data_ptr()), C.byref(step)), self._h)
        return codes, deq, float(step.value)

    # ---------------------------------------------------------------- building blocks
    def ttm(self, x, mode: int, U):
        """x x_mode U^T (U is x.shape[mode] x r)."""
        import torch
        x = _f32_device(x, "x")
        U = _f32_device(U, "U")
        dims = list(x.shape)
        out_dims = list(dims)
        out_dims[mode] = int(U.shape[1])
        out = torch.empty(out_dims, dtype=torch.float32, device=x.device)
        _check(_lib.lib().tucker_ttm(self._h, C.c_void_p(x.data_ptr()), len(dims), _lib.i64(dims), int(mode),
                                     C.c_void_p(U.data_ptr()), int(U.shape[1]), C.c_void_p(out.data_ptr())),
               self._h)
        return out

    def gram(self, x, mode: int):
        import torch
        x = _f32_device(x, "x")
        dims = list(x.shape)
        out = torch.empty((dims[mode], dims[mode]), dtype=torch.float32, device=x.device)
        _check(_lib.lib().tucker_gram(self._h, C.c_void_p(x.data_ptr()), len(dims), _lib.i64(dims), int(mode),
                                      C.c_void_p(out.data_ptr())), self._h)
        return out

    def quantize(self, x, precision: str):
        """Encode/decode round trip of a (rows, L) matrix; returns (values, scales or None)."""
        import torch
        x = _f32_device(x, "x")
        if x.dim() != 2:
            raise ValueError("x must be 2-D (rows, L)")
        out = torch.empty_like(x)
        scales = torch.empty(x.shape[1], dtype=torch.float32, device=x.device)
        _check(_lib.lib().tucker_quantize(self._h, C.c_void_p(x.data_ptr()), int(x.shape[0]), int(x.shape[1]),
                                          _PRECISIONS[precision], C.c_void_p(out.data_ptr()),
                                          C.c_void_p(scales.data_ptr())), self._h)
        return out, (scales if precision == "fp8" else None)

    def ttm_lowp(self, x, mode: int, U, precision: str):
        """Q(x) x_mode Q(U)^T on the reduced-precision matrix cores (float result)."""
        import torch
        x = _f32_device(x, "x")
        U = _f32_device(U, "U")
        dims = list(x.shape)
        out_dims = list(dims)
        out_dims[mode] = int(U.shape[1])
        out = torch.empty(out_dims, dtype=torch.float32, device=x.device)
        _check(_lib.lib().tucker_ttm_lowp(self._h, C.c_void_p(x.data_ptr()), len(dims), _lib.i64(dims), int(mode),
                                          C.c_void_p(U.data_ptr()), int(U.shape[1]), _PRECISIONS[precision],
                                          C.c_void_p(out.data_ptr())), self._h)
        return out

    def gram_lowp(self, x, mode: int, precision: str):
        """Mode Gram of Q(x) on the BF16 / FP16 matrix cores (float result)."""
        import torch
        x = _f32_device(x, "x")
        dims = list(x.shape)
        out = torch.empty((dims[mode], dims[mode]), dtype=torch.float32, device=x.device)
        _check(_lib.lib().tucker_gram_lowp(self._h, C.c_void_p(x.data_ptr()), len(dims), _lib.i64(dims), int(mode),
                                           _PRECISIONS[precision], C.c_void_p(out.data_ptr())), self._h)
        return out

    def orthonormalize(self, Z):
        import torch
        Z = _f32_device(Z, "Z")
        out = torch.empty_like(Z)
        _check(_lib.lib().tucker_orthonormalize(self._h, C.c_void_p(Z.data_ptr()), int(Z.shape[0]),
                                                int(Z.shape[1]), C.c_void_p(out.data_ptr())), self._h)
        return out

    def gram_tn64(self, Z):
        """Z^T Z accumulated in FP64 (float64 result)."""
        import torch
        Z = _f32_device(Z, "Z")
        W = torch.empty((Z.shape[1], Z.shape[1]), dtype=torch.float64, device=Z.device)
        _check(_lib.lib().tucker_gram_tn64(self._h, C.c_void_p(Z.data_ptr()), int(Z.shape[0]), int(Z.shape[1]),
                                           C.c_void_p(W.data_ptr())), self._h)
        return W

    def chol_inv(self, W):
        """T = L^-1 D^-1 for D^-1 W D^-1 = L L^T (float64 in and out)."""
        import torch
        if W.dtype != torch.float64 or W.device.type != "cuda":
            raise TypeError("W must be a float64 CUDA tensor")
        W = W.contiguous()
        T = torch.empty_like(W)
        _check(_lib.lib().tucker_chol_inv(self._h, C.c_void_p(W.data_ptr()), int(W.shape[0]),
                                          C.c_void_p(T.data_ptr())), self._h)
        return T

    def sym_eig(self, S, r: int):
        import torch
        S = _f32_device(S, "S")
        n = int(S.shape[0])
        U = torch.empty((n, r), dtype=torch.float32, device=S.device)
        lam = torch.empty((n,), dtype=torch.float64, device=S.device)
        _check(_lib.lib().tucker_sym_eig(self._h, C.c_void_p(S.data_ptr()), n, int(r), C.c_void_p(U.data_ptr()),
                                         C.c_void_p(lam.data_ptr())), self._h)
        return U, lam

    def sumsq(self, x) -> float:
        x = _f32_device(x, "x")
        out = C.c_double(0.0)
        _check(_lib.lib().tucker_sumsq(self._h, C.c_void_p(x.data_ptr()), int(x.numel()), C.byref(out)), self._h)
        return float(out.value)

    def set_timing(self, on: bool, stages=None):
        """Stage timing of later calls: every stage (stages None), or only the named ones."""
        mask = 0
        for name in stages or ():
            mask |= 1 << _lib.STAGES.index(name)
        _check(_lib.lib().tucker_set_timing(self._h, 1 if on else 0, mask), self._h)

    def stats(self) -> dict:
        st = _lib.Stats()
        _check(_lib.lib().tucker_get_stats(self._h, C.byref(st)))
        out = {k: getattr(st, k) for k, _ in _lib.Stats._fields_ if k not in ("stage_ms", "stage_calls")}
        out["stages"] = {name: (float(st.stage_ms[i]), int(st.stage_calls[i]))
                         for i, name in enumerate(_lib.STAGES) if st.stage_calls[i]}
        return out


def autotune_table() -> str:
    """The autotuner's choices so far in this process, one line per (operation, shape, device)."""
    need = C.c_size_t(0)
    _lib.lib().tucker_autotune_dump(None, 0, C.byref(need))
    buf = C.create_string_buffer(int(need.value) + 1)
    _lib.lib().tucker_autotune_dump(buf, len(buf), C.byref(need))
    return buf.value.decode()


def autotune_clear() -> None:
    _lib.lib().tucker_autotune_clear()


def autotune_force(op: int, choice: int) -> None:
    """Every later call of autotuner operation `op` (1 FP32 tiles, 2 FP64 Gram splits, 3 reduced-precision
    tiles) takes candidate `choice`; a negative choice lifts the override."""
    _check(_lib.lib().tucker_autotune_force(int(op), int(choice)))


_default = {}


def default_context(device: int = 0) -> Context:
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def decompose(x, ranks, max_iters: int = 10, tol: float = 0.0, init_factors=None) -> Result:
    return default_context(x.device.index or 0).decompose(x, ranks, max_iters, tol, init_factors)


def reconstruct(core, factors):
    return default_context(core.device.index or 0).reconstruct(core, factors)


# ---------------------------------------------------------------------------------------------
# Served execution
# ---------------------------------------------------------------------------------------------

@dataclass
class Served:
    """Result of one served request (host arrays)."""
    status: int
    error: str
    fit: float
    sweeps: int
    tag: int
    slot: int
    footprint_bytes: int
    t_submit: float
    t_admit: float
    t_start: float
    t_finish: float
    core: "object" = None           # numpy float32 (R_1, ..., R_N)
    factors: List = field(default_factory=list)   # numpy float32 (s_n, R_n)

    @property
    def latency(self) -> float:
        return self.t_finish - self.t_submit


def _host_ptr(a):
    """Address of a C-contiguous float32 host array (numpy array or CPU torch tensor)."""
    try:
        import torch
        if isinstance(a, torch.Tensor):
            if a.is_cuda or a.dtype != torch.float32 or not a.is_contiguous():
                raise TuckerError(_lib.ERR_INVALID_ARG, "host tensor must be a contiguous float32 CPU tensor")
            return a.data_ptr(), tuple(a.shape)
    except ImportError:
        pass
    import numpy as np
    if not (isinstance(a, np.ndarray) and a.dtype == np.float32 and a.flags["C_CONTIGUOUS"]):
        raise TuckerError(_lib.ERR_INVALID_ARG, "host tensor must be a C-contiguous float32 numpy array")
    return a.ctypes.data, tuple(a.shape)


class Server:
    """Request loop of the library (tucker_server_*): admission by HBM budget, `slots` requests
    in flight on their own streams.  With group_requests > 1, consecutive requests of one shape class
    (up to group_requests of them) are admitted together and share grouped persistent launches of
    their reduced-precision products.
    submit() copies nothing and returns at once; the host tensor must stay alive until wait()
    returns its result."""

    def __init__(self, device: int = 0, slots: int = 4, hbm_budget_bytes: int = 0, inner_iters: int = 1,
                 init_iters: int = 20, seed: int = 0x5EED, use_graphs: bool = True, autotune: bool = True,
                 group_requests: int = 0):
        o = _lib.ServerOptions()
        _lib.lib().tucker_default_server_options(C.byref(o))
        o.device, o.slots, o.hbm_budget_bytes = int(device), int(slots), int(hbm_budget_bytes)
        o.inner_iters, o.init_iters, o.seed = int(inner_iters), int(init_iters), int(seed)
        o.use_graphs = 1 if use_graphs else 0
        o.autotune = 1 if autotune else 0
        o.group_requests = int(group_requests)
        h = C.c_void_p()
        _check(_lib.lib().tucker_server_create(C.byref(o), C.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, x, ranks: Sequence[int], max_iters: int = 10, tol: float = 0.0, precision: str = "fp32",
               refine_sweeps: int = 1, tag: int = 0) -> int:
        import numpy as np
        ptr, dims = _host_ptr(x)
        n = len(dims)
        ranks = [int(r) for r in ranks]
        if len(ranks) != n or not 2 <= n <= _lib.MAX_ORDER:
            raise TuckerError(_lib.ERR_INVALID_ARG, "ranks must match the tensor order (2..8)")
        core = np.empty(ranks, dtype=np.float32)
        factors = [np.empty((dims[i], ranks[i]), dtype=np.float32) for i in range(n)]
        q = _lib.Request()
        q.host_tensor = ptr
        q.ndim = n
        for i in range(n):
            q.dims[i] = int(dims[i])
            q.ranks[i] = ranks[i]
            q.host_factors[i] = factors[i].ctypes.data
        q.max_iters, q.tol = int(max_iters), float(tol)
        q.precision, q.refine_sweeps, q.tag = _PRECISIONS[precision], int(refine_sweeps), int(tag)
        q.host_core = core.ctypes.data
        rid = C.c_uint64()
        _check(_lib.lib().tucker_server_submit(self._h, C.byref(q), C.byref(rid)))
        self._keep[rid.value] = (x, core, factors)
        return rid.value

    def wait(self, rid: int, timeout: Optional[float] = None) -> Served:
        r = _lib.ServedResult()
        _check(_lib.lib().tucker_server_wait(self._h, int(rid), -1.0 if timeout is None else float(timeout),
                                             C.byref(r)))
        _, core, factors = self._keep.pop(int(rid))
        return Served(int(r.status), r.error.decode(errors="replace"), float(r.fit), int(r.sweeps), int(r.tag),
                      int(r.slot), int(r.footprint_bytes), float(r.t_submit), float(r.t_admit), float(r.t_start),
                      float(r.t_finish), core, factors)

    def stats(self) -> dict:
        st = _lib.ServerStats()
        _check(_lib.lib().tucker_server_get_stats(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in _lib.ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().tucker_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
