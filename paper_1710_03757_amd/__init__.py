"""Python binding of the MI355X Monte Carlo TRG library (libmctrg.so).

Argument marshalling only: every step of the method runs in the HIP
kernels behind the C ABI declared in include/mctrg.h.  PyTorch supplies
device buffers (``tensor.data_ptr()``) and the current HIP stream.  There
is no CPU fallback: importing this package without the built library, or
calling it without a GPU, raises.

Functions keep the C names without the ``mctrg_`` prefix:
  init_tensor, run_samples, estimate_lnZ, capacity_dim, default_config,
  svd_batched, sample_batched, contract_batched.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmctrg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1710_03757_amd/build.py` "
                      "(the HIP library is the only implementation; there is no fallback)")
# torch ships its own HIP runtime under the same soname as the one the library
# links (libamdhip64.so.7).  Loading torch first makes the dynamic loader bind
# the library to that runtime, so both share one device context; loaded the
# other way round, the first HIP call of the library fails.
import torch  # noqa: E402,F401
_lib = ctypes.CDLL(LIB_PATH)

# ---- constants (include/mctrg.h) ------------------------------------------------
OK, EINVAL, ENOMEM, EDEVICE, ENUMERIC, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
ISING_SITE, ISING_PLAQUETTE, USER = 0, 1, 2
SHARED, INDEPENDENT, TOPK = 0, 1, 2
F64, F32, BF16, FP8_E4M3 = 0, 1, 2, 3
RECORD, PROFILE, ONE_STREAM = 1, 4, 8

MODES = {"shared": SHARED, "independent": INDEPENDENT, "topk": TOPK}
DEC_SVD, DEC_QR3, DEC_QR5 = 0, 1, 2
DECOMPOSITIONS = {"svd": DEC_SVD, "qr3": DEC_QR3, "qr5": DEC_QR5}
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16, "fp8": FP8_E4M3}
MODELS = {"site": ISING_SITE, "vertex": ISING_SITE, "plaquette": ISING_PLAQUETTE, "user": USER}

EXPORTED = ("mctrg_init_tensor", "mctrg_tensor_set_info", "mctrg_default_config", "mctrg_capacity_dim",
            "mctrg_run_samples", "mctrg_estimate_lnZ", "mctrg_destroy", "mctrg_status_string",
            "mctrg_svd_batched", "mctrg_sample_batched", "mctrg_contract_batched", "mctrg_chain_create",
            "mctrg_chain_step", "mctrg_chain_finish", "mctrg_chain_get_profile", "mctrg_chain_destroy",
            "mctrg_chain_tensor", "mctrg_sample_batched_noalloc")


class RunConfig(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("sample_offset", ctypes.c_int64), ("n_steps", ctypes.c_int32),
                ("k", ctypes.c_int32), ("mode", ctypes.c_int32), ("contract_dtype", ctypes.c_int32),
                ("tau_null", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("record_buf", ctypes.c_void_p), ("out_tensor", ctypes.c_void_p),
                ("max_workspace_bytes", ctypes.c_size_t), ("n_det", ctypes.c_int32),
                ("decomposition", ctypes.c_int32)]


class Estimate(ctypes.Structure):
    _fields_ = [("ln_meanZ_per_site", ctypes.c_double), ("rel_stderr_Z", ctypes.c_double),
                ("mean_lnZ_per_site", ctypes.c_double), ("stderr_mean_lnZ", ctypes.c_double),
                ("n_used", ctypes.c_int64), ("n_negative", ctypes.c_int64), ("n_failed", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ChainProfile(ctypes.Structure):
    _fields_ = [("jacobi_ms", ctypes.c_double), ("jacobi_launches", ctypes.c_int64), ("gemm_ms", ctypes.c_double),
                ("gemm_launches", ctypes.c_int64), ("steps_done", ctypes.c_int32), ("last_sweeps", ctypes.c_int32),
                ("last_pairs", ctypes.c_int32 * 64), ("last_active", ctypes.c_int32 * 64),
                ("jacobi_busy_ms", ctypes.c_double), ("gemm_busy_ms", ctypes.c_double), ("parts", ctypes.c_int32),
                ("step_sweeps", ctypes.c_int32 * 64), ("qr128_ms", ctypes.c_double),
                ("qr128_launches", ctypes.c_int64), ("qr128_busy_ms", ctypes.c_double),
                ("qr128_flops", ctypes.c_double), ("jacobi_rotated_pairs", ctypes.c_int64),
                ("jacobi_flops", ctypes.c_double)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        n = max(0, min(64, self.last_sweeps))
        d["last_pairs"] = list(self.last_pairs)[:n]
        d["last_active"] = list(self.last_active)[:n]
        d["step_sweeps"] = list(self.step_sweeps)[:max(0, min(64, self.steps_done))]
        return d


_vp, _i32, _i64, _u64, _f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
_lib.mctrg_init_tensor.argtypes = [ctypes.c_int, _i32, _vp, _vp, _i32, _vp, ctypes.POINTER(_vp)]
_lib.mctrg_init_tensor.restype = ctypes.c_int
_lib.mctrg_tensor_set_info.argtypes = [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]
_lib.mctrg_default_config.argtypes = [ctypes.POINTER(RunConfig)]
_lib.mctrg_default_config.restype = None
_lib.mctrg_capacity_dim.argtypes = [_i32, _i32, _i32]
_lib.mctrg_capacity_dim.restype = _i32
_lib.mctrg_run_samples.argtypes = [_vp, ctypes.POINTER(RunConfig), _i64, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.mctrg_run_samples.restype = ctypes.c_int
_lib.mctrg_estimate_lnZ.argtypes = [_i64, _vp, _vp, _f64, ctypes.POINTER(Estimate), _vp]
_lib.mctrg_estimate_lnZ.restype = ctypes.c_int
_lib.mctrg_destroy.argtypes = [_vp]
_lib.mctrg_destroy.restype = None
_lib.mctrg_status_string.argtypes = [ctypes.c_int]
_lib.mctrg_status_string.restype = ctypes.c_char_p
_lib.mctrg_svd_batched.argtypes = [_i64, _i32, _i32, _vp, _f64, _vp, _vp, _vp, _vp]
_lib.mctrg_svd_batched.restype = ctypes.c_int
_lib.mctrg_sample_batched.argtypes = [_i64, _i32, _i32, _i32, _u64, _f64, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                      _vp, _vp]
_lib.mctrg_sample_batched.restype = ctypes.c_int
_lib.mctrg_sample_batched_noalloc.argtypes = _lib.mctrg_sample_batched.argtypes
_lib.mctrg_sample_batched_noalloc.restype = ctypes.c_int
_lib.mctrg_contract_batched.argtypes = [_i64, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.mctrg_contract_batched.restype = ctypes.c_int
_lib.mctrg_chain_create.argtypes = [_vp, ctypes.POINTER(RunConfig), _i64, _vp, _vp, ctypes.POINTER(_vp)]
_lib.mctrg_chain_create.restype = ctypes.c_int
_lib.mctrg_chain_step.argtypes = [_vp, _i32]
_lib.mctrg_chain_step.restype = ctypes.c_int
_lib.mctrg_chain_finish.argtypes = [_vp, _vp, _vp, _vp]
_lib.mctrg_chain_finish.restype = ctypes.c_int
_lib.mctrg_chain_tensor.argtypes = [_vp, _vp]
_lib.mctrg_chain_tensor.restype = ctypes.c_int
_lib.mctrg_chain_get_profile.argtypes = [_vp, ctypes.POINTER(ChainProfile)]
_lib.mctrg_chain_get_profile.restype = ctypes.c_int
_lib.mctrg_chain_destroy.argtypes = [_vp]
_lib.mctrg_chain_destroy.restype = None


class MctrgError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


def status_string(status: int) -> str:
    return _lib.mctrg_status_string(status).decode()


def _check(status: int, where: str, allow=(OK,)):
    if status not in allow:
        raise MctrgError(status, where)
    return status


def library():
    """The loaded ctypes library (for ABI checks)."""
    return _lib


# ---- torch helpers ------------------------------------------------------------------
def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_1710_03757_amd needs a ROCm GPU (cuda:0); none is visible")
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(torch, t, dtype, name):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on the GPU")
    return t


# ---- API ------------------------------------------------------------------------------
class TensorSet:
    """Owner of the library's initial tensors (mctrg_tensor_set)."""

    def __init__(self, handle: int, n_groups: int, d0: int):
        self._h = ctypes.c_void_p(handle)
        self.n_groups = n_groups
        self.d0 = d0

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h and self._h.value:
            _lib.mctrg_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def init_tensor(model="site", betas: Sequence[float] = (), hs: Optional[Sequence[float]] = None,
                user_T=None) -> TensorSet:
    import numpy as np
    _torch()
    m = MODELS[model] if isinstance(model, str) else int(model)
    out = ctypes.c_void_p()
    if m == USER:
        arr = np.ascontiguousarray(user_T, dtype=np.float64)
        if arr.ndim == 4:
            arr = arr[None]
        n_groups, d = arr.shape[0], arr.shape[1]
        st = _lib.mctrg_init_tensor(m, n_groups, None, None, d, arr.ctypes.data_as(ctypes.c_void_p),
                                    ctypes.byref(out))
    else:
        b = np.ascontiguousarray(betas, dtype=np.float64).reshape(-1)
        h = np.zeros_like(b) if hs is None else np.ascontiguousarray(hs, dtype=np.float64).reshape(-1)
        if h.size != b.size:
            raise ValueError("betas and hs must have the same length")
        n_groups = b.size
        st = _lib.mctrg_init_tensor(m, n_groups, b.ctypes.data_as(ctypes.c_void_p),
                                    h.ctypes.data_as(ctypes.c_void_p), 0, None, ctypes.byref(out))
    _check(st, "mctrg_init_tensor")
    ng, d0 = _i32(), _i32()
    _check(_lib.mctrg_tensor_set_info(out, ctypes.byref(ng), ctypes.byref(d0)), "mctrg_tensor_set_info")
    return TensorSet(out.value, ng.value, d0.value)


def default_config() -> RunConfig:
    cfg = RunConfig()
    _lib.mctrg_default_config(ctypes.byref(cfg))
    return cfg


def capacity_dim(d0: int, k: int, n_steps: int) -> int:
    return int(_lib.mctrg_capacity_dim(d0, k, n_steps))


@dataclass
class SampleResult:
    sign: "object"           # torch int8, device
    ln_abs_Z: "object"       # torch float64, device
    ln_c: "object"           # torch float64 (n_samples, n_steps) or None
    status: int
    record: "object" = None
    tensor: "object" = None


def run_samples(ts: TensorSet, n_samples: int, *, n_steps: int, k: int, mode="shared", dtype="f64",
                seed: int = 0, sample_offset: int = 0, tau_null: float = 1e-11, groups=None,
                ks=None, want_ln_c: bool = False, record: bool = False, want_tensor: bool = False,
                out_sign=None, out_ln_abs_Z=None, one_stream: bool = False,
                max_workspace_bytes: int = 0, out_ln_c=None, allow=(), n_det: int = 0,
                decomposition="svd") -> SampleResult:
    """mctrg_run_samples.  ``groups`` / ``ks``: host sequences (one per sample).
    ``one_stream``: run every wave as one part (MCTRG_ONE_STREAM).  ``allow``:
    further status codes returned instead of raised (as ``status``)."""
    import numpy as np
    torch = _torch()
    cfg = default_config()
    cfg.seed = seed
    cfg.sample_offset = sample_offset
    cfg.n_steps = n_steps
    cfg.k = k
    cfg.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    cfg.contract_dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    cfg.tau_null = tau_null
    if one_stream:
        cfg.flags |= ONE_STREAM
    dev = torch.device("cuda", torch.cuda.current_device())
    sign = out_sign if out_sign is not None else torch.empty(n_samples, dtype=torch.int8, device=dev)
    ln = out_ln_abs_Z if out_ln_abs_Z is not None else torch.empty(n_samples, dtype=torch.float64, device=dev)
    _dev(torch, sign, torch.int8, "out_sign")
    _dev(torch, ln, torch.float64, "out_ln_abs_Z")
    lnc = out_ln_c if out_ln_c is not None else \
        (torch.empty((n_samples, n_steps), dtype=torch.float64, device=dev) if want_ln_c else None)
    rec = None
    if record:
        shape = (n_samples, n_steps, 4 + 2 * k) if cfg.mode != INDEPENDENT else \
            (n_samples, record_positions(n_steps), 2 + k)
        rec = torch.full(shape, -7, dtype=torch.int32, device=dev)
        cfg.flags |= RECORD
        cfg.record_buf = rec.data_ptr()
    ten = None
    if want_tensor:
        Dc = capacity_dim(ts.d0, k, n_steps)
        ten = torch.empty((n_samples, Dc, Dc, Dc, Dc), dtype=torch.float64, device=dev)
        cfg.out_tensor = ten.data_ptr()
    cfg.max_workspace_bytes = int(max_workspace_bytes)
    cfg.n_det = int(n_det)
    cfg.decomposition = DECOMPOSITIONS[decomposition] if isinstance(decomposition, str) else int(decomposition)
    g = None if groups is None else np.ascontiguousarray(groups, dtype=np.int32)
    kk = None if ks is None else np.ascontiguousarray(ks, dtype=np.int32)
    for arr, nm in ((g, "groups"), (kk, "ks")):
        if arr is not None and arr.size != n_samples:
            raise ValueError(f"{nm} must have one entry per sample")
    st = _lib.mctrg_run_samples(ts.handle, ctypes.byref(cfg), n_samples,
                                None if g is None else g.ctypes.data_as(ctypes.c_void_p),
                                None if kk is None else kk.ctypes.data_as(ctypes.c_void_p),
                                _ptr(sign), _ptr(ln), _ptr(lnc), _stream(torch))
    _check(st, "mctrg_run_samples", allow=(OK, ENUMERIC) + tuple(allow))
    return SampleResult(sign, ln, lnc, st, rec, ten)


def record_positions(n_steps: int) -> int:
    """Positions over all levels of an independent-mode record: level s of a
    2^n_steps-site torus holds 2^(n_steps - s) tensors."""
    return sum(2 ** (n_steps - s) for s in range(n_steps))


def split_independent_record(rec, n_steps: int):
    """Host view of one sample's independent-mode record (positions x (2 + k)
    int array) as a list over steps of (c, kept, sel) arrays per position."""
    out, base = [], 0
    for s in range(n_steps):
        npos = 2 ** (n_steps - s)
        out.append(rec[base:base + npos])
        base += npos
    return out


def estimate_lnZ(sign, ln_abs_Z, n_sites: float) -> dict:
    torch = _torch()
    _dev(torch, sign, torch.int8, "sign")
    _dev(torch, ln_abs_Z, torch.float64, "ln_abs_Z")
    est = Estimate()
    _check(_lib.mctrg_estimate_lnZ(sign.numel(), _ptr(sign), _ptr(ln_abs_Z), float(n_sites), ctypes.byref(est),
                                   _stream(torch)), "mctrg_estimate_lnZ")
    return est.as_dict()


def svd_batched(M, d1: int, d2: int, want_V: bool = True, tau_null: float = 1e-11):
    """mctrg_svd_batched on a (n_mats, n, n) float64 device tensor: the chain
    step's decomposition, with the approximation budget of the candidate cut
    tau_null.  Returns (sigma, V or None, sweeps)."""
    torch = _torch()
    _dev(torch, M, torch.float64, "M")
    nm, n = M.shape[0], d1 * d2
    if tuple(M.shape[1:]) != (n, n):
        raise ValueError("M must be (n_mats, d1*d2, d1*d2)")
    sig = torch.empty((nm, n), dtype=torch.float64, device=M.device)
    V = torch.empty((nm, n, n), dtype=torch.float64, device=M.device) if want_V else None
    sw = torch.empty(nm, dtype=torch.int32, device=M.device)
    _check(_lib.mctrg_svd_batched(nm, d1, d2, _ptr(M), float(tau_null), _ptr(sig), _ptr(V), _ptr(sw),
                                  _stream(torch)), "mctrg_svd_batched")
    return sig, V, sw


def sample_batched(sigma, rng, split, k: int, mode="shared", seed: int = 0, tau_null: float = 1e-11,
                   no_alloc: bool = False):
    """mctrg_sample_batched (mctrg_sample_batched_noalloc with ``no_alloc``).
    sigma (n_jobs, n) float64, rng (n_jobs, 3) int64 (sample id, position
    id, step), split (n_jobs,) int32 - all on the device.  Returns dict of
    kept, cand, sel, log_r, weight."""
    torch = _torch()
    _dev(torch, sigma, torch.float64, "sigma")
    _dev(torch, rng, torch.int64, "rng")
    _dev(torch, split, torch.int32, "split")
    nj, n = sigma.shape
    d = sigma.device
    kept = torch.empty(nj, dtype=torch.int32, device=d)
    cand = torch.empty(nj, dtype=torch.int32, device=d)
    sel = torch.empty((nj, k), dtype=torch.int32, device=d)
    lr = torch.empty((nj, k), dtype=torch.float64, device=d)
    w = torch.empty((nj, k), dtype=torch.float64, device=d)
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    fn = _lib.mctrg_sample_batched_noalloc if no_alloc else _lib.mctrg_sample_batched
    _check(fn(nj, n, k, m, seed, tau_null, _ptr(sigma), _ptr(rng), _ptr(split), _ptr(kept), _ptr(cand), _ptr(sel),
              _ptr(lr), _ptr(w), _stream(torch)), fn.__name__)
    return {"kept": kept, "cand": cand, "sel": sel, "log_r": lr, "weight": w}


def contract_batched(GA, GB, FA, FB, dtype="f64"):
    """mctrg_contract_batched: GA, GB (n, kk, D, D); FA, FB (n, D, D, kk)
    float64 device tensors -> T' (n, kk, kk, kk, kk) float64."""
    torch = _torch()
    for t, nm in ((GA, "GA"), (GB, "GB"), (FA, "FA"), (FB, "FB")):
        _dev(torch, t, torch.float64, nm)
    nj, kk, D = GA.shape[0], GA.shape[1], GA.shape[2]
    out = torch.empty((nj, kk, kk, kk, kk), dtype=torch.float64, device=GA.device)
    dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    _check(_lib.mctrg_contract_batched(nj, D, kk, dt, _ptr(GA), _ptr(GB), _ptr(FA), _ptr(FB), _ptr(out),
                                       _stream(torch)), "mctrg_contract_batched")
    return out


class Chain:
    """mctrg_chain_*: one wave of samples advanced step by step."""

    def __init__(self, ts: TensorSet, n_samples: int, *, n_steps: int, k: int, mode="shared", dtype="f64",
                 seed: int = 0, sample_offset: int = 0, tau_null: float = 1e-11, groups=None, profile=False,
                 one_stream=False, record=False, n_det: int = 0, decomposition="svd"):
        import numpy as np
        torch = _torch()
        cfg = default_config()
        cfg.seed, cfg.sample_offset, cfg.n_steps, cfg.k = seed, sample_offset, n_steps, k
        cfg.mode = MODES[mode] if isinstance(mode, str) else int(mode)
        cfg.contract_dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        cfg.tau_null = tau_null
        cfg.n_det = int(n_det)
        cfg.decomposition = DECOMPOSITIONS[decomposition] if isinstance(decomposition, str) else int(decomposition)
        if profile:
            cfg.flags |= PROFILE
        if one_stream:
            cfg.flags |= ONE_STREAM
        self.k = k
        self.record = None
        if record:
            dev = torch.device("cuda", torch.cuda.current_device())
            self.record = torch.full((n_samples, n_steps, 4 + 2 * k), -7, dtype=torch.int32, device=dev)
            cfg.flags |= RECORD
            cfg.record_buf = self.record.data_ptr()
        g = None if groups is None else np.ascontiguousarray(groups, dtype=np.int32)
        self._ts = ts
        self.steps_done = 0
        self.n_samples, self.n_steps = n_samples, n_steps
        self._h = ctypes.c_void_p()
        _check(_lib.mctrg_chain_create(ts.handle, ctypes.byref(cfg), n_samples,
                                       None if g is None else g.ctypes.data_as(ctypes.c_void_p),
                                       _stream(torch), ctypes.byref(self._h)), "mctrg_chain_create")

    def step(self, n: int = 1):
        _check(_lib.mctrg_chain_step(self._h, n), "mctrg_chain_step")
        self.steps_done += n

    def tensor(self):
        """mctrg_chain_tensor: the current normalised tensors (n, D, D, D, D)."""
        torch = _torch()
        D = capacity_dim(self._ts.d0, self.k, self.steps_done)
        out = torch.empty((self.n_samples, D, D, D, D), dtype=torch.float64,
                          device=torch.device("cuda", torch.cuda.current_device()))
        _check(_lib.mctrg_chain_tensor(self._h, _ptr(out)), "mctrg_chain_tensor")
        return out

    def finish(self, want_ln_c=False):
        torch = _torch()
        dev = torch.device("cuda", torch.cuda.current_device())
        sign = torch.empty(self.n_samples, dtype=torch.int8, device=dev)
        ln = torch.empty(self.n_samples, dtype=torch.float64, device=dev)
        lnc = torch.zeros((self.n_samples, self.n_steps), dtype=torch.float64, device=dev) if want_ln_c else None
        st = _lib.mctrg_chain_finish(self._h, _ptr(sign), _ptr(ln), _ptr(lnc))
        _check(st, "mctrg_chain_finish", allow=(OK, ENUMERIC))   # ENUMERIC: some samples failed (sign 0)
        return SampleResult(sign, ln, lnc, st)

    def profile(self) -> dict:
        p = ChainProfile()
        _check(_lib.mctrg_chain_get_profile(self._h, ctypes.byref(p)), "mctrg_chain_get_profile")
        return p.as_dict()

    def close(self):
        if self._h and self._h.value:
            _lib.mctrg_chain_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
