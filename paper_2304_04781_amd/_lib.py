"""ctypes binding of libwavecomp.so: one Python function per C entry point,
same names, argument marshalling only (device tensors -> pointers, host
scalars by reference, status codes -> exceptions). Every computation runs
in the HIP library; if the library is missing, loading fails loudly."""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwavecomp.so")

STORE_NONE, STORE_FULL, STORE_CHECKPOINT, STORE_AE_BF16, STORE_AE_FP8, STORE_AE_TIME = range(6)
TWIN = 32   # levels per time-compression window
LATENT_BF16, LATENT_FP8 = 0, 1
FALLBACK_NONE, FALLBACK_CHECKPOINT = 0, 1
OK, OK_FALLBACK = 0, 1
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESTATE", -5: "EUNSTABLE", -6: "ESHAPE"}


class WvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class WvGrid(C.Structure):
    _fields_ = [("nz", C.c_int32), ("ny", C.c_int32), ("nx", C.c_int32), ("dx", C.c_double),
                ("dt", C.c_double), ("nt", C.c_int32), ("sponge", C.c_int32), ("c_ref", C.c_double),
                ("nsrc", C.c_int32), ("nrec", C.c_int32)]


class AeTrainCfg(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double),
                ("decay_every", C.c_int32), ("decay_factor", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double), ("weighting", C.c_int32)]


class WvNewtonCfg(C.Structure):
    _fields_ = [("max_newton", C.c_int32), ("max_cg", C.c_int32), ("eta_max", C.c_double),
                ("rel_tol", C.c_double), ("c_armijo", C.c_double), ("max_backtrack", C.c_int32),
                ("gauss_newton", C.c_int32), ("precondition", C.c_int32)]


class WvNewtonRec(C.Structure):
    _fields_ = [("cost", C.c_double), ("misfit", C.c_double), ("prior", C.c_double), ("gnorm", C.c_double),
                ("step", C.c_double), ("cg_rel_res", C.c_double), ("cg_iters", C.c_int32),
                ("neg_curv", C.c_int32), ("backtracks", C.c_int32), ("status", C.c_int32)]


EXPORTS = {
    # name: (restype, argtypes)
    "wv_create": (C.c_int, [C.POINTER(WvGrid), C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "wv_destroy": (C.c_int, [C.c_void_p]),
    "wv_set_source_stencil": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "wv_set_storage": (C.c_int, [C.c_void_p, C.c_int, C.c_int32, C.c_void_p, C.c_int64, C.c_double, C.c_int]),
    "wv_storage_bytes": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "wave_forward": (C.c_int, [C.c_void_p] + [C.c_void_p] * 5 + [C.c_int32]),
    "wave_adjoint": (C.c_int, [C.c_void_p] * 4),
    "gradient": (C.c_int, [C.c_void_p] * 4 + [C.c_double, C.c_void_p, C.POINTER(C.c_double)]),
    "hessvec": (C.c_int, [C.c_void_p] * 4 + [C.c_int]),
    "wave_inc_forward": (C.c_int, [C.c_void_p] * 4),
    "ae_create": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "ae_destroy": (None, [C.c_void_p]),
    "ae_param_count": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "ae_get_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ae_set_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ae_set_beta": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ae_get_beta": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ae_fit_beta": (C.c_int, [C.c_void_p, C.POINTER(WvGrid), C.c_void_p, C.c_int64, C.c_double, C.c_void_p]),
    "ae_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "ae_load": (C.c_int, [C.c_char_p, C.POINTER(C.c_void_p)]),
    "ae_normalize": (C.c_int, [C.c_void_p, C.POINTER(WvGrid), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ae_encode": (C.c_int, [C.c_void_p, C.POINTER(WvGrid), C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                            C.c_void_p, C.c_void_p]),
    "ae_encode_noalloc": (C.c_int, [C.c_void_p, C.POINTER(WvGrid), C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p]),
    "ae_decode": (C.c_int, [C.c_void_p, C.POINTER(WvGrid), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                            C.c_uint32, C.c_void_p, C.c_void_p]),
    "ae_train": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(AeTrainCfg), C.c_void_p,
                           C.c_void_p, C.c_void_p]),
    "ae_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_double,
                                C.POINTER(AeTrainCfg), C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    "wv_set_ae_exceptions": (C.c_int, [C.c_void_p, C.c_int32]),
    "wv_revolve_schedule": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_int64, C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64)]),
    "wv_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "wv_set_timing": (C.c_int, [C.c_void_p, C.c_int32]),
    "wv_kernel_time": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "wv_stream_probe": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.c_int32, C.c_void_p,
                                  C.POINTER(C.c_double)]),
    "wv_last_error": (C.c_char_p, []),
    "wv_version": (C.c_char_p, []),
    "wv_accumulation_block": (C.c_int, []),
    "wv_set_delta_storage": (C.c_int, [C.c_void_p, C.c_int32]),
    "wv_set_ae_metadata": (C.c_int, [C.c_void_p, C.c_int32]),
    "wv_decode_delta": (C.c_int, [C.c_void_p, C.c_int32, C.c_uint32, C.c_void_p]),
    "wv_set_prior": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]),
    "wave_forward_e": (C.c_int, [C.c_void_p] * 4 + [C.c_int32, C.c_void_p]),
    "wv_load_e": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "ae_time_fit_beta": (C.c_int, [C.c_void_p, C.POINTER(WvGrid), C.c_void_p, C.c_int64, C.c_double, C.c_void_p]),
    "ae_time_normalize": (C.c_int, [C.c_void_p, C.POINTER(WvGrid), C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                                    C.c_void_p, C.c_void_p, C.c_void_p]),
    "ae_time_encode": (C.c_int, [C.c_void_p, C.POINTER(WvGrid), C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                 C.c_void_p]),
    "ae_time_decode": (C.c_int, [C.c_void_p, C.POINTER(WvGrid), C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                 C.c_void_p]),
    "wv_prior_sample": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                                  C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "ae_normalize_rows": (C.c_int, [C.c_void_p, C.POINTER(WvGrid), C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                    C.c_void_p, C.c_void_p]),
    "wv_prior": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "wv_prior_hessvec": (C.c_int, [C.c_void_p] * 3),
    "wv_newton_cg": (C.c_int, [C.c_void_p] * 4 + [C.c_double, C.POINTER(WvNewtonCfg), C.c_void_p,
                                                   C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
}

_lib: Optional[C.CDLL] = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_2304_04781_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int) -> int:
    if rc < 0:
        raise WvError(rc, load().wv_last_error().decode())
    return rc


def ptr(t: Optional[torch.Tensor], dtype=None) -> Optional[int]:
    """Device pointer of a contiguous GPU tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return t.data_ptr()


def stream_handle(stream: Optional[torch.cuda.Stream] = None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def make_grid(nz, ny, nx, dx, dt, nt, sponge, c_ref, nsrc, nrec) -> WvGrid:
    return WvGrid(int(nz), int(ny), int(nx), float(dx), float(dt), int(nt), int(sponge), float(c_ref),
                  int(nsrc), int(nrec))


# ----- thin wrappers (same names as the C ABI) ----------------------------------------------
def wv_create(grid: WvGrid, src: Sequence, rec: Sequence, stream=None) -> int:
    s = np.ascontiguousarray(np.asarray(src, dtype=np.int32).reshape(-1))
    r = np.ascontiguousarray(np.asarray(rec, dtype=np.int32).reshape(-1))
    out = C.c_void_p()
    _check(load().wv_create(C.byref(grid), s.ctypes.data, r.ctypes.data if r.size else None,
                            stream_handle(stream), C.byref(out)))
    return out.value


def wv_destroy(ctx: int) -> None:
    load().wv_destroy(ctx)


def wv_set_storage(ctx, mode, n_checkpoints=0, ae=None, mem_budget_bytes=0, guard_tol=0.0,
                   fallback_policy=FALLBACK_NONE) -> int:
    return _check(load().wv_set_storage(ctx, mode, n_checkpoints, ae, mem_budget_bytes, guard_tol,
                                        fallback_policy))


def wv_set_source_stencil(ctx, weights: np.ndarray) -> int:
    """weights: (2R+1, 2R+1 | 1, 2R+1) array; R inferred from its first axis."""
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32))
    R = (w.shape[0] - 1) // 2
    return _check(load().wv_set_source_stencil(ctx, R, w.ctypes.data))


def wv_storage_bytes(ctx) -> int:
    v = C.c_int64()
    _check(load().wv_storage_bytes(ctx, C.byref(v)))
    return v.value


def wave_forward(ctx, c, wavelet, traces=None, final_state=None, capture=None, capture_every=0) -> int:
    f32 = torch.float32
    return _check(load().wave_forward(ctx, ptr(c, f32), ptr(wavelet, f32), ptr(traces, f32),
                                      ptr(final_state, f32), ptr(capture, f32), int(capture_every)))


def wave_adjoint(ctx, c, residual, g) -> int:
    f32 = torch.float32
    return _check(load().wave_adjoint(ctx, ptr(c, f32), ptr(residual, f32), ptr(g, f32)))


def gradient(ctx, c, wavelet, d_obs, sigma, g):
    """Returns (status, J)."""
    f32 = torch.float32
    J = C.c_double()
    rc = _check(load().gradient(ctx, ptr(c, f32), ptr(wavelet, f32), ptr(d_obs, f32), float(sigma),
                                ptr(g, f32), C.byref(J)))
    return rc, J.value


def hessvec(ctx, c, dc, Hdc, gauss_newton=1) -> int:
    f32 = torch.float32
    return _check(load().hessvec(ctx, ptr(c, f32), ptr(dc, f32), ptr(Hdc, f32), int(gauss_newton)))


def wave_inc_forward(ctx, c, dc, dtraces) -> int:
    f32 = torch.float32
    return _check(load().wave_inc_forward(ctx, ptr(c, f32), ptr(dc, f32), ptr(dtraces, f32)))


def wv_stats(ctx):
    fs, ge, dg = C.c_int64(), C.c_double(), C.c_int()
    _check(load().wv_stats(ctx, C.byref(fs), C.byref(ge), C.byref(dg)))
    return fs.value, ge.value, bool(dg.value)


# kernel classes of wv_kernel_time
TIMED_KERNELS = ("forward_stencil", "adjoint_stencil", "incremental_stencil", "encode", "decode_e",
                 "exceptions_select", "exceptions_restore", "exceptions_gather")


def wv_set_timing(ctx, every: int) -> None:
    _check(load().wv_set_timing(ctx, int(every)))


def wv_kernel_time(ctx, cls: int):
    """(mean duration in microseconds, number of timed launches) of one kernel class."""
    m, n = C.c_double(), C.c_int64()
    _check(load().wv_kernel_time(ctx, int(cls), C.byref(m), C.byref(n)))
    return m.value, n.value


def wv_revolve_schedule(nsteps: int, nslots: int):
    """Returns (actions int32 [n, 3], forward_steps)."""
    L = load()
    n, fs = C.c_int64(), C.c_int64()
    _check(L.wv_revolve_schedule(nsteps, nslots, None, 0, C.byref(n), C.byref(fs)))
    out = np.zeros((n.value, 3), dtype=np.int32)
    _check(L.wv_revolve_schedule(nsteps, nslots, out.ctypes.data, n.value, C.byref(n), C.byref(fs)))
    return out, fs.value


def ae_create(in_dim, hidden, latent, init_params: np.ndarray, beta=None) -> int:
    p = np.ascontiguousarray(init_params, dtype=np.float32)
    b = None if beta is None else np.ascontiguousarray(beta, dtype=np.float64)
    out = C.c_void_p()
    _check(load().ae_create(int(in_dim), int(hidden), int(latent), p.ctypes.data,
                            None if b is None else b.ctypes.data, C.byref(out)))
    return out.value


def ae_destroy(net) -> None:
    load().ae_destroy(net)


def ae_param_count(net) -> int:
    v = C.c_int64()
    _check(load().ae_param_count(net, C.byref(v)))
    return v.value


def ae_get_params(net) -> np.ndarray:
    out = np.zeros(ae_param_count(net), dtype=np.float32)
    _check(load().ae_get_params(net, out.ctypes.data))
    return out


def ae_set_params(net, params: np.ndarray) -> None:
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(load().ae_set_params(net, p.ctypes.data))


def ae_set_beta(net, beta) -> None:
    b = np.ascontiguousarray(beta, dtype=np.float64)
    _check(load().ae_set_beta(net, b.ctypes.data))


def ae_get_beta(net) -> np.ndarray:
    b = np.zeros(4, dtype=np.float64)
    _check(load().ae_get_beta(net, b.ctypes.data))
    return b


def ae_fit_beta(net, grid: WvGrid, states, nstates: int, rel: float = 1e-7, stream=None) -> None:
    _check(load().ae_fit_beta(net, C.byref(grid), ptr(states, torch.float32), int(nstates), float(rel),
                              stream_handle(stream)))


def ae_save(net, path: str) -> None:
    _check(load().ae_save(net, path.encode()))


def ae_load(path: str) -> int:
    out = C.c_void_p()
    _check(load().ae_load(path.encode(), C.byref(out)))
    return out.value


def ae_normalize(net, grid: WvGrid, state, y, meta, stream=None) -> None:
    _check(load().ae_normalize(net, C.byref(grid), ptr(state, torch.float32), ptr(y, torch.int16),
                               ptr(meta, torch.float32), stream_handle(stream)))


def ae_encode(net, grid: WvGrid, state, latent_fmt, latent, meta, qscale=None, stream=None) -> None:
    _check(load().ae_encode(net, C.byref(grid), ptr(state, torch.float32), int(latent_fmt), ptr(latent),
                            ptr(meta, torch.float32), ptr(qscale, torch.float32), stream_handle(stream)))


def ae_encode_noalloc(net, grid: WvGrid, state, latent_fmt, latent, meta, qscale=None, stream=None) -> None:
    _check(load().ae_encode_noalloc(net, C.byref(grid), ptr(state, torch.float32), int(latent_fmt), ptr(latent),
                                    ptr(meta, torch.float32), ptr(qscale, torch.float32), stream_handle(stream)))


def ae_decode(net, grid: WvGrid, latent, meta, qscale, latent_fmt, field_mask, state, stream=None) -> None:
    _check(load().ae_decode(net, C.byref(grid), ptr(latent), ptr(meta, torch.float32),
                            ptr(qscale, torch.float32), int(latent_fmt), int(field_mask),
                            ptr(state, torch.float32), stream_handle(stream)))


def train_cfg(epochs=20, batch=4096, lr=1e-3, decay_every=5, decay_factor=0.5, beta1=0.9, beta2=0.999,
              eps=1e-8, weighting=0) -> AeTrainCfg:
    return AeTrainCfg(int(epochs), int(batch), float(lr), int(decay_every), float(decay_factor),
                      float(beta1), float(beta2), float(eps), int(weighting))


def ae_train(net, y, nsamples: int, cfg: AeTrainCfg, perm=None, meta=None, stream=None) -> np.ndarray:
    loss = np.zeros(max(cfg.epochs, 1), dtype=np.float32)
    _check(load().ae_train(net, ptr(y, torch.int16), ptr(meta, torch.float32), int(nsamples), C.byref(cfg),
                           ptr(perm, torch.int32), loss.ctypes.data, stream_handle(stream)))
    return loss


def ae_train_step(net, y, idx, batch: int, lr: float, cfg: AeTrainCfg, want_grads: bool = False,
                  meta=None, stream=None):
    grads = np.zeros(ae_param_count(net), dtype=np.float32) if want_grads else None
    loss = C.c_double()
    _check(load().ae_train_step(net, ptr(y, torch.int16), ptr(meta, torch.float32), ptr(idx, torch.int32),
                                int(batch), float(lr), C.byref(cfg), None if grads is None else grads.ctypes.data,
                                C.byref(loss), stream_handle(stream)))
    return loss.value, grads


def wv_set_ae_exceptions(ctx, k_per_step: int) -> int:
    return _check(load().wv_set_ae_exceptions(ctx, int(k_per_step)))


def wv_stream_probe(inp, out, n_in: int, n_out: int, n: int, reps: int = 10, stream=None) -> float:
    """Mean microseconds per launch of the streaming probe (n_in arrays read, n_out written, n floats each)."""
    us = C.c_double()
    _check(load().wv_stream_probe(ptr(inp, torch.float32), ptr(out, torch.float32), int(n_in), int(n_out), int(n),
                                  int(reps), stream_handle(stream), C.byref(us)))
    return us.value


def wv_last_error() -> str:
    return load().wv_last_error().decode()


def wv_version() -> str:
    return load().wv_version().decode()


def wv_accumulation_block() -> int:
    return int(load().wv_accumulation_block())


def wv_set_ae_metadata(ctx, bits: int) -> int:
    return _check(load().wv_set_ae_metadata(ctx, int(bits)))


def wv_set_delta_storage(ctx, enable: bool) -> int:
    return _check(load().wv_set_delta_storage(ctx, 1 if enable else 0))


def wv_decode_delta(ctx, n: int, field_mask: int, state) -> int:
    return _check(load().wv_decode_delta(ctx, int(n), int(field_mask), ptr(state)))


def wv_set_prior(ctx, alpha: float, theta: Sequence[float] = (0.0, 0.0, 0.0), c0=None) -> int:
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(3))
    return _check(load().wv_set_prior(ctx, float(alpha), th.ctypes.data, ptr(c0, torch.float32)))


def wv_prior(ctx, c, g=None, want_cost: bool = True):
    """Returns R(c) (None when want_cost is False); g += grad R if g is given."""
    R = C.c_double()
    _check(load().wv_prior(ctx, ptr(c, torch.float32), ptr(g, torch.float32), C.byref(R) if want_cost else None))
    return R.value if want_cost else None


def wv_prior_hessvec(ctx, dc, Hdc) -> int:
    return _check(load().wv_prior_hessvec(ctx, ptr(dc, torch.float32), ptr(Hdc, torch.float32)))


NEWTON_FIELDS = [f for f, _ in WvNewtonRec._fields_]


def wv_newton_cg(ctx, c, wavelet, d_obs, sigma, max_newton=5, max_cg=10, eta_max=0.5, rel_tol=1e-6,
                 c_armijo=1e-4, max_backtrack=10, gauss_newton=1, precondition=0):
    """Runs Newton-CG in place on c; returns (records as dicts, iterations, reason)."""
    cfg = WvNewtonCfg(int(max_newton), int(max_cg), float(eta_max), float(rel_tol), float(c_armijo),
                      int(max_backtrack), int(gauss_newton), int(precondition))
    recs = (WvNewtonRec * (int(max_newton) + 1))()
    it, reason = C.c_int32(), C.c_int32()
    f32 = torch.float32
    _check(load().wv_newton_cg(ctx, ptr(c, f32), ptr(wavelet, f32), ptr(d_obs, f32), float(sigma), C.byref(cfg),
                               recs, C.byref(it), C.byref(reason)))
    log = [{f: getattr(recs[i], f) for f in NEWTON_FIELDS} for i in range(it.value + 1)]
    return log, it.value, reason.value


def wv_prior_sample(ctx, w, out, rtol=1e-6, maxit=1000):
    """out = c0 + A^-1 w / sqrt(vol); returns (CG iterations, final relative residual)."""
    it, rr = C.c_int32(), C.c_double()
    f32 = torch.float32
    _check(load().wv_prior_sample(ctx, ptr(w, f32), ptr(out, f32), float(rtol), int(maxit), C.byref(it),
                                  C.byref(rr)))
    return it.value, rr.value


def ae_normalize_rows(net, grid, state, rows, y, meta, stream=None) -> int:
    n = 0 if rows is None else int(rows.numel())
    return _check(load().ae_normalize_rows(net, C.byref(grid), ptr(state, torch.float32), ptr(rows, torch.int32), n,
                                           ptr(y), ptr(meta, torch.float32), stream_handle(stream)))


def wave_forward_e(ctx, c, wavelet, steps, e_out) -> int:
    st = np.ascontiguousarray(np.asarray(steps, dtype=np.int32).reshape(-1))
    return _check(load().wave_forward_e(ctx, ptr(c, torch.float32), ptr(wavelet, torch.float32),
                                        st.ctypes.data if st.size else None, int(st.size), ptr(e_out, torch.float32)))


def wv_load_e(ctx, n: int, out) -> int:
    return _check(load().wv_load_e(ctx, int(n), ptr(out, torch.float32)))


def ae_time_fit_beta(net, grid, e, nlevels: int, rel: float, stream=None) -> int:
    return _check(load().ae_time_fit_beta(net, C.byref(grid), ptr(e, torch.float32), int(nlevels), float(rel),
                                          stream_handle(stream)))


def ae_time_normalize(net, grid, e_win, nvalid: int, y, meta, rows=None, stream=None) -> int:
    n = 0 if rows is None else int(rows.numel())
    return _check(load().ae_time_normalize(net, C.byref(grid), ptr(e_win, torch.float32), int(nvalid),
                                           ptr(rows, torch.int32), n, ptr(y), ptr(meta, torch.float32),
                                           stream_handle(stream)))


def ae_time_encode(net, grid, e_win, nvalid: int, latent, meta, stream=None) -> int:
    return _check(load().ae_time_encode(net, C.byref(grid), ptr(e_win, torch.float32), int(nvalid), ptr(latent),
                                        ptr(meta, torch.float32), stream_handle(stream)))


def ae_time_decode(net, grid, latent, meta, nvalid: int, e_win, stream=None) -> int:
    return _check(load().ae_time_decode(net, C.byref(grid), ptr(latent), ptr(meta, torch.float32), int(nvalid),
                                        ptr(e_win, torch.float32), stream_handle(stream)))
