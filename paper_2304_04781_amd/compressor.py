"""The learned compressor: an autoencoder handle and the training pipelines
of Sec. 3.3.1. train_from_forward feeds it snapshots of the solver's own
forward solve (Algorithm 1 with the current model in place of prior draws);
prior_draw_samples + train_samples follow Algorithm 1 itself: forward solves
at draws from the prior, each state's patch vectors kept or discarded at
random.

Every step runs in libwavecomp.so: the forward solve captures raw states,
ae_fit_beta sets the per-field floors, ae_normalize builds the bfloat16
training vectors and ae_train runs the MFMA forward/backward passes and
Adam. Initial weights and shuffle orders are inputs (drawn by the caller).
"""
from __future__ import annotations

import time
from typing import Optional

import numpy as np
import torch

from . import _lib as L

PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")


def flatten(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[k], dtype=np.float32).ravel() for k in PARAM_ORDER])


class Autoencoder:
    """Owns an ae_net (weights, Adam state, floors) on the current device."""

    def __init__(self, init_params, in_dim=2048, hidden=512, latent=32, beta=None):
        flat = init_params if isinstance(init_params, np.ndarray) else flatten(init_params)
        self.dims = (in_dim, hidden, latent)
        self.handle = L.ae_create(in_dim, hidden, latent, flat, beta)

    @classmethod
    def load(cls, path: str) -> "Autoencoder":
        obj = cls.__new__(cls)
        obj.handle = L.ae_load(path)
        obj.dims = (2048, 0, 0)
        return obj

    def save(self, path: str) -> None:
        L.ae_save(self.handle, path)

    def params(self) -> np.ndarray:
        return L.ae_get_params(self.handle)

    def beta(self) -> np.ndarray:
        return L.ae_get_beta(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            L.ae_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def prior_draw_samples(solver, ae: Autoencoder, draws, wavelet, every: int, rows, beta_rel: float = 1e-7):
    """Training vectors from forward solves at the speed models `draws` (prior
    draws, Sec. 3.3.1 Algorithm 1). Of every `every`-th state of draw i, the
    patches rows[i][q] (int32 arrays, the random keep choice) are normalised into
    y [n][2048] bfloat16 bits and meta [n][4][2]. The floors beta_f come from the
    first draw's captured states. Returns (y, meta, capture seconds)."""
    nz, ny, nx = solver.shape
    total = sum(len(r) for rr in rows for r in rr)
    dev = solver.device
    y = torch.empty((total, 2048), dtype=torch.int16, device=dev)
    meta = torch.empty((total, 4, 2), dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    off = 0
    for i, c in enumerate(draws):
        _, _, cap = solver.forward(c, wavelet, capture_every=every)
        ncap = cap.shape[0] * solver.S
        cap = cap.reshape((ncap, 4) + solver.shape)
        if len(rows[i]) != ncap:
            raise ValueError(f"draw {i}: {len(rows[i])} row lists for {ncap} captured states")
        if i == 0:
            L.ae_fit_beta(ae.handle, solver.grid, cap, ncap, beta_rel)
        for q in range(ncap):
            n = len(rows[i][q])
            r = torch.as_tensor(rows[i][q], dtype=torch.int32, device=dev)
            L.ae_normalize_rows(ae.handle, solver.grid, cap[q], r, y[off:off + n], meta[off:off + n])
            off += n
        torch.cuda.synchronize()
        del cap
    torch.cuda.empty_cache()
    return y, meta, time.perf_counter() - t0


def time_window_samples(solver, ae: Autoencoder, c, wavelet, windows, rows=None, beta_rel: float = 1e-7):
    """Training vectors of the time-compression scheme (Sec. 3.2): e over the
    listed windows (window w holds levels 32 w + 1 .. 32 w + 32, the last one
    possibly short) of one forward solve at c, normalised per vector; rows[i]
    (int32 arrays, optional) keeps only those vectors of window i. The floor
    beta_e comes from the captured levels. Returns (y, meta, capture seconds)."""
    T1 = solver.nt - 1
    nv = [min(L.TWIN, T1 - L.TWIN * w) for w in windows]
    if min(nv) < 1:
        raise ValueError("window beyond the stored levels")
    steps = [L.TWIN * w + 1 + t for w, n in zip(windows, nv) for t in range(n)]
    t0 = time.perf_counter()
    e = solver.forward_e(c, wavelet, steps)
    torch.cuda.synchronize()
    t_cap = time.perf_counter() - t0
    L.ae_time_fit_beta(ae.handle, solver.grid, e, len(steps), beta_rel)
    nz, ny, nx = solver.shape
    M = solver.S * (nz // 4) * (ny // 4) * (nx // 4)
    counts = [M if rows is None else len(rows[i]) for i in range(len(windows))]
    y = torch.empty((sum(counts), 2048), dtype=torch.int16, device=solver.device)
    meta = torch.empty((sum(counts), 2), dtype=torch.float32, device=solver.device)
    off = lvl = 0
    for i, n in enumerate(nv):
        r = None if rows is None else torch.as_tensor(rows[i], dtype=torch.int32, device=solver.device)
        L.ae_time_normalize(ae.handle, solver.grid, e[lvl:lvl + n], n, y[off:off + counts[i]],
                            meta[off:off + counts[i]], rows=r)
        off += counts[i]
        lvl += n
    torch.cuda.synchronize()
    del e
    torch.cuda.empty_cache()
    return y, meta, t_cap


def _perm_tensor(perms, device):
    """Visiting orders [epochs, nsamples] as a contiguous int32 device tensor (a numpy array
    or a torch tensor; None: in order)."""
    if perms is None:
        return None
    if torch.is_tensor(perms):
        return perms.to(device=device, dtype=torch.int32).contiguous()
    return torch.as_tensor(np.ascontiguousarray(perms, dtype=np.int32), device=device)


def train_samples(ae: Autoencoder, y, meta, epochs: int, batch: int, perms: Optional[np.ndarray] = None,
                  weighting: int = 0, lr: float = 1e-3, decay_every: int = 5, decay_factor: float = 0.5):
    """Adam on the training vectors y (with meta for the weighted loss).
    Returns a dict with sizes, first/last epoch losses and timings."""
    nsamp = int(y.shape[0])
    perm_t = _perm_tensor(perms, y.device)
    cfg = L.train_cfg(epochs=epochs, batch=batch, lr=lr, decay_every=decay_every, decay_factor=decay_factor,
                      weighting=weighting)
    t1 = time.perf_counter()
    losses = L.ae_train(ae.handle, y, nsamp, cfg, perm_t, meta=meta)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    steps = epochs * (nsamp // batch)
    flops = steps * batch * 6.0 * 2 * (2048 * 512 + 512 * 32 + 32 * 512 + 512 * 2048) / 2
    return {"samples": nsamp, "epochs": int(epochs), "batch": int(batch), "adam_steps": int(steps),
            "loss_first": float(losses[0]) if len(losses) else None,
            "loss_last": float(losses[-1]) if len(losses) else None,
            "train_s": round(t_train, 3), "train_TFLOP/s": round(flops / max(t_train, 1e-9) / 1e12, 1)}


def train_from_forward(solver, ae: Autoencoder, c, wavelet, every: int, epochs: int, batch: int,
                       perms: Optional[np.ndarray] = None, weighting: int = 0, lr: float = 1e-3,
                       decay_every: int = 5, decay_factor: float = 0.5, beta_rel: float = 1e-7):
    """Capture every `every`-th state of a forward solve at c, set the floors
    beta_f = beta_rel * max|x_f|, normalise the snapshots and train.
    perms: [epochs, nsamples] int32 visiting orders, numpy or a torch tensor (None: in order).
    Returns a dict with sizes, per-epoch losses and timings."""
    S = solver.S
    t0 = time.perf_counter()
    _, _, cap = solver.forward(c, wavelet, capture_every=every)      # [ncap, S, 4, nz, ny, nx]
    ncap = cap.shape[0] * S
    cap = cap.reshape((ncap, 4) + solver.shape)
    torch.cuda.synchronize()
    t_cap = time.perf_counter() - t0
    L.ae_fit_beta(ae.handle, solver.grid, cap, ncap, beta_rel)
    nz, ny, nx = solver.shape
    P = (nz // 8) * (ny // 8) * (nx // 8)
    nsamp = ncap * P
    y = torch.empty((nsamp, 2048), dtype=torch.int16, device=cap.device)
    meta = torch.empty((nsamp, 4, 2), dtype=torch.float32, device=cap.device)
    for q in range(ncap):
        L.ae_normalize(ae.handle, solver.grid, cap[q], y[q * P:(q + 1) * P], meta[q * P:(q + 1) * P])
    torch.cuda.synchronize()
    del cap
    torch.cuda.empty_cache()
    perm_t = _perm_tensor(perms, y.device)
    cfg = L.train_cfg(epochs=epochs, batch=batch, lr=lr, decay_every=decay_every, decay_factor=decay_factor,
                      weighting=weighting)
    t1 = time.perf_counter()
    losses = L.ae_train(ae.handle, y, nsamp, cfg, perm_t, meta=meta)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    steps = epochs * (nsamp // batch)
    flops = steps * batch * 6.0 * 2 * (2048 * 512 + 512 * 32 + 32 * 512 + 512 * 2048) / 2
    return {"snapshots": int(ncap), "samples": int(nsamp), "epochs": int(epochs), "batch": int(batch),
            "adam_steps": int(steps), "loss_first": float(losses[0]) if len(losses) else None,
            "loss_last": float(losses[-1]) if len(losses) else None, "capture_s": round(t_cap, 3),
            "train_s": round(t_train, 3), "train_TFLOP/s": round(flops / max(t_train, 1e-9) / 1e12, 1)}
