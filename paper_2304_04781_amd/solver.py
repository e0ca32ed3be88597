"""A solver context with torch-allocated device buffers around the C ABI.

Only argument marshalling and buffer allocation happen here; every step of
the forward, adjoint, incremental and autoencoder computations runs in
libwavecomp.so on the current HIP stream."""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import _lib as L


class WaveSolver:
    """One wv_ctx: grid, sources, receivers, history storage.

    Shapes: c [nz, ny, nx] float32; wavelet [S, T]; traces / data [S, T, R];
    states [S, 4, nz, ny, nx] with field order (e, v_z, v_y, v_x)."""

    def __init__(self, nz, ny, nx, dx, dt, nt, sponge, c_ref, src, rec, device="cuda", stream=None):
        L.load()
        self.shape = (int(nz), int(ny), int(nx))
        self.dx, self.dt, self.nt = float(dx), float(dt), int(nt)
        self.src = np.asarray(src, dtype=np.int32).reshape(-1, 3)
        self.rec = np.asarray(rec, dtype=np.int32).reshape(-1, 3)
        self.S, self.R = len(self.src), len(self.rec)
        self.device = torch.device(device)
        self.grid = L.make_grid(nz, ny, nx, dx, dt, nt, sponge, c_ref, self.S, self.R)
        self.stream = stream
        self.ctx = L.wv_create(self.grid, self.src, self.rec, stream)
        self.ae = None

    @classmethod
    def for_problem(cls, p, **kw):
        s = cls(p.nz, p.ny, p.nx, p.dx, p.dt, p.nt, p.sponge, p.c_ref, p.src, p.rec, **kw)
        if getattr(p, "src_w", None) is not None:
            s.set_source_stencil(p.src_w)
        return s

    def set_source_stencil(self, weights):
        L.wv_set_source_stencil(self.ctx, weights)

    def close(self):
        if getattr(self, "ctx", None):
            L.wv_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----- storage ---------------------------------------------------------------------------
    def set_storage(self, mode, n_checkpoints=64, ae=None, mem_budget_bytes=0, guard_tol=0.0,
                    fallback_policy=L.FALLBACK_NONE):
        self.ae = ae
        L.wv_set_storage(self.ctx, mode, n_checkpoints, None if ae is None else ae.handle,
                         mem_budget_bytes, guard_tol, fallback_policy)

    def storage_bytes(self) -> int:
        return L.wv_storage_bytes(self.ctx)

    def stats(self):
        return L.wv_stats(self.ctx)

    def set_delta_storage(self, enable: bool = True) -> None:
        """Also compress the incremental forward states (AE modes; e only in the time mode) in hessvec / inc_forward."""
        L.wv_set_delta_storage(self.ctx, enable)

    def decode_delta(self, n: int, field_mask: int = 0xF):
        """Stored incremental state dx_n [S, 4, nz, ny, nx] (fields outside the mask zero)."""
        out = torch.zeros((self.S, 4) + self.shape, dtype=torch.float32, device=self.device)
        L.wv_decode_delta(self.ctx, n, field_mask, out)
        return out

    def set_timing(self, every: int) -> None:
        """Time every `every`-th launch of each kernel class with HIP events (0: off)."""
        L.wv_set_timing(self.ctx, every)

    def kernel_times(self) -> dict:
        """{class name: (mean microseconds, timed launches)} since set_timing."""
        return {name: L.wv_kernel_time(self.ctx, i) for i, name in enumerate(L.TIMED_KERNELS)}

    # ----- helpers ------------------------------------------------------------------------------
    def _f32(self, x) -> torch.Tensor:
        if isinstance(x, torch.Tensor):
            t = x.to(device=self.device, dtype=torch.float32)
        else:
            t = torch.as_tensor(np.asarray(x, dtype=np.float32), device=self.device)
        return t.contiguous()

    def empty_traces(self):
        return torch.empty((self.S, self.nt, self.R), dtype=torch.float32, device=self.device)

    def empty_state(self):
        return torch.empty((self.S, 4) + self.shape, dtype=torch.float32, device=self.device)

    # ----- solves ---------------------------------------------------------------------------------
    def forward(self, c, wavelet, final_state: bool = False, capture_every: int = 0):
        c, w = self._f32(c), self._f32(wavelet)
        tr = self.empty_traces()
        fs = self.empty_state() if final_state else None
        cap = None
        if capture_every:
            ncap = (self.nt - 1) // capture_every
            cap = torch.empty((ncap, self.S, 4) + self.shape, dtype=torch.float32, device=self.device)
        L.wave_forward(self.ctx, c, w, tr, fs, cap, capture_every)
        return tr, fs, cap

    def adjoint(self, c, residual):
        g = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        L.wave_adjoint(self.ctx, self._f32(c), self._f32(residual), g)
        return g

    def gradient(self, c, wavelet, d_obs, sigma):
        g = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        status, J = L.gradient(self.ctx, self._f32(c), self._f32(wavelet), self._f32(d_obs), sigma, g)
        self.last_status = status
        return J, g

    def hessvec(self, c, dc, gauss_newton: bool = True):
        """Gauss-Newton (default) or full-Newton Hessian action at the last gradient's c."""
        H = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        self.last_status = L.hessvec(self.ctx, self._f32(c), self._f32(dc), H, 1 if gauss_newton else 0)
        return H

    def inc_forward(self, c, dc):
        dtr = self.empty_traces()
        L.wave_inc_forward(self.ctx, self._f32(c), self._f32(dc), dtr)
        return dtr

    def forward_e(self, c, wavelet, steps):
        """Forward solve returning e^n of every source at the listed levels [len][S][nz][ny][nx]."""
        e = torch.empty((len(steps), self.S) + self.shape, dtype=torch.float32, device=self.device)
        L.wave_forward_e(self.ctx, self._f32(c), self._f32(wavelet), steps, e)
        return e

    def load_e(self, n: int):
        """e^n [S][nz][ny][nx] as the reverse solves read it from the store."""
        out = torch.empty((self.S,) + self.shape, dtype=torch.float32, device=self.device)
        L.wv_load_e(self.ctx, n, out)
        return out

    # ----- MAP point: BiLaplacian prior and Newton-CG --------------------------------------------
    def set_prior(self, alpha: float, theta=(0.0, 0.0, 0.0), c0=None) -> None:
        """BiLaplacian prior with mean c0 (copied); alpha = 0 removes it."""
        L.wv_set_prior(self.ctx, alpha, theta, None if c0 is None else self._f32(c0))

    def prior_sample(self, w, rtol: float = 1e-6, maxit: int = 2000):
        """A prior draw c0 + A^-1 w / sqrt(vol) for white noise w; returns
        (draw, CG iterations, final relative residual)."""
        out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        it, rr = L.wv_prior_sample(self.ctx, self._f32(w), out, rtol, maxit)
        return out, it, rr

    def prior(self, c):
        """(R(c), grad R(c))."""
        g = torch.zeros(self.shape, dtype=torch.float32, device=self.device)
        R = L.wv_prior(self.ctx, self._f32(c), g)
        return R, g

    def prior_hessvec(self, dc):
        H = torch.zeros(self.shape, dtype=torch.float32, device=self.device)
        L.wv_prior_hessvec(self.ctx, self._f32(dc), H)
        return H

    def newton_cg(self, c, wavelet, d_obs, sigma, **cfg):
        """Newton-CG from c for the MAP point; returns (c, records, iterations, reason)."""
        c = self._f32(c).clone()
        log, it, reason = L.wv_newton_cg(self.ctx, c, self._f32(wavelet), self._f32(d_obs), sigma, **cfg)
        return c, log, it, reason
