"""FP64 reference of the patch autoencoder: layout, normalisation,
encoder/decoder, backward pass, Adam and the training loop.

TEST INFRASTRUCTURE ONLY (see the package docstring).

  * Space compression (paper Sec. 3.1): the state is cut into identical
    blocks and each block's values, field by field, form one vector (the
    "compression data structure" of Sec. 3.3.1). Here a block is 8^3 cells
    of the 4 fields (e, v_z, v_y, v_x): x_p[f*512 + lz*64 + ly*8 + lx],
    patch p = (pz*Py + py)*Px + px.
  * Time compression (Sec. 3.2): one field on a 4^3 block of cells over a
    window of 32 consecutive time levels forms a vector (see time_vectors).
  * Normalisation (Sec. 3.3.1): r = max(max x - min x, beta),
    y = (x - min x) / r, applied per field slice of 512 values
    (the paper treats each state variable independently, Sec. 3);
    inverse x = lo + r y.
  * Dense layer (Eq. (single_layer)): sigma(y W + b), W stored [fan_in, fan_out].
    Encoder 2048 -> 512 -> 32, decoder 32 -> 512 -> 2048; GELU (exact erf
    form) on the two hidden layers, affine latent and output.
  * Loss: mean squared error over batch and vector entries (Sec. 3.3.1).
  * Adam (Kingma and Ba, 2015) with bias correction; learning rate halved
    every 5 epochs (Table 2's schedule).

Rounding emulation (emulate=True) applies the HIP path's precision
contract so that differences reduce to FP32 summation order:
  y, W, hidden activations, latent -> bfloat16 (RNE); biases float32;
  products exact and summed (here in FP64); GELU on the unrounded
  pre-activation (here with the exact erf; the kernels use a published
  erf approximation whose error, at most 1.5e-7, sits far below the
  bfloat16 rounding that follows); output float32. An FP8 latent (per-patch scale
  s = max|z|/448, code = e4m3(z/s)) enters the decoder as bfloat16(code*s). Backward: upstream gradients are
  rounded to bfloat16 before they meet a bfloat16 operand in a product,
  bias gradients are plain sums, GELU' uses the stored pre-activation,
  and the latent rounding is treated as the identity.
With emulate=False every step is plain FP64.
"""
from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np
from scipy.special import erf

from . import rounding as rd

PATCH = 8
NFIELD = 4
VEC = NFIELD * PATCH ** 3
NAMES = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")


# ----- layout ---------------------------------------------------------------
def patchify(state: np.ndarray) -> np.ndarray:
    """state [4, nz, ny, nx] -> X [P, 2048]."""
    nf, nz, ny, nx = state.shape
    x = state.reshape(nf, nz // 8, 8, ny // 8, 8, nx // 8, 8)
    x = x.transpose(1, 3, 5, 0, 2, 4, 6)
    return x.reshape(-1, nf * 512).copy()


def unpatchify(X: np.ndarray, nz: int, ny: int, nx: int) -> np.ndarray:
    nf = X.shape[1] // 512
    x = X.reshape(nz // 8, ny // 8, nx // 8, nf, 8, 8, 8)
    x = x.transpose(3, 0, 4, 1, 5, 2, 6)
    return x.reshape(nf, nz, ny, nx).copy()


# ----- time compression layout (Sec. 3.2) ---------------------------------------
# Each vector holds one field (e, the only one the reverse solves read) on a
# 4^3 block of cells over a window of TWIN consecutive time levels:
# x_b[t*64 + lz*16 + ly*4 + lx], block b = (bz*By + by)*Bx + bx, t = 0..TWIN-1.
TBLOCK = 4
TWIN = 32


def time_vectors(e_win: np.ndarray) -> np.ndarray:
    """e_win [TWIN, nz, ny, nx] (consecutive levels) -> X [B, TWIN*64]."""
    w, nz, ny, nx = e_win.shape
    x = e_win.reshape(w, nz // 4, 4, ny // 4, 4, nx // 4, 4)
    x = x.transpose(1, 3, 5, 0, 2, 4, 6)
    return x.reshape(-1, w * 64).copy()


def untime_vectors(X: np.ndarray, nz: int, ny: int, nx: int) -> np.ndarray:
    w = X.shape[1] // 64
    x = X.reshape(nz // 4, ny // 4, nx // 4, w, 4, 4, 4)
    x = x.transpose(3, 0, 4, 1, 5, 2, 6)
    return x.reshape(w, nz, ny, nx).copy()


def pad_window(e_states: np.ndarray, w: int = TWIN) -> np.ndarray:
    """A window with fewer than w levels (the last one of a solve) is filled by
    repeating its last level."""
    n = e_states.shape[0]
    return np.concatenate([e_states, np.repeat(e_states[n - 1:n], w - n, axis=0)]) if n < w else e_states


def normalize_vectors(X: np.ndarray, beta: float, emulate: bool = False):
    """Min/range normalisation of each whole vector (Sec. 3.3.1): lo [B], r [B],
    Y = (X - lo) / r with r = max(max - min, beta); emulate as in normalize."""
    lo = X.min(axis=1)
    hi = X.max(axis=1)
    if emulate:
        r = np.maximum(rd.f32(hi - lo), rd.f32(np.float64(beta)))
        rinv = rd.f32(1.0 / r)
        Y = rd.f32(rd.f32(X - lo[:, None]) * rinv[:, None])
    else:
        r = np.maximum(hi - lo, beta)
        Y = (X - lo[:, None]) / r[:, None]
    return Y, lo, r


# ----- normalisation ----------------------------------------------------------
def normalize(X: np.ndarray, beta, emulate: bool = False, meta_bits: int = 32):
    """Per-(patch, field) min/range normalisation. Returns Y [P, 2048],
    lo [P, 4], r [P, 4]. emulate=True forms the range in FP32 and the
    quotient as the FP32 product of FP32(x - lo) with the FP32-rounded
    reciprocal of the range, as the kernels do.
    meta_bits=16: the offset and scale are kept as bfloat16 (a reading of the
    per-vector offset and scale of Sec. 3.3.1 that fits the 8-source store in
    one GPU): lo is rounded down to bfloat16 first, then r = max(max - lo, beta)
    is rounded up, so lo <= min and lo + r >= max, and the normalisation uses
    exactly the stored values."""
    P = X.shape[0]
    Xf = X.reshape(P, NFIELD, 512)
    lo = Xf.min(axis=2)
    hi = Xf.max(axis=2)
    beta = np.asarray(beta, dtype=np.float64)[None, :]
    if meta_bits == 16:
        lo = rd.bf16_down(lo)
        r = np.maximum(rd.f32(hi - lo), rd.f32(beta)) if emulate else np.maximum(hi - lo, beta)
        r = rd.bf16_up(r)
        if emulate:
            rinv = rd.f32(1.0 / r)
            Y = rd.f32(rd.f32(Xf - lo[..., None]) * rinv[..., None])
        else:
            Y = (Xf - lo[..., None]) / r[..., None]
        return Y.reshape(P, VEC), lo, r
    if meta_bits != 32:
        raise ValueError("meta_bits must be 32 or 16")
    if emulate:
        r = np.maximum(rd.f32(hi - lo), rd.f32(beta))
        rinv = rd.f32(1.0 / r)
        Y = rd.f32(rd.f32(Xf - lo[..., None]) * rinv[..., None])
    else:
        r = np.maximum(hi - lo, beta)
        Y = (Xf - lo[..., None]) / r[..., None]
    return Y.reshape(P, VEC), lo, r


def denormalize(Yhat: np.ndarray, lo: np.ndarray, r: np.ndarray) -> np.ndarray:
    P = Yhat.shape[0]
    nf = Yhat.shape[1] // 512
    return (lo[:, :nf, None] + r[:, :nf, None] * Yhat.reshape(P, nf, 512)).reshape(P, nf * 512)


# ----- activation -------------------------------------------------------------
def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_prime(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


# ----- network ----------------------------------------------------------------
class AE:
    def __init__(self, params: Dict[str, np.ndarray], act: str = "gelu"):
        self.p = {k: np.array(v, dtype=np.float64) for k, v in params.items()}
        self.act = act

    def _sigma(self, a):
        return gelu(a) if self.act == "gelu" else a

    def _sigma_prime(self, a):
        return gelu_prime(a) if self.act == "gelu" else np.ones_like(a)

    def weights(self, emulate: bool):
        if not emulate:
            return self.p
        return {k: (rd.bf16(v) if k.startswith("W") else rd.f32(v)) for k, v in self.p.items()}

    def forward(self, Y: np.ndarray, emulate: bool = False, latent: str = "bf16"):
        """Full pass; returns a dict of intermediates (a = pre-activation,
        h = rounded activation) and the output yhat."""
        w = self.weights(emulate)
        q = rd.bf16 if emulate else (lambda t: t)
        y = q(Y)
        a1 = y @ w["W1"] + w["b1"]
        h1 = q(self._sigma(a1))
        z = h1 @ w["W2"] + w["b2"]
        if emulate:
            zs = rd.f32(z)
            zq = rd.bf16(zs) if latent == "bf16" else rd.bf16(fp8_roundtrip(zs))
        else:
            zq = z
        a3 = zq @ w["W3"] + w["b3"]
        h3 = q(self._sigma(a3))
        yhat = h3 @ w["W4"] + w["b4"]
        if emulate:
            yhat = rd.f32(yhat)
        return dict(y=y, a1=a1, h1=h1, z=z, zq=zq, a3=a3, h3=h3, yhat=yhat)

    def encode(self, Y, emulate: bool = False):
        w = self.weights(emulate)
        q = rd.bf16 if emulate else (lambda t: t)
        h1 = q(self._sigma(q(Y) @ w["W1"] + w["b1"]))
        z = h1 @ w["W2"] + w["b2"]
        return rd.f32(z) if emulate else z

    def decode(self, Z, emulate: bool = False, rows: Optional[slice] = None):
        w = self.weights(emulate)
        q = rd.bf16 if emulate else (lambda t: t)
        h3 = q(self._sigma(Z @ w["W3"] + w["b3"]))
        W4, b4 = w["W4"], w["b4"]
        if rows is not None:
            W4, b4 = W4[:, rows], b4[rows]
        out = h3 @ W4 + b4
        return rd.f32(out) if emulate else out

    def loss_and_grads(self, Y: np.ndarray, emulate: bool = False, latent: str = "bf16",
                       field_weights: Optional[np.ndarray] = None):
        """MSE loss (1/(B*n)) sum (yhat - y)^2 and its parameter gradients.
        field_weights [B, F] (optional) weights each sample's F equal field
        slices of length n/F: loss = sum_bf w_bf sum_i (yhat - y)^2 /
        ((n/F) sum_bf w_bf), which reduces to the plain MSE for equal weights."""
        w = self.weights(emulate)
        f = self.forward(Y, emulate, latent)
        q = rd.bf16 if emulate else (lambda t: t)
        B, n = Y.shape
        diff = f["yhat"] - f["y"]
        if field_weights is None:
            fw, norm = 1.0, float(B * n)
        else:
            fwb = np.asarray(field_weights, dtype=np.float64)
            seg = n // fwb.shape[1]
            fw = np.repeat(fwb, seg, axis=1)
            norm = seg * float(np.sum(fwb))
        loss = float(np.sum(fw * diff * diff)) / norm
        g = {}
        d4 = 2.0 * fw * diff / norm
        d4q = q(d4)
        g["W4"] = f["h3"].T @ d4q
        g["b4"] = d4.sum(axis=0)
        dh3 = d4q @ w["W4"].T
        d3 = dh3 * self._sigma_prime(f["a3"])
        d3q = q(d3)
        g["W3"] = f["zq"].T @ d3q
        g["b3"] = d3.sum(axis=0)
        dz = d3q @ w["W3"].T
        dzq = q(dz)
        g["W2"] = f["h1"].T @ dzq
        g["b2"] = dz.sum(axis=0)
        dh1 = dzq @ w["W2"].T
        d1 = dh1 * self._sigma_prime(f["a1"])
        d1q = q(d1)
        g["W1"] = f["y"].T @ d1q
        g["b1"] = d1.sum(axis=0)
        return loss, g


def fp8_roundtrip(z: np.ndarray) -> np.ndarray:
    """Per-row FP8 storage of latents: s = max|z|/448 (1 if the row is 0),
    code = e4m3(z / s), value = code * s (scale and quotient in FP32)."""
    zmax = np.max(np.abs(z), axis=1, keepdims=True)
    s = np.where(zmax > 0, rd.f32(zmax / rd.E4M3_MAX), 1.0)
    return rd.e4m3(rd.f32(z / s)) * s


def fp8_quantize(z: np.ndarray):
    zmax = np.max(np.abs(z), axis=1, keepdims=True)
    s = np.where(zmax > 0, rd.f32(zmax / rd.E4M3_MAX), 1.0)
    return rd.e4m3_bits(rd.f32(z / s)), s[:, 0]


class Adam:
    def __init__(self, params: Dict[str, np.ndarray], lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = {k: np.zeros_like(v) for k, v in params.items()}
        self.v = {k: np.zeros_like(v) for k, v in params.items()}
        self.t = 0

    def step(self, params: Dict[str, np.ndarray], grads: Dict[str, np.ndarray],
             lr: Optional[float] = None):
        lr = self.lr if lr is None else lr
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for k in params:
            self.m[k] = self.b1 * self.m[k] + (1.0 - self.b1) * grads[k]
            self.v[k] = self.b2 * self.v[k] + (1.0 - self.b2) * grads[k] ** 2
            mhat = self.m[k] / c1
            vhat = self.v[k] / c2
            params[k] = params[k] - lr * mhat / (np.sqrt(vhat) + self.eps)


def train(ae: AE, Y: np.ndarray, perms: np.ndarray, batch: int, lr: float = 1e-3,
          decay_every: int = 5, decay: float = 0.5, emulate: bool = False,
          opt: Optional[Adam] = None, max_steps: Optional[int] = None):
    """Epoch loop: per epoch e the learning rate is lr * decay^(e // decay_every),
    samples are visited in the order perms[e], the last partial batch is
    dropped. Returns the per-epoch mean batch loss."""
    opt = opt or Adam(ae.p, lr=lr)
    losses = []
    steps = 0
    for e, perm in enumerate(perms):
        lr_e = lr * decay ** (e // decay_every)
        tot, nb = 0.0, 0
        for b in range(len(perm) // batch):
            idx = perm[b * batch:(b + 1) * batch]
            loss, g = ae.loss_and_grads(Y[idx], emulate=emulate)
            opt.step(ae.p, g, lr=lr_e)
            tot += loss
            nb += 1
            steps += 1
            if max_steps is not None and steps >= max_steps:
                break
        losses.append(tot / max(nb, 1))
        if max_steps is not None and steps >= max_steps:
            break
    return losses, opt
