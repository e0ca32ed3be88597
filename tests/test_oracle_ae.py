"""Pins of the autoencoder, rounding and checkpointing oracles (paper
Sec. 3.1 layout, Sec. 3.3 dense network and training, Sec. 3.3.1
normalisation; Sec. 1 checkpointing)."""
import math
import struct

import numpy as np
import pytest
import torch

import workloads as W
from oracle import ae as oae
from oracle import revolve as orv
from oracle import rounding as rd


# ----- layout and normalisation ------------------------------------------------------------
def test_patch_layout_brute_force():
    rng = np.random.default_rng(0)
    st = rng.standard_normal((4, 16, 8, 24))
    X = oae.patchify(st)
    Py, Px = 1, 3
    for p in range(X.shape[0]):
        pz, rem = divmod(p, Py * Px)
        py, px = divmod(rem, Px)
        for f in range(4):
            for lz in (0, 5, 7):
                for ly in (0, 3, 7):
                    for lx in (0, 6, 7):
                        assert X[p, f * 512 + lz * 64 + ly * 8 + lx] == \
                            st[f, pz * 8 + lz, py * 8 + ly, px * 8 + lx]
    assert np.array_equal(oae.unpatchify(X, 16, 8, 24), st)


def test_time_layout_brute_force():
    """Time vectors by explicit loops over the definition: e on block (bz, by, bx)
    at level t, cell (lz, ly, lx) sits at entry t*64 + lz*16 + ly*4 + lx of vector
    (bz*By + by)*Bx + bx; the inverse layout returns the window."""
    rng = np.random.default_rng(3)
    nz, ny, nx, w = 8, 4, 12, 32
    e = rng.standard_normal((w, nz, ny, nx))
    X = oae.time_vectors(e)
    By, Bx = ny // 4, nx // 4
    ref = np.zeros(((nz // 4) * By * Bx, w * 64))
    for t in range(w):
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    b = ((k // 4) * By + j // 4) * Bx + i // 4
                    ref[b, t * 64 + (k % 4) * 16 + (j % 4) * 4 + i % 4] = e[t, k, j, i]
    assert np.array_equal(X, ref)
    assert np.array_equal(oae.untime_vectors(X, nz, ny, nx), e)
    # a short last window repeats its last level
    part = oae.pad_window(e[:5])
    assert part.shape == e.shape and np.array_equal(part[:5], e[:5])
    assert all(np.array_equal(part[t], e[4]) for t in range(5, w))
    assert oae.pad_window(e) is e


def test_vector_normalisation_special_cases():
    """Whole-vector min/range: a constant vector maps to 0 with r = beta; the
    minimum maps to 0 and the maximum to 1; x = lo + r y within FP32 rounding."""
    rng = np.random.default_rng(4)
    X = rng.standard_normal((6, 2048)) * 1e-6
    X[2] = 3.0e-7
    Y, lo, r = oae.normalize_vectors(X, 1e-12, emulate=True)
    assert np.all(Y[2] == 0.0) and r[2] == rd.f32(np.float64(1e-12))
    for q in (0, 1, 3):
        assert Y[q, np.argmin(X[q])] == 0.0
        assert abs(Y[q, np.argmax(X[q])] - 1.0) < 1e-6
        assert np.max(np.abs(lo[q] + r[q] * Y[q] - X[q])) < 1e-6 * r[q]
    Y64, lo64, r64 = oae.normalize_vectors(X, 1e-12)
    assert np.max(np.abs(Y64 - Y)) < 1e-6


def test_normalisation_special_cases():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((6, 2048)) * 10.0 ** rng.uniform(-12, 3, size=(6, 1))
    X[2, 512:1024] = 3.25                      # constant field slice
    beta = np.array([1e-7, 2e-7, 3e-7, 4e-7])
    Y, lo, r = oae.normalize(X, beta)
    Yf = Y.reshape(6, 4, 512)
    assert np.all(Yf >= 0.0) and np.all(Yf <= 1.0)
    for p in range(6):
        for f in range(4):
            if p == 2 and f == 1:
                assert r[p, f] == beta[f] and np.all(Yf[p, f] == 0.0) and lo[p, f] == 3.25
                continue
            if r[p, f] > beta[f]:
                assert Yf[p, f].min() == 0.0 and Yf[p, f].max() == 1.0
    Xr = oae.denormalize(Y, lo, r).reshape(6, 4, 512)
    bound = 4 * np.finfo(float).eps * (np.abs(lo) + r)[..., None]
    assert np.all(np.abs(Xr - X.reshape(6, 4, 512)) <= bound)


# ----- activation ---------------------------------------------------------------------------------
def test_gelu_matches_torch_exact_form():
    x = np.linspace(-8, 8, 2001)
    ref = torch.nn.functional.gelu(torch.tensor(x, dtype=torch.float64)).numpy()
    assert np.max(np.abs(oae.gelu(x) - ref)) < 1e-15
    h = 1e-6
    fd = (oae.gelu(x + h) - oae.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - oae.gelu_prime(x))) < 1e-8


# ----- network backward and Adam --------------------------------------------------------------------
def _tiny_params(seed=3, dims=(24, 10, 4)):
    i, h, l = dims
    return W.ae_init(i, h, l, seed=seed)


def test_backward_matches_finite_differences():
    ae = oae.AE(_tiny_params())
    rng = np.random.default_rng(2)
    Y = rng.random((7, 24))
    loss, g = ae.loss_and_grads(Y)
    for name in oae.NAMES:
        P = ae.p[name]
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in P.shape)
            old = P[idx]
            h = 1e-6
            P[idx] = old + h
            lp, _ = ae.loss_and_grads(Y)
            P[idx] = old - h
            lm, _ = ae.loss_and_grads(Y)
            P[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-7 * max(1.0, abs(fd)) + 1e-10


def test_backward_matches_torch_autograd():
    """Independent check of every gradient with torch's CPU autograd in FP64."""
    prm = _tiny_params(seed=5, dims=(32, 16, 6))
    ae = oae.AE(prm)
    rng = np.random.default_rng(3)
    Y = rng.random((9, 32))
    loss, g = ae.loss_and_grads(Y)
    t = {k: torch.tensor(v, requires_grad=True) for k, v in prm.items()}
    y = torch.tensor(Y)
    gel = torch.nn.functional.gelu
    z = gel(y @ t["W1"] + t["b1"]) @ t["W2"] + t["b2"]
    yh = gel(z @ t["W3"] + t["b3"]) @ t["W4"] + t["b4"]
    lt = torch.mean((yh - y) ** 2)
    lt.backward()
    assert abs(lt.item() - loss) < 1e-14
    for k in oae.NAMES:
        assert np.allclose(t[k].grad.numpy(), g[k], rtol=1e-12, atol=1e-15)


def test_adam_first_step_closed_form():
    """Bias correction makes the first Adam step -lr g / (|g| + eps)."""
    rng = np.random.default_rng(4)
    p = {"w": rng.standard_normal(50)}
    g = {"w": rng.standard_normal(50) * 10.0 ** rng.uniform(-6, 2, 50)}
    w0 = p["w"].copy()
    opt = oae.Adam(p, lr=1e-3)
    opt.step(p, g)
    assert np.allclose(p["w"] - w0, -1e-3 * g["w"] / (np.abs(g["w"]) + 1e-8), rtol=1e-12)


def test_linear_autoencoder_reaches_pca_optimum():
    """With identity activations the trained affine AE attains the PCA
    optimum: MSE = (sum of covariance eigenvalues beyond the latent size) / n."""
    rng = np.random.default_rng(5)
    n, lat, ns = 16, 3, 400
    A = rng.standard_normal((n, n)) * np.exp(-0.35 * np.arange(n))[None, :]
    Y = 0.5 + rng.standard_normal((ns, n)) @ A.T * 0.2
    ev = np.sort(np.linalg.eigvalsh(np.cov(Y.T, bias=True)))[::-1]
    opt_mse = ev[lat:].sum() / n
    ae = oae.AE(W.ae_init(n, 8, lat, seed=6), act="identity")
    # the oracle's own training loop: full-batch epochs, rate 1e-2 cut to 3e-3
    # and 9e-4 after 2000 and 4000 epochs
    perms = np.tile(np.arange(ns), (6000, 1))
    oae.train(ae, Y, perms, batch=ns, lr=1e-2, decay_every=2000, decay=0.3)
    loss, _ = ae.loss_and_grads(Y)
    assert loss >= opt_mse * (1 - 1e-9)
    assert loss <= opt_mse * 1.01


def _bf16_torch(x: float) -> float:
    """bfloat16 RNE of the float32 RNE of x, by torch's CPU casts."""
    return float(torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64))


def _f32_struct(x: float) -> float:
    return struct.unpack("f", struct.pack("f", x))[0]


def _e4m3_torch(x: float) -> float:
    return float(torch.tensor(x, dtype=torch.float64).to(torch.float8_e4m3fn).to(torch.float64))


def _hand_chain(prm, Y, latent="bf16", act=True):
    """The HIP path's precision contract applied by hand, one scalar at a time:
    y, weights, hidden activations and the latent rounded to bfloat16 (torch
    casts), biases and the latent and output to float32 (struct), exact sums
    (math.fsum), GELU from math.erf."""
    gel = (lambda a: 0.5 * a * (1.0 + math.erf(a / math.sqrt(2.0)))) if act else (lambda a: a)
    Wq = {k: [[_bf16_torch(v) for v in row] for row in prm[k]] for k in ("W1", "W2", "W3", "W4")}
    bq = {k: [_f32_struct(v) for v in prm[k]] for k in ("b1", "b2", "b3", "b4")}
    i, h = len(Wq["W1"]), len(Wq["W1"][0])
    l = len(Wq["W2"][0])
    out = {k: [] for k in ("y", "a1", "h1", "z", "zq", "a3", "h3", "yhat")}
    for row in Y:
        y = [_bf16_torch(v) for v in row]
        a1 = [math.fsum(y[q] * Wq["W1"][q][j] for q in range(i)) + bq["b1"][j] for j in range(h)]
        h1 = [_bf16_torch(gel(a)) for a in a1]
        z = [math.fsum(h1[q] * Wq["W2"][q][j] for q in range(h)) + bq["b2"][j] for j in range(l)]
        zf = [_f32_struct(v) for v in z]
        if latent == "bf16":
            zq = [_bf16_torch(v) for v in zf]
        else:
            s = max(abs(v) for v in zf)
            s = _f32_struct(s / 448.0) if s > 0 else 1.0
            zq = [_bf16_torch(_e4m3_torch(_f32_struct(v / s)) * s) for v in zf]
        a3 = [math.fsum(zq[q] * Wq["W3"][q][j] for q in range(l)) + bq["b3"][j] for j in range(h)]
        h3 = [_bf16_torch(gel(a)) for a in a3]
        yh = [_f32_struct(math.fsum(h3[q] * Wq["W4"][q][j] for q in range(h)) + bq["b4"][j]) for j in range(i)]
        for k, v in (("y", y), ("a1", a1), ("h1", h1), ("z", z), ("zq", zq), ("a3", a3), ("h3", h3), ("yhat", yh)):
            out[k].append(v)
    return {k: np.array(v) for k, v in out.items()}


@pytest.mark.parametrize("latent", ["bf16", "fp8"])
def test_emulated_chain_equals_hand_rounding(latent):
    """Every rounding point of the emulation mode, checked against the contract
    applied by hand on a tiny network (8 -> 6 -> 3 -> 6 -> 8): rounded quantities
    (h1, latent, h3, output) bit for bit, unrounded pre-activations to float64
    summation order. Dropping any rounding point (of y, a weight, a bias, a hidden
    layer, the latent or the output) changes a compared quantity by far more than
    that order."""
    prm = W.ae_init(8, 6, 3, seed=21)
    for k in prm:                       # weights of order 1 (the fan-ins are small)
        prm[k] = prm[k] * (3.0 if k.startswith("W") else 1.0)
    rng = np.random.default_rng(22)
    Y = rng.random((5, 8))
    hand = _hand_chain(prm, Y, latent)
    ae = oae.AE(prm)
    f = ae.forward(Y, emulate=True, latent=latent)
    for k in ("y", "h1", "zq", "h3", "yhat"):
        assert np.array_equal(f[k], hand[k]), k
    assert np.array_equal(rd.f32(f["z"]), rd.f32(hand["z"]))
    for k in ("a1", "z", "a3"):
        assert np.allclose(f[k], hand[k], rtol=0, atol=1e-14 * np.abs(hand[k]).max()), k
    # encode and decode (row subset) follow the same points
    assert np.array_equal(ae.encode(Y, emulate=True), rd.f32(hand["z"]))
    assert np.array_equal(ae.decode(hand["zq"], emulate=True), hand["yhat"])
    assert np.array_equal(ae.decode(hand["zq"], emulate=True, rows=slice(2, 5)), hand["yhat"][:, 2:5])
    # the test data exercises every rounding point: each omission moves a quantity
    assert not np.array_equal(oae.AE(prm).forward(Y)["yhat"], hand["yhat"])
    assert np.max(np.abs(np.asarray([_bf16_torch(v) for v in Y.ravel()]) - Y.ravel())) > 1e-4
    Wd = max(abs(_bf16_torch(v) - v) for v in prm["W1"].ravel())
    bd = max(abs(_f32_struct(v) - v) for v in prm["b1"].ravel())
    assert Wd > 1e-4 and bd > 1e-12 > 1e-14 * np.abs(hand["a1"]).max()
    assert np.max(np.abs(oae.gelu(hand["a1"]) - hand["h1"])) > 1e-4
    assert np.max(np.abs(hand["z"] - hand["zq"])) > 1e-4
    assert np.max(np.abs(oae.gelu(hand["a3"]) - hand["h3"])) > 1e-4
    out_unrounded = hand["h3"] @ np.vectorize(_bf16_torch)(prm["W4"]) + np.vectorize(_f32_struct)(prm["b4"])
    assert np.max(np.abs(out_unrounded - hand["yhat"])) > 1e-12


def test_fp8_scale_rule_hand_rows():
    """Per-row FP8 storage of the latents: s = max|z| / 448 (float32), s = 1 for a
    zero row, codes e4m3(z / s). Rows worked out by hand."""
    z = np.array([[448.0, -224.0, 1.0, 0.0],
                  [3.5, -1.75, 0.875, 0.0],          # s = 2^-7: quotients 448, -224, 112, 0
                  [0.0, 0.0, 0.0, 0.0],              # zero row: s = 1, all codes 0
                  [2e-3, 1e-3, -5e-4, 7.77e-4]])     # quotients 448, 224, -112, 174.05 -> 176
    codes, s = oae.fp8_quantize(z)
    assert s.shape == (4,)
    assert s[0] == 1.0 and s[1] == 2.0 ** -7 and s[2] == 1.0
    assert s[3] == np.float32(2e-3 / 448.0)
    # 448 = 1.75 * 2^8 -> (15 << 3) | 6; 224 -> (14 << 3) | 6; 1 -> 7 << 3;
    # 112 -> (13 << 3) | 6; 176 = 1.375 * 2^7 -> (14 << 3) | 3; sign bit 0x80
    assert codes.tolist() == [[0x7E, 0xF6, 0x38, 0x00],
                              [0x7E, 0xF6, 0x6E, 0x00],
                              [0x00, 0x00, 0x00, 0x00],
                              [0x7E, 0x76, 0xEE, 0x73]]
    back = oae.fp8_roundtrip(z)
    assert np.array_equal(back[:3], z[:3])            # exactly representable after scaling
    assert np.allclose(back[3], np.array([448.0, 224.0, -112.0, 176.0]) * s[3], rtol=0, atol=0)


def test_fp8_row_maximum_maps_to_448():
    """For any nonzero row the entry of largest magnitude is stored as +-448 times
    the scale (code 0x7E or 0xFE), every value keeps its sign, and the round trip
    is within the e4m3 half-spacing (2^-4 relative above 2^-6 s, 2^-10 s below)."""
    rng = np.random.default_rng(23)
    z = rng.standard_normal((200, 32)) * 10.0 ** rng.uniform(-8, 4, (200, 1))
    codes, s = oae.fp8_quantize(z)
    top = np.argmax(np.abs(z), axis=1)
    c = codes[np.arange(200), top]
    assert np.all((c == 0x7E) | (c == 0xFE))
    assert np.all(np.sign(z[np.arange(200), top]) == np.where(c == 0x7E, 1.0, -1.0))
    back = oae.fp8_roundtrip(z)
    a = np.abs(z) / s[:, None]
    bound = np.where(a >= 2.0 ** -6, 2.0 ** -4 * np.abs(z) * (1 + 1e-6), 2.0 ** -10 * s[:, None] * (1 + 1e-6))
    assert np.all(np.abs(back - z) <= bound)
    assert np.all((back == 0) | (np.sign(back) == np.sign(z)))


def test_train_loop_schedule_and_dropped_batch():
    """oracle.ae.train: epoch e visits perms[e] in batches, drops the last partial
    batch, steps Adam at rate lr * decay^(e // decay_every) and reports each
    epoch's mean batch loss; max_steps ends the loop early."""
    class Probe:
        def __init__(self):
            self.p = {"w": np.zeros(1)}
            self.batches = []

        def loss_and_grads(self, Yb, emulate=False):
            self.batches.append(Yb[:, 0].astype(int).tolist())
            return float(Yb[:, 0].sum()), {"w": np.zeros(1)}

    class Opt:
        def __init__(self):
            self.rates = []

        def step(self, params, grads, lr=None):
            self.rates.append(lr)

    n, batch, epochs = 10, 4, 12
    Y = np.arange(n, dtype=np.float64)[:, None]
    perms = W.shuffles(n, epochs, seed=31)
    probe, opt = Probe(), Opt()
    losses, _ = oae.train(probe, Y, perms, batch, lr=1e-3, decay_every=5, decay=0.5, opt=opt)
    expect = [perms[e][b * 4:(b + 1) * 4].tolist() for e in range(epochs) for b in range(2)]
    assert probe.batches == expect                      # samples perm[8:10] never seen
    assert opt.rates == [1e-3 * 0.5 ** (e // 5) for e in range(epochs) for _ in range(2)]
    assert opt.rates[9] == 1e-3 and opt.rates[10] == 5e-4 and opt.rates[-1] == 2.5e-4
    assert losses == [float(np.mean([sum(perms[e][:4]), sum(perms[e][4:8])])) for e in range(epochs)]
    probe2, opt2 = Probe(), Opt()
    losses2, _ = oae.train(probe2, Y, perms, batch, opt=opt2, max_steps=7)
    assert len(probe2.batches) == 7 and len(losses2) == 4
    assert losses2[3] == float(sum(perms[3][:4]))


def test_emulated_forward_close_to_fp64():
    prm = W.ae_init(2048, 512, 32, seed=4)
    ae = oae.AE(prm)
    rng = np.random.default_rng(6)
    Y = rng.random((16, 2048))
    a = ae.forward(Y)["yhat"]
    b = ae.forward(Y, emulate=True)["yhat"]
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 2e-2
    assert np.linalg.norm(a - b) / np.linalg.norm(a) > 0.0


# ----- rounding -------------------------------------------------------------------------------------
def test_bf16_codes_roundtrip_and_nearest():
    codes = np.arange(1 << 16, dtype=np.uint16)
    vals = rd.bf16_from_bits(codes)
    fin = np.isfinite(vals)
    assert np.array_equal(rd.bf16_bits(vals[fin]), codes[fin])
    rng = np.random.default_rng(7)
    x = rd.f32(rng.standard_normal(200000) * 10.0 ** rng.uniform(-30, 30, 200000))
    r = rd.bf16(x)
    # brute force: no representable neighbour is strictly closer; ties go to even code
    b = rd.bf16_bits(x).astype(np.int64)
    for d in (-1, 1):
        nb = rd.bf16_from_bits((b + d).astype(np.uint16))
        ok = np.isfinite(nb)
        closer = np.abs(nb - x) < np.abs(r - x)
        assert not np.any(closer & ok)
        tie = (np.abs(nb - x) == np.abs(r - x)) & ok
        assert np.all((b[tie] & 1) == 0)
    t = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(t, r)


def test_e4m3_table_and_rounding():
    codes = np.arange(256, dtype=np.uint8)
    vals = rd.e4m3_decode(codes)
    finite = np.isfinite(vals)
    assert finite.sum() == 254 and np.nanmax(vals) == 448.0
    assert np.nanmin(np.abs(vals[vals != 0])) == 2.0 ** -9
    pos = np.unique(vals[finite & (vals >= 0)])
    # every midpoint between neighbours rounds to the neighbour with even code
    mids = 0.5 * (pos[1:] + pos[:-1])
    got = rd.e4m3(mids)
    lo_codes = rd.e4m3_bits(pos[:-1])
    expect = np.where((lo_codes & 1) == 0, pos[:-1], pos[1:])
    assert np.array_equal(got, expect)
    rng = np.random.default_rng(8)
    x = rng.uniform(-460, 460, 100000) * 10.0 ** rng.integers(-4, 1, 100000)
    r = rd.e4m3(x)
    allv = np.concatenate([-pos, pos])
    nearest = np.min(np.abs(allv[None, :] - x[:, None]), axis=1)
    assert np.allclose(np.abs(r - x), nearest, rtol=0, atol=0)
    assert np.all(np.abs(r) <= 448.0)
    assert np.array_equal(rd.e4m3_decode(rd.e4m3_bits(r)), r)
    inr = np.abs(x) <= 448.0
    t = torch.tensor(x[inr]).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(t, r[inr])


def test_bf16_directed_rounding_brute_force():
    """bf16_down / bf16_up against the sorted table of every finite bfloat16 value:
    the largest value <= x and the smallest >= x (exact values map to themselves)."""
    codes = np.arange(1 << 16, dtype=np.uint16)
    vals = rd.bf16_from_bits(codes)
    table = np.unique(vals[np.isfinite(vals)])
    rng = np.random.default_rng(24)
    x = rng.standard_normal(100000) * 10.0 ** rng.uniform(-30, 30, 100000)
    x = np.concatenate([x, rd.f32(x[:50000]), table[1:-1], [0.0, -0.0, 1.0, -1.0]])
    dn, up = rd.bf16_down(x), rd.bf16_up(x)
    i = np.searchsorted(table, x, side="right") - 1          # table[i] <= x < table[i + 1]
    assert np.array_equal(dn, table[i])
    j = np.searchsorted(table, x, side="left")               # table[j - 1] < x <= table[j]
    assert np.array_equal(up, table[j])


def test_normalisation_16_bit_metadata():
    """16-bit metadata: lo and r are bfloat16 values with lo <= min and lo + r >= max
    (so y stays in [0, 1] up to the quotient's rounding), r >= beta, and each is the
    tightest such bfloat16 (one step less would break an inequality); a patch with a
    large offset keeps it to within one bfloat16 step below its minimum."""
    rng = np.random.default_rng(25)
    X = rng.standard_normal((40, 2048)) * 10.0 ** rng.uniform(-9, 3, size=(40, 1))
    X[3] += 7.0                                # offset far above the range
    X[5, 512:1024] = 0.125                     # constant slice: r = beta rounded up
    X = rd.f32(X)
    beta = rd.f32(np.array([1e-7, 2e-7, 3e-7, 4e-7]))
    for emulate in (False, True):
        Y, lo, r = oae.normalize(X, beta, emulate=emulate, meta_bits=16)
        Xf = X.reshape(40, 4, 512)
        mn, mx = Xf.min(axis=2), Xf.max(axis=2)
        assert np.array_equal(rd.bf16(lo), lo) and np.array_equal(rd.bf16(r), r)
        assert np.all(lo <= mn) and np.all(lo + r >= mx) and np.all(r >= beta)
        o = rd._bf16_ordered(rd.bf16_bits(lo))
        above = rd.bf16_from_bits(rd._bf16_from_ordered(o + 1))
        assert np.all(above > mn)                              # lo is the largest bfloat16 <= min
        assert np.all(Y >= 0.0) and np.all(Y <= 1.0 + 1e-6)
    assert r[5, 1] == rd.bf16_up(beta[1]) and np.all(Y.reshape(40, 4, 512)[5, 1] == 0.0)
    assert np.all(mn[3] - lo[3] <= 2.0 ** -7 * np.abs(mn[3]))


# ----- checkpointing cost -----------------------------------------------------------------------------
def test_revolve_closed_form_equals_dp():
    T = orv.dp_table(120, 7)
    for l in range(1, 121):
        for s in range(1, 8):
            assert T[l, s] == orv.closed_form(l, s), (l, s)


def test_revolve_counts_for_the_workloads():
    assert orv.closed_form(2000, 64) == 3934
    assert orv.closed_form(3000, 64) == 6789
    assert orv.closed_form(4000, 64) == 9789
    assert orv.closed_form(50, 1) == 50 * 49 // 2


def test_weighted_loss_reduces_to_mse_and_matches_fd():
    ae = oae.AE(_tiny_params(seed=7, dims=(24, 10, 4)))
    rng = np.random.default_rng(9)
    Y = rng.random((6, 24))
    l0, g0 = ae.loss_and_grads(Y)
    l1, g1 = ae.loss_and_grads(Y, field_weights=np.full((6, 4), 3.5))
    assert abs(l0 - l1) < 1e-15 and all(np.allclose(g0[k], g1[k], rtol=1e-13) for k in oae.NAMES)
    w = rng.uniform(0.1, 10.0, (6, 4))
    loss, g = ae.loss_and_grads(Y, field_weights=w)
    # brute force: weighted sum of per-slice squared errors
    yh = ae.forward(Y)["yhat"]
    ref = sum(w[b, f] * np.sum((yh[b, 6 * f:6 * f + 6] - Y[b, 6 * f:6 * f + 6]) ** 2)
              for b in range(6) for f in range(4)) / (6 * w.sum())
    assert abs(loss - ref) < 1e-14
    for name in ("W1", "b4", "W3"):
        P = ae.p[name]
        idx = tuple(rng.integers(0, s) for s in P.shape)
        old = P[idx]
        P[idx] = old + 1e-6
        lp, _ = ae.loss_and_grads(Y, field_weights=w)
        P[idx] = old - 1e-6
        lm, _ = ae.loss_and_grads(Y, field_weights=w)
        P[idx] = old
        assert abs((lp - lm) / 2e-6 - g[name][idx]) <= 1e-7 * max(1.0, abs(g[name][idx]))
