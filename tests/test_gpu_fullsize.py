"""Parity and properties at the full sizes of the workloads, in the launch
configuration the benchmark times (same grid, same kernels, same tiling).

* 256^3 (the gradient workload): a full-grid gradient over a short horizon
  against the FP64 oracle; checkpointed and all-patches-exact compressed
  stores bit for bit against full storage; the fused encoder and decoder on
  sampled patches of a full-grid state against the oracle.
* 384^3 x 3000 (the Gauss-Newton workload): symmetry of the checkpointed GN
  Hessian and the compressed Hv against the checkpointed one.
* 512 x 512 x 256 with 8 sources (the multi-source FP8 workload) on the full
  grid with a shortened horizon: compressed FP8 gradient against the
  checkpointed one.

The oracle's cost sets the short horizons: one FP64 numpy step of the 256^3
grid takes about a quarter of a second on one core."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import ae as oae
from oracle import rounding as rd
from oracle import wave as ow
from paper_2304_04781_amd import _lib as L
from paper_2304_04781_amd.compressor import Autoencoder, train_from_forward
from paper_2304_04781_amd.solver import WaveSolver

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cosine(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(a @ b / np.linalg.norm(a) / np.linalg.norm(b))


# latents-only (K = 0) gradient at 256^3 x 2000 with the in-run network (bf16,
# plain loss): measured 0.3998 / cosine 0.928; the bounds leave a margin for
# kernel changes that alter the summation order
K0_GRAD_BOUND = 0.45
K0_COS_BOUND = 0.91


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def rounded(p):
    p.c_true = f32(p.c_true)
    p.c_start = f32(p.c_start)
    p.wavelet = f32(p.wavelet)
    return p


# ----- 256^3 ----------------------------------------------------------------------------------------
def test_gradient_256_cube_matches_oracle():
    """Forward, misfit, adjoint and gradient over the full 256^3 grid (40 steps)
    against the FP64 oracle; revolve checkpointing and an all-exact compressed
    store reproduce full storage bit for bit at this size."""
    p = rounded(W.problem_256(40))
    print("case", p.name, flush=True)
    sol = ow.solver_for(p)
    d, sigma, _ = ow.observed_data(sol, p)
    d = f32(d)
    J_o, g_o, _, e_hist = ow.gradient(sol, p.c_start, p.wavelet, p.src, p.rec, d, sigma, src_w=p.src_w)
    del e_hist
    full = WaveSolver.for_problem(p)
    full.set_storage(L.STORE_FULL)
    J, g = full.gradient(p.c_start, p.wavelet, d, sigma)
    g = g.cpu().numpy()
    print("J", J, J_o, "grad rel err", rel(g, g_o), flush=True)
    assert abs(J - J_o) / J_o < 1e-5
    assert rel(g, g_o) < 1e-4
    ck = WaveSolver.for_problem(p)
    ck.set_storage(L.STORE_CHECKPOINT, n_checkpoints=8)
    _, gc = ck.gradient(p.c_start, p.wavelet, d, sigma)
    assert np.array_equal(gc.cpu().numpy(), g)
    net = Autoencoder(W.ae_init(2048, 512, 32, seed=4))
    ae = WaveSolver.for_problem(p)
    P = (p.nz // 8) * (p.ny // 8) * (p.nx // 8)
    L.wv_set_ae_exceptions(ae.ctx, P)
    ae.set_storage(L.STORE_AE_BF16, ae=net)
    Ja, ga = ae.gradient(p.c_start, p.wavelet, d, sigma)
    assert Ja == J
    assert np.array_equal(ga.cpu().numpy(), g)


def test_encode_decode_256_cube_sampled_patches():
    """The fused encoder over a full 256^3 state and the decoder over full-grid
    latents, checked on sampled patches against the oracle's emulated network.
    Decoder inputs are seeded synthetic latents and metadata (not the encoder's
    output), so each direction is checked on its own."""
    shape = (256, 256, 256)
    P = 32 ** 3
    prm = W.ae_init(seed=4)
    prm32 = {k: f32(v) for k, v in prm.items()}
    flat = np.concatenate([prm32[k].ravel() for k in oae.NAMES])
    net = L.ae_create(2048, 512, 32, flat, np.full(4, 1e-7))
    g = L.make_grid(*shape, 20.0, 1e-3, 10, 0, 1.0, 1, 0)
    st = W.smooth_random_state(4, *shape, seed=7).astype(np.float32)
    ts = torch.tensor(st, device="cuda")
    lat = torch.empty((P, 32), dtype=torch.int16, device="cuda")
    meta = torch.empty((P, 4, 2), dtype=torch.float32, device="cuda")
    L.ae_encode(net, g, ts, L.LATENT_BF16, lat, meta)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(P, 96, replace=False))
    pz, py, px = sample // (32 * 32), (sample // 32) % 32, sample % 32
    X = np.stack([st[:, 8 * z:8 * z + 8, 8 * y:8 * y + 8, 8 * x:8 * x + 8].reshape(4, 512)
                  for z, y, x in zip(pz, py, px)]).reshape(-1, 2048).astype(np.float64)
    Y, lo, r = oae.normalize(X, [1e-7] * 4, emulate=True)
    meta_g = meta.cpu().numpy()[sample]
    assert np.array_equal(meta_g[:, :, 0], np.asarray(lo, np.float32))
    assert np.array_equal(meta_g[:, :, 1], np.asarray(r, np.float32))
    ae = oae.AE(prm32)
    z_ref = rd.bf16(ae.encode(Y, emulate=True))
    bits = lat.cpu().numpy().view(np.uint16)[sample]
    z_gpu = rd.bf16_from_bits(bits)
    same = float(np.mean(bits == rd.bf16_bits(z_ref)))
    # codes differ only at rounding ties, by one step, or near zero by what a flipped hidden unit moves them
    near = np.all(np.abs(z_gpu - z_ref) <= 2.0 ** -7 * np.abs(z_ref) + 3e-3 * np.sqrt(np.mean(z_ref ** 2)))
    print("encode rel err on sampled patches", rel(z_gpu, z_ref), "identical codes", same, flush=True)
    assert rel(z_gpu, z_ref) < 5e-4 and same > 0.99 and near
    # decoder: seeded latents (bf16) and metadata for every patch of the grid
    zs = rd.bf16(0.5 * rng.standard_normal((P, 32)))
    ms = np.zeros((P, 4, 2), np.float32)
    ms[:, :, 0] = rng.uniform(-1.0, 1.0, (P, 4))
    ms[:, :, 1] = rng.uniform(0.5, 2.0, (P, 4))
    lat_in = torch.tensor(rd.bf16_bits(zs).view(np.int16), device="cuda")
    meta_in = torch.tensor(ms, device="cuda")
    out = torch.zeros((4,) + shape, dtype=torch.float32, device="cuda")
    L.ae_decode(net, g, lat_in, meta_in, None, L.LATENT_BF16, 0x1, out)
    torch.cuda.synchronize()
    e_gpu = out[0].cpu().numpy()
    got = np.stack([e_gpu[8 * z:8 * z + 8, 8 * y:8 * y + 8, 8 * x:8 * x + 8].ravel()
                    for z, y, x in zip(pz, py, px)])
    yhat = ae.decode(zs[sample], emulate=True)[:, :512]
    ref = ms[sample, 0, 0][:, None].astype(np.float64) + ms[sample, 0, 1][:, None].astype(np.float64) * yhat
    print("decode rel err on sampled patches", rel(got, ref), flush=True)
    assert rel(got, ref) < 3e-5
    L.ae_destroy(net)


def test_compressed_gradient_256_cube_headline():
    """The gradient workload exactly as the benchmark runs it (256^3 x 2000 steps,
    network trained for 20 epochs at batch 4096 on every 10th state of the solve at
    the start model, bf16 latents): with the 1 % largest-range patches of every
    state kept exact (K = 328) the compressed gradient is within 5e-2 relative L2
    of the checkpointed float32 gradient with cosine >= 0.99; latents alone (K = 0,
    the paper's method) are reported and held to their measured level. A central
    difference of the misfit along a GRF direction (h = 1e-3) checks both
    gradients' directional derivative."""
    p = rounded(W.problem_256(2000))
    print("case", p.name, flush=True)
    dev = torch.device("cuda", 0)
    c = torch.tensor(p.c_start, dtype=torch.float32, device=dev)
    wav = torch.tensor(p.wavelet, dtype=torch.float32, device=dev)
    plain = WaveSolver.for_problem(p)
    plain.set_storage(L.STORE_NONE)
    clean, _, _ = plain.forward(torch.tensor(p.c_true, dtype=torch.float32, device=dev), wav)
    sigma = 0.01 * float(clean.abs().max())
    d = (clean.double() + sigma * torch.tensor(p.noise, device=dev)).float()
    del clean
    P = 32 ** 3
    net = Autoencoder(W.ae_init(2048, 512, 32, seed=4))
    nsamp = (1999 // 10) * P
    info = train_from_forward(plain, net, c, wav, every=10, epochs=20, batch=4096,
                              perms=W.shuffles(nsamp, 20, seed=5))
    print("training", info, flush=True)
    ck = WaveSolver.for_problem(p)
    ck.set_storage(L.STORE_CHECKPOINT, n_checkpoints=64)
    J0, g0 = ck.gradient(c, wav, d, sigma)
    ck.close()
    g0n = g0.double()
    res = {}
    for K in (328, 0):
        ae = WaveSolver.for_problem(p)
        L.wv_set_ae_exceptions(ae.ctx, K)
        ae.set_storage(L.STORE_AE_BF16, ae=net)
        J, g = ae.gradient(c, wav, d, sigma)
        assert ae.last_status == 0 and J == J0
        gn = g.double()
        res[K] = (float(torch.linalg.norm(gn - g0n) / torch.linalg.norm(g0n)),
                  float(torch.sum(gn * g0n) / torch.linalg.norm(gn) / torch.linalg.norm(g0n)), gn)
        print(f"K {K}: gradient rel err {res[K][0]:.4f}, cosine {res[K][1]:.5f}", flush=True)
        ae.close()
    assert res[328][0] < 5e-2 and res[328][1] > 0.99
    assert res[0][0] < K0_GRAD_BOUND and res[0][1] > K0_COS_BOUND
    # directional derivative: (J(c + h u) - J(c - h u)) / 2h against <g, u>, u = c * GRF(12 cells)
    u = c * torch.tensor(W.direction_grf(p.c_start.shape, 12.0, 2), dtype=torch.float32, device=dev)
    h = 1e-3
    Js = []
    for sgn in (1.0, -1.0):
        tr, _, _ = plain.forward(c + sgn * h * u, wav)
        Js.append(float(torch.sum((tr.double() - d.double()) ** 2)) * p.dt / (2.0 * sigma ** 2))
    fd = (Js[0] - Js[1]) / (2.0 * h)
    ud = u.double()
    dd = {"checkpoint": float(torch.sum(g0n * ud)), "K=328": float(torch.sum(res[328][2] * ud)),
          "K=0": float(torch.sum(res[0][2] * ud))}
    print("directional derivative: FD", fd, {k: (v, abs(v - fd) / abs(fd)) for k, v in dd.items()}, flush=True)
    assert abs(dd["checkpoint"] - fd) < 1e-3 * abs(fd)
    assert abs(dd["K=328"] - fd) < 2e-2 * abs(fd)


# ----- 384^3 x 3000 ---------------------------------------------------------------------------------
def test_gradient_fd_equals_gn_hessvec_384_cube():
    """At a zero-residual point (data = F(c), noise-free) the Gauss-Newton and the
    full Hessian coincide, so the central difference of the gradient along
    dc = c * GRF(12 cells) with h = 1e-3 must reproduce the Gauss-Newton Hv. Full
    384^3 x 3000 grid, every gradient and the Hv with revolve checkpointing (64
    slots); the gradient at the point itself is zero."""
    p = rounded(W.problem_384(3000))
    print("case", p.name, flush=True)
    dev = torch.device("cuda", 0)
    c = torch.tensor(p.c_start, dtype=torch.float32, device=dev)
    wav = torch.tensor(p.wavelet, dtype=torch.float32, device=dev)
    dc = torch.tensor(p.c_start * W.direction_grf(p.c_start.shape, 12.0, 2), dtype=torch.float32, device=dev)
    ck = WaveSolver.for_problem(p)
    ck.set_storage(L.STORE_CHECKPOINT, n_checkpoints=64)
    d, _, _ = ck.forward(c, wav)
    sigma = 0.01 * float(d.abs().max())
    h = 1e-3
    gs = []
    for sgn in (1.0, -1.0):
        _, g = ck.gradient(c + sgn * h * dc, wav, d, sigma)
        gs.append(g.double())
    fd = (gs[0] - gs[1]) / (2.0 * h)
    del gs
    J, g = ck.gradient(c, wav, d, sigma)
    assert J == 0.0 and not bool(torch.any(g))
    H = ck.hessvec(c, dc).double()
    err = float(torch.linalg.norm(fd - H) / torch.linalg.norm(H))
    print("FD of the gradient vs GN Hv: rel err", err, "cos", float(torch.sum(fd * H) / torch.linalg.norm(fd) /
                                                                   torch.linalg.norm(H)), flush=True)
    assert err < 1e-3



def test_gn_hessvec_384_cube():
    """The Gauss-Newton workload at full size: the checkpointed GN Hessian is
    symmetric to FP32 round-off, and the compressed Hv (trained network, 1 %
    exact patches) agrees with the checkpointed one."""
    p = rounded(W.problem_384(3000))
    print("case", p.name, flush=True)
    dev = torch.device("cuda", 0)
    c = torch.tensor(p.c_start, dtype=torch.float32, device=dev)
    wav = torch.tensor(p.wavelet, dtype=torch.float32, device=dev)
    u = torch.tensor(p.c_start * W.direction_grf(p.c_start.shape, 12.0, 2), dtype=torch.float32, device=dev)
    w = torch.tensor(p.c_start * W.direction_grf(p.c_start.shape, 12.0, 9), dtype=torch.float32, device=dev)
    d = torch.zeros((len(p.src), p.nt, len(p.rec)), dtype=torch.float32, device=dev)
    sigma = 1.0  # GN Hv depends on the data only through the weight dt / sigma^2
    ck = WaveSolver.for_problem(p)
    ck.set_storage(L.STORE_CHECKPOINT, n_checkpoints=64)
    ck.gradient(c, wav, d, sigma)             # Hv linearises about the last gradient's solve
    Hu = ck.hessvec(c, u)
    Hw = ck.hessvec(c, w)
    a = float(torch.sum(w.double() * Hu.double()))
    b = float(torch.sum(u.double() * Hw.double()))
    print("symmetry", a, b, abs(a - b) / abs(a), flush=True)
    assert abs(a - b) / abs(a) < 1e-4
    net = Autoencoder(W.ae_init(2048, 512, 32, seed=4))
    P = (p.nz // 8) * (p.ny // 8) * (p.nx // 8)
    nsamp = ((p.nt - 1) // 60) * P
    info = train_from_forward(ck, net, c, wav, every=60, epochs=6, batch=4096,
                              perms=W.shuffles(nsamp, 6, seed=5))
    print("training", info, flush=True)
    ae = WaveSolver.for_problem(p)
    L.wv_set_ae_exceptions(ae.ctx, int(round(0.01 * P)))
    ae.set_storage(L.STORE_AE_BF16, ae=net)
    ae.gradient(c, wav, d, sigma)
    assert ae.last_status == 0  # compressed, no fallback
    Hu_ae = ae.hessvec(c, u)
    assert ae.last_status == 0
    err = rel(Hu_ae.cpu().numpy(), Hu.cpu().numpy())
    cs = cosine(Hu_ae.cpu().numpy(), Hu.cpu().numpy())
    print("compressed Hv rel err", err, "cos", cs, flush=True)
    assert err < 0.1 and cs > 0.995
    # the configuration stores the incremental forward states as latents too
    ae.set_delta_storage(True)
    b0 = ae.storage_bytes()
    assert torch.equal(ae.hessvec(c, u), Hu_ae)      # storing them changes nothing
    b1 = ae.storage_bytes()
    print("stores: forward %.2f GB, incremental %.2f GB" % (b0 / 1e9, (b1 - b0) / 1e9), flush=True)
    assert b1 == 2 * b0
    dx = ae.decode_delta(p.nt - 1)
    assert bool(torch.isfinite(dx).all()) and float(dx[:, 0].abs().max()) > 0


# ----- 512 x 512 x 256, 8 sources ---------------------------------------------------------------
def test_multisource_fp8_gradient_full_grid():
    """All 8 sources of the multi-source workload in one launch per step on its
    full grid (horizon shortened to 400 steps), FP8 latents with per-patch
    scales: the summed compressed gradient against the checkpointed one."""
    T = 400
    p = rounded(W.problem_multisource(T))
    print("case", p.name, flush=True)
    dev = torch.device("cuda", 0)
    c = torch.tensor(p.c_start, dtype=torch.float32, device=dev)
    wav = torch.tensor(p.wavelet, dtype=torch.float32, device=dev)
    ck = WaveSolver.for_problem(p)
    ck.set_storage(L.STORE_CHECKPOINT, n_checkpoints=6)
    clean, _, _ = ck.forward(torch.tensor(p.c_true, dtype=torch.float32, device=dev), wav)
    clean = clean.cpu().numpy().astype(np.float64)
    sigma = 0.01 * float(np.abs(clean).max())
    d = torch.tensor((clean + sigma * p.noise).astype(np.float32), device=dev)
    J0, g0 = ck.gradient(c, wav, d, sigma)
    net = Autoencoder(W.ae_init(2048, 512, 32, seed=4))
    P = (p.nz // 8) * (p.ny // 8) * (p.nx // 8)
    nsamp = ((T - 1) // 50) * P * len(p.src)
    info = train_from_forward(ck, net, c, wav, every=50, epochs=4, batch=4096,
                              perms=W.shuffles(nsamp, 4, seed=5))
    print("training", info, flush=True)
    errs = {}
    for K in (0, int(round(0.01 * P))):
        ae = WaveSolver.for_problem(p)
        L.wv_set_ae_exceptions(ae.ctx, K)
        ae.set_storage(L.STORE_AE_FP8, ae=net)
        J, g = ae.gradient(c, wav, d, sigma)
        assert ae.last_status == 0  # compressed, no fallback
        err = rel(g.cpu().numpy(), g0.cpu().numpy())
        cs = cosine(g.cpu().numpy(), g0.cpu().numpy())
        print("J", J, J0, "K", K, "FP8 compressed gradient rel err", err, "cos", cs, flush=True)
        assert J == J0
        errs[K] = (err, cs)
        ae.close()
    err, cs = errs[int(round(0.01 * P))]
    assert err < 0.1 and cs > 0.995


# ----- 256^3: MAP layer and time compression ---------------------------------------------------------
def test_prior_and_prior_draw_256_cube():
    """BiLaplacian prior on the full 256^3 grid: cost, gradient and Hessian action
    against the FP64 oracle (1e-5), and a prior draw by CG against the oracle's
    exact cosine-mode solve (1e-4)."""
    from oracle import inverse as oi
    p = rounded(W.problem_256(10))
    print("case", p.name, flush=True)
    alpha, theta = 2.2e-6, (1e4, 1e4, 1e4)
    u = f32(p.c_start * (1.0 + 0.02 * W.direction_grf(p.c_start.shape, 12.0, 5)))
    R_o, g_o = oi.prior_cost_grad(u, p.c_start, alpha, theta, p.dx)
    s = WaveSolver.for_problem(p)
    s.set_prior(alpha, theta, p.c_start)
    R, g = s.prior(u)
    assert abs(R - R_o) < 1e-5 * R_o
    assert rel(g.cpu().numpy(), g_o) < 1e-5
    del g, g_o
    H_o = oi.prior_hessvec(u - p.c_start, alpha, theta, p.dx)
    assert rel(s.prior_hessvec(u - p.c_start).cpu().numpy(), H_o) < 1e-5
    del H_o
    w = f32(W.white_noise(p.c_start.shape, 101))
    c, it, rr = s.prior_sample(w, rtol=1e-6)
    print("CG iterations", it, "residual", rr, flush=True)
    ref = oi.prior_sample(w, p.c_start, alpha, theta, p.dx)
    assert rr <= 1e-6 and rel(c.cpu().numpy() - p.c_start, ref - p.c_start) < 1e-4


def test_time_store_256_cube():
    """Time compression on the full 256^3 grid (69 stored levels: two full windows
    and a short one of 5): the levels the reverse solves read equal the encode-decode
    round trip of the exact windows bit for bit, and the store is 3 windows of
    262,144 vectors."""
    p = rounded(W.problem_256(70))
    print("case", p.name, flush=True)
    net = Autoencoder(W.ae_init(2048, 512, 32, seed=4))
    s = WaveSolver.for_problem(p)
    s.set_storage(L.STORE_NONE)
    e_all = s.forward_e(p.c_start, p.wavelet, list(range(1, 70)))
    L.ae_time_fit_beta(net.handle, s.grid, e_all, 69, 1e-7)
    t = WaveSolver.for_problem(p)
    t.set_storage(L.STORE_AE_TIME, ae=net)
    B = 64 ** 3
    assert t.storage_bytes() == 3 * B * (32 * 2 + 8)
    d = torch.zeros((1, p.nt, len(p.rec)), dtype=torch.float32, device="cuda")
    J, g = t.gradient(p.c_start, p.wavelet, d, 1.0)
    assert torch.isfinite(g).all()
    lat = torch.empty((B, 32), dtype=torch.int16, device="cuda")
    meta = torch.empty((B, 2), dtype=torch.float32, device="cuda")
    dec = torch.empty((32, 1) + t.shape, dtype=torch.float32, device="cuda")
    for w, nvalid in ((0, 32), (1, 32), (2, 5)):
        L.ae_time_encode(net.handle, t.grid, e_all[32 * w:32 * w + nvalid], nvalid, lat, meta)
        L.ae_time_decode(net.handle, t.grid, lat, meta, nvalid, dec)
        for lvl in sorted({0, nvalid // 2, nvalid - 1}):
            n = 32 * w + 1 + lvl
            assert torch.equal(t.load_e(n), dec[lvl]), n


def test_newton_cg_256_cube_checkpointing_equals_full_storage():
    """One Gauss-Newton CG iteration (two Hv) with the BiLaplacian prior on the full
    256^3 grid over 40 steps: revolve checkpointing takes the full-storage path bit
    for bit, and the cost falls."""
    p = rounded(W.problem_256(40))
    print("case", p.name, flush=True)
    s0 = WaveSolver.for_problem(p)
    s0.set_storage(L.STORE_NONE)
    clean, _, _ = s0.forward(p.c_true, p.wavelet)
    sigma = 0.01 * float(clean.abs().max())
    d = clean + sigma * torch.tensor(p.noise, dtype=torch.float32, device="cuda")
    del s0
    out = []
    for mode in (L.STORE_FULL, L.STORE_CHECKPOINT):
        s = WaveSolver.for_problem(p)
        s.set_storage(mode, n_checkpoints=8)
        s.set_prior(2.2e-6, (1e4, 1e4, 1e4), p.c_start)
        out.append(s.newton_cg(p.c_start, p.wavelet, d, sigma, max_newton=1, max_cg=2))
        del s
    (c0, log0, _, _), (c1, log1, _, _) = out
    assert torch.equal(c0, c1)
    assert [r["cost"] for r in log0] == [r["cost"] for r in log1]
    assert log0[1]["cost"] < log0[0]["cost"]
