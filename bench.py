"""Benchmark: autoencoder-compressed adjoint gradient of the 3D acoustic
velocity-strain misfit at 256^3 cells x 2000 steps on one MI355X, against the
same gradient with optimal binomial checkpointing (64 state slots).

    python bench.py [--steps K] [--warmup W] [--gpus 1]

One "step" is one misfit gradient: forward solve with every state compressed
(normalise, encode, latent store), misfit, and the time-reversed adjoint solve
that decompresses e^k at every step and accumulates the gradient. Inputs are
seeded synthetic layered media (workloads.problem_256); observations are the
forward solve at the true model plus 1 % Gaussian noise. Before timing, the
autoencoder is trained by the library on 200 snapshots of the first forward
solve at the start model (every 10th step). Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--nt", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--snapshot-every", type=int, default=10)
    ap.add_argument("--exceptions", type=float, default=0.01, help="fraction of patches kept exactly")
    ap.add_argument("--latent", choices=["bf16", "fp8"], default="bf16")
    ap.add_argument("--weighting", type=int, default=0,
                    help="training loss: 0 plain MSE of the normalised vectors (the paper's), 1 each field slice "
                         "weighted by (r / beta)^2")
    ap.add_argument("--checkpoints", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--multisource", action="store_true",
                    help="the 8-source 512 x 512 x 256 workload with FP8 latents at its full horizon (--ms-nt): "
                         "compressed gradient vs checkpointing source by source, kernel rates; prints its own JSON "
                         "line")
    ap.add_argument("--ms-nt", type=int, default=4000)
    ap.add_argument("--ms-every", type=int, default=500, help="training states of the multi-source leg")
    ap.add_argument("--ms-epochs", type=int, default=10)
    ap.add_argument("--ms-rate-nt", type=int, default=120, help="horizon of the multi-source kernel-rate pass")
    ap.add_argument("--bayes", action="store_true",
                    help="training on prior draws (Algorithm 1) against in-run snapshots at 256^3: "
                         "compression and gradient errors on the start, true, midway and a held-out model")
    ap.add_argument("--draws", type=int, default=4)
    ap.add_argument("--no-time", action="store_true",
                    help="skip the time-compression leg of the default run")
    ap.add_argument("--inversion", action="store_true",
                    help="a short MAP inversion at 256^3 x 2000 (prior-preconditioned Gauss-Newton CG) with the "
                         "AE store and with checkpointing: wall time, Hv count, cost and model error")
    ap.add_argument("--inv-iters", type=int, default=5)
    ap.add_argument("--hv384", action="store_true",
                    help="the 384^3 x 3000 Gauss-Newton Hv with both histories compressed vs checkpointing")
    ap.add_argument("--hv-nt", type=int, default=3000)
    ap.add_argument("--hv-epochs", type=int, default=10)
    ap.add_argument("--inv-store", choices=["space", "time"], default="space",
                    help="compressed store of the inversion: space patches (bf16) or time windows")
    ap.add_argument("--time", action="store_true",
                    help="time-compression scheme at 256^3 x 2000: gradient and Gauss-Newton Hv against "
                         "checkpointing (network trained on every 4th window of the start model's solve)")
    ap.add_argument("--no-newton", action="store_true",
                    help="skip the timed Newton-CG iteration (AE store vs checkpointing)")
    ap.add_argument("--newton-cg", type=int, default=10, help="CG iterations of the timed Newton step")
    ap.add_argument("--counters", action="store_true",
                    help="short run for rocprofv3 --pmc passes: a device copy of known size, then a few steps of "
                         "every hot-path kernel at the full grid")
    return ap.parse_args()


COUNTERS_FILE = os.path.join(ROOT, "profiles", "adjoint_stencil_256cube_hbm_counters.txt")
STENCIL_SOURCE = os.path.join(ROOT, "paper_2304_04781_amd", "csrc", "stencil.hip")


def stencil_source_hash() -> str:
    import hashlib
    with open(STENCIL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None
    when there is none or the stencil source changed since it was taken."""
    try:
        with open(COUNTERS_FILE) as f:
            rows = [json.loads(l[5:]) for l in f if l.startswith("JSON:")]
    except OSError:
        return None
    for r in rows:
        if r.get("kernel") == kernel and r.get("stencil_source_sha256") == stencil_source_hash():
            return r.get("traffic_bytes_per_launch")
    return None


def counters_pass():
    import torch
    import workloads as W
    from paper_2304_04781_amd import _lib as L
    from paper_2304_04781_amd.solver import WaveSolver
    from paper_2304_04781_amd.compressor import Autoencoder
    L.load()
    dev = torch.device("cuda", 0)
    n = 1 << 28  # 1 GiB of float32: the copy reads and writes exactly this
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    T = 12
    p = W.problem_256(T)
    c0 = torch.tensor(p.c_start, dtype=torch.float32, device=dev)
    wav = torch.tensor(p.wavelet, dtype=torch.float32, device=dev)
    d = torch.zeros((len(p.src), T, len(p.rec)), dtype=torch.float32, device=dev)
    ck = WaveSolver.for_problem(p)
    ck.set_storage(L.STORE_CHECKPOINT, n_checkpoints=4)
    ck.gradient(c0, wav, d, 1.0)
    net = Autoencoder(W.ae_init(2048, 512, 32, seed=4))
    ae = WaveSolver.for_problem(p)
    L.wv_set_ae_exceptions(ae.ctx, 328)
    ae.set_storage(L.STORE_AE_BF16, ae=net)
    ae.gradient(c0, wav, d, 1.0)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 4 * n, "grid": [p.nz, p.ny, p.nx], "steps": T,
                      "stencil_source_sha256": stencil_source_hash()}), flush=True)


def timed_kernels(sol, c0, wav, d_obs, sigma, every=4):
    """Mean launch durations per kernel class over one gradient, with HIP events
    around every `every`-th launch of each class (a pass of its own, so the timed
    gradients carry no events)."""
    sol.set_timing(every)
    sol.gradient(c0, wav, d_obs, sigma)
    kt = sol.kernel_times()
    sol.set_timing(0)
    return kt



def device_shuffles(n, epochs, seed=5):
    """One random permutation of range(n) per training epoch, int32 [epochs, n], drawn on
    cuda:0 by torch's generator seeded with `seed`: twenty host permutations of the 256^3
    training set take about two seconds, on the device a few milliseconds."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return torch.stack([torch.randperm(n, generator=g, device="cuda", dtype=torch.int32) for _ in range(epochs)])

def stream_ceilings(torch, dev, n, reps=20):
    """HBM rate (read + write bytes per second) of the library's streaming probe with
    the stencils' array mixes, n floats per array: the practical ceiling beside the
    published 8 TB/s."""
    from paper_2304_04781_amd import _lib as L
    n = n // 4 * 4
    inp = torch.ones((7, n), dtype=torch.float32, device=dev)
    out = torch.empty((5, n), dtype=torch.float32, device=dev)
    res = {}
    for name, (a, b) in (("copy_1in_1out", (1, 1)), ("forward_mix_5in_4out", (5, 4)),
                         ("adjoint_mix_7in_5out", (7, 5))):
        us = L.wv_stream_probe(inp, out, a, b, n, reps)
        res[name] = round((a + b) * 4.0 * n / (us * 1e-6) / 1e9, 1)
    torch.cuda.synchronize()
    del inp, out
    torch.cuda.empty_cache()
    return res


def gemm_peak_tflops(torch, dev, n=8192, reps=10):
    """Dense bf16 GEMM rate of the vendor library (torch.matmul, n x n x n, contiguous
    operands): the measured MFMA reference next to the published 2.5 PFLOP/s."""
    a = torch.randn((n, n), dtype=torch.bfloat16, device=dev)
    b = torch.randn((n, n), dtype=torch.bfloat16, device=dev)
    for _ in range(3):
        c = torch.matmul(a, b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        c = torch.matmul(a, b)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del a, b, c
    return 2.0 * n ** 3 / t / 1e12


def copy_peak_gbs(torch, dev, nbytes=1 << 30, reps=10):
    """Device-to-device copy rate (read + write bytes per second) of a 1 GiB buffer: the
    measured reference next to the published 8 TB/s."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return 2.0 * nbytes / t / 1e9


def multisource_pass(args):
    """The 8-source 512 x 512 x 256 workload at its full horizon (--ms-nt, default 4000
    steps): one launch per step for all sources, FP8 latents with per-patch scales and
    16-bit (lo, r) metadata, latents only (the 8 x 3999 stored states take 218 GB; with
    float32 metadata 285 GB, and exact patches would add 86 GB). The network is trained
    on a random half of the patches of every 500th state of all sources at the start
    model; the summed compressed gradient is compared with the checkpointed float32
    gradient computed source by source (64 slots each). Also reports kernel rates."""
    import torch
    import workloads as W
    from paper_2304_04781_amd import _lib as L
    from paper_2304_04781_amd import compressor as C
    from paper_2304_04781_amd.solver import WaveSolver
    L.load()
    dev = torch.device("cuda", 0)
    T = args.ms_nt
    p = W.problem_multisource(T)
    S, N = len(p.src), p.n
    P = (p.nz // 8) * (p.ny // 8) * (p.nx // 8)
    c0 = torch.tensor(p.c_start, dtype=torch.float32, device=dev)
    wav = torch.tensor(p.wavelet, dtype=torch.float32, device=dev)
    t_all = time.perf_counter()
    # observations: the 8-source forward solve at the true model plus 1 % noise
    plain = WaveSolver.for_problem(p)
    plain.set_storage(L.STORE_NONE)
    clean, _, _ = plain.forward(torch.tensor(p.c_true, dtype=torch.float32, device=dev), wav)
    sigma = 0.01 * float(clean.abs().max())
    d = (clean.double() + sigma * torch.tensor(p.noise, device=dev)).float()
    del clean
    log(f"multisource: observations done ({time.perf_counter() - t_all:.1f} s)")
    # training vectors: half the patches of every ms_every-th state of every source at c0
    every = args.ms_every
    net = C.Autoencoder(W.ae_init(2048, 512, 32, seed=4))
    ncap = (T - 1) // every
    rows = W.keep_rows(1, ncap * S, P, 0.5, seed=6)
    y, meta, t_cap = C.prior_draw_samples(plain, net, [c0], p.wavelet, every, rows)
    n = int(y.shape[0])
    info = C.train_samples(net, y, meta, epochs=args.ms_epochs, batch=args.batch,
                           perms=device_shuffles(n, args.ms_epochs, seed=5))
    del y, meta
    plain.close()
    torch.cuda.empty_cache()
    log(f"multisource: training {info}")
    # compressed gradient, all sources per launch
    free, total = torch.cuda.mem_get_info()
    log(f"multisource: device memory free {free / 1e9:.1f} GB of {total / 1e9:.1f} GB")
    ae = WaveSolver.for_problem(p)
    L.wv_set_ae_metadata(ae.ctx, 16)
    ae.set_storage(L.STORE_AE_FP8, ae=net)
    store_gb = ae.storage_bytes() / 1e9
    log(f"multisource: AE store {store_gb:.1f} GB")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    J, g_ae = ae.gradient(c0, wav, d, sigma)
    ev1.record()
    torch.cuda.synchronize()
    t_ae = ev0.elapsed_time(ev1) / 1e3
    log(f"multisource: AE gradient {t_ae:.2f} s")
    # kernel rates over a short horizon (the same kernels; timed launches every 2nd)
    g_ae = g_ae.double().cpu().reshape(-1)
    ae.close()
    torch.cuda.empty_cache()
    # checkpointed reference, one source at a time (64 slots of one wavefield each)
    g_ck = torch.zeros(N, dtype=torch.float64)
    J_ck, t_ck = 0.0, 0.0
    import copy
    for src in range(S):
        ps = copy.copy(p)
        ps.src = ps.src[src:src + 1]
        ps.wavelet = ps.wavelet[src:src + 1]
        ps.noise = ps.noise[src:src + 1]
        ck = WaveSolver.for_problem(ps)
        ck.set_storage(L.STORE_CHECKPOINT, n_checkpoints=64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Js, gs = ck.gradient(c0, wav[src:src + 1].contiguous(), d[src:src + 1].contiguous(), sigma)
        torch.cuda.synchronize()
        t_ck += time.perf_counter() - t0
        J_ck += Js
        g_ck += gs.double().cpu().reshape(-1)
        ck.close()
        log(f"multisource: checkpointed source {src} done ({t_ck:.1f} s so far)")
    err = float(torch.linalg.norm(g_ae - g_ck) / torch.linalg.norm(g_ck))
    cos = float(torch.sum(g_ae * g_ck) / torch.linalg.norm(g_ae) / torch.linalg.norm(g_ck))
    # kernel rates on a short horizon of the same grid
    rates = multisource_rates(args, p, net, c0, wav)
    print(json.dumps({"workload": f"{p.name}: 8 sources per launch, FP8 latents + per-patch scale, 16-bit (lo, r) "
                                  f"metadata, latents only, horizon {T} steps",
                      "grid": [p.nz, p.ny, p.nx], "sources": S, "nt": T,
                      "training": info, "capture_s": round(t_cap, 2),
                      "ae_gradient_s": round(t_ae, 3), "checkpoint_gradient_s_sum_over_sources": round(t_ck, 3),
                      "speedup_vs_checkpoint": round(t_ck / t_ae, 4),
                      "summed_grad_rel_err_vs_checkpoint_fp32": round(err, 5), "summed_grad_cos": round(cos, 6),
                      "misfit": {"ae": J, "checkpoint_sum": J_ck},
                      "ae_store_GB": round(store_gb, 2),
                      "compression_vs_float32_history": round(16.0 * N * (T - 1) * S / (store_gb * 1e9), 1),
                      "kernels": rates, "wall_s": round(time.perf_counter() - t_all, 1)}), flush=True)


def multisource_rates(args, p, net, c0, wav):
    """Mean kernel durations of the 8-source workload over a short horizon (the same grid
    and launches) and their HBM / MFMA rates."""
    import torch
    import workloads as W
    from paper_2304_04781_amd import _lib as L
    from paper_2304_04781_amd.solver import WaveSolver
    import copy
    T = args.ms_rate_nt
    pr = copy.copy(p)
    pr.nt = T
    S, N = len(pr.src), pr.n
    P = (pr.nz // 8) * (pr.ny // 8) * (pr.nx // 8)
    d = torch.zeros((S, T, len(pr.rec)), dtype=torch.float32, device=c0.device)
    ae = WaveSolver.for_problem(pr)
    L.wv_set_ae_metadata(ae.ctx, 16)
    ae.set_storage(L.STORE_AE_FP8, ae=net)
    w = wav[:, :T].contiguous()
    ae.gradient(c0, w, d, 1.0)
    kt = timed_kernels(ae, c0, w, d, 1.0, every=2)
    ae.close()
    blk = L.wv_accumulation_block()
    work = {  # per timed launch (the stencils launch all sources at once; encode/decode time one state)
        "forward_stencil": ("hbm", (32.0 * S + 4.0) * N),
        "adjoint_stencil": ("hbm", ((adjoint_bytes_per_cell(T, blk) - 4.0) * S + 4.0) * N),
        "encode": ("mfma", S * 2.0 * P * (2048 * 512 + 512 * 32)),
        "decode_e": ("mfma", 2.0 * P * (32 * 512 + 512 * 512)),
    }
    rows = {}
    for name, (us, n) in kt.items():
        if not n:
            continue
        row = {"us": round(us, 2), "timed_launches": n}
        if name in work:
            kind, wk = work[name]
            rate = wk / (us * 1e-6)
            if kind == "hbm":
                row.update({"GB/s": round(rate / 1e9, 1), "frac_hbm": round(rate / 1e9 / HBM_PEAK_GBS, 4)})
            else:
                row.update({"TFLOP/s": round(rate / 1e12, 1),
                            "frac_mfma_bf16": round(rate / 1e12 / BF16_PEAK_TFLOPS, 4)})
        rows[name] = row
    rows["note"] = (f"horizon {T} steps; with several sources the encode and decode run in order on the main "
                    "stream")
    return rows


def bayes_pass(args):
    """Algorithm 1 at 256^3 x 2000: the in-run network (every 10th state at c_start) against a
    network trained on `draws` forward solves at BiLaplacian prior draws about c_start (pointwise
    std 100 m/s, theta = 1e4 m^2), each state's patches kept with probability 1/draws, so both
    training sets hold the same number of vectors; same epochs, batch and schedule."""
    import torch
    import workloads as W
    from paper_2304_04781_amd import _lib as L
    from paper_2304_04781_amd import compressor as C
    from paper_2304_04781_amd.solver import WaveSolver
    L.load()
    dev = torch.device("cuda", 0)
    T, every = args.nt, args.snapshot_every
    p = W.problem_256(T)
    P = (p.nz // 8) * (p.ny // 8) * (p.nx // 8)
    K_exc = int(round(args.exceptions * P))
    c_true = torch.tensor(p.c_true, dtype=torch.float32, device=dev)
    c0 = torch.tensor(p.c_start, dtype=torch.float32, device=dev)
    wav = torch.tensor(p.wavelet, dtype=torch.float32, device=dev)
    s = WaveSolver.for_problem(p)
    s.set_storage(L.STORE_NONE)
    clean, _, _ = s.forward(c_true, wav)
    clean_h = clean.cpu().numpy().astype(np.float64)
    sigma = 0.01 * float(np.abs(clean_h).max())
    d_obs = torch.tensor((clean_h + sigma * p.noise).astype(np.float32), device=dev)
    del clean
    ncap = (T - 1) // every
    nets, info = {}, {}
    net = C.Autoencoder(W.ae_init(2048, 512, 32, seed=4))
    info["in-run"] = C.train_from_forward(s, net, c0, wav, every=every, epochs=args.epochs, batch=args.batch,
                                          perms=device_shuffles(ncap * P, args.epochs, seed=5))
    nets["in-run"] = net
    log(f"in-run training {info['in-run']}")
    theta = (1e4, 1e4, 1e4)
    s.set_prior(1.0, theta, c0)
    probe, _, _ = s.prior_sample(torch.tensor(W.white_noise(p.c_start.shape, 100), dtype=torch.float32, device=dev))
    alpha = float((probe - c0).std()) / 100.0        # a draw scales as 1 / alpha
    del probe
    s.set_prior(alpha, theta, c0)
    draws, cg = [], []
    for i in range(args.draws + 1):
        c, it, rr = s.prior_sample(torch.tensor(W.white_noise(p.c_start.shape, 101 + i), dtype=torch.float32,
                                                device=dev))
        draws.append(c)
        cg.append(it)
    held_out = draws.pop()
    rows = W.keep_rows(args.draws, ncap, P, 1.0 / args.draws, seed=6)
    net = C.Autoencoder(W.ae_init(2048, 512, 32, seed=4))
    y, meta, t_cap = C.prior_draw_samples(s, net, draws, wav, every, rows)
    n = int(y.shape[0])
    info["prior draws"] = dict(C.train_samples(net, y, meta, args.epochs, args.batch,
                                               perms=device_shuffles(n, args.epochs, seed=5)), capture_s=round(t_cap, 2))
    del y, meta
    torch.cuda.empty_cache()
    nets["prior draws"] = net
    log(f"prior-draw training {info['prior draws']}")
    models = {"start": c0, "true": c_true, "mid": 0.5 * (c0 + c_true), "held-out draw": held_out}
    g = s.grid
    lat = torch.empty((P, 32), dtype=torch.int16, device=dev)
    meta = torch.empty((P, 4, 2), dtype=torch.float32, device=dev)
    out = torch.zeros((4,) + s.shape, dtype=torch.float32, device=dev)
    table = {}
    for name, c in models.items():
        _, _, cap = s.forward(c, wav, capture_every=4 * every)
        row = {}
        for label, nt_ in nets.items():
            num = den = 0.0
            for q in range(cap.shape[0]):
                L.ae_encode(nt_.handle, g, cap[q, 0], L.LATENT_BF16, lat, meta)
                L.ae_decode(nt_.handle, g, lat, meta, None, L.LATENT_BF16, 1, out)
                e = cap[q, 0, 0].double()
                num += float(((out[0].double() - e) ** 2).sum())
                den += float((e ** 2).sum())
            row[label] = {"e_rel_err": round((num / den) ** 0.5, 4)}
        del cap
        if name in ("start", "mid"):
            ck = WaveSolver.for_problem(p)
            ck.set_storage(L.STORE_CHECKPOINT, n_checkpoints=args.checkpoints)
            _, gc = ck.gradient(c, wav, d_obs, sigma)
            gc = gc.double()
            ck.close()
            for label, nt_ in nets.items():
                a = WaveSolver.for_problem(p)
                L.wv_set_ae_exceptions(a.ctx, K_exc)
                a.set_storage(L.STORE_AE_BF16, ae=nt_)
                _, ga = a.gradient(c, wav, d_obs, sigma)
                ga = ga.double()
                row[label]["grad_rel_err"] = round(float(torch.linalg.norm(ga - gc) / torch.linalg.norm(gc)), 4)
                row[label]["grad_cos"] = round(float(torch.sum(ga * gc) / torch.linalg.norm(ga) /
                                                     torch.linalg.norm(gc)), 5)
                a.close()
        table[name] = row
        log(f"model {name}: {row}")
    print(json.dumps({"workload": f"{p.name}: compressor trained in-run vs on {args.draws} prior draws",
                      "prior": {"alpha": alpha, "theta_m2": theta[0], "pointwise_std_target": 100.0,
                                "cg_iterations": cg},
                      "training": info, "exceptions": K_exc,
                      "e_error_every_states": 4 * every, "errors": table}), flush=True)


def inversion_pass(args):
    """The analogue of the paper's inversion experiment (speedup and inverse-solution error of
    the compressed path against the uncompressed one): Newton-CG from c_start with the
    BiLaplacian prior (mean c_start), CG preconditioned by the prior covariance, Eisenstat-Walker
    forcing with eta_max 0.5, at most 10 CG iterations per step. The network is trained once on
    snapshots of the forward solve at c_start and kept for every iterate."""
    import torch
    import workloads as W
    from paper_2304_04781_amd import _lib as L
    from paper_2304_04781_amd import compressor as C
    from paper_2304_04781_amd.solver import WaveSolver
    L.load()
    dev = torch.device("cuda", 0)
    T = args.nt
    p = W.problem_256(T)
    P = (p.nz // 8) * (p.ny // 8) * (p.nx // 8)
    K_exc = int(round(args.exceptions * P))
    c_true = torch.tensor(p.c_true, dtype=torch.float32, device=dev)
    c0 = torch.tensor(p.c_start, dtype=torch.float32, device=dev)
    wav = torch.tensor(p.wavelet, dtype=torch.float32, device=dev)
    s = WaveSolver.for_problem(p)
    s.set_storage(L.STORE_NONE)
    clean, _, _ = s.forward(c_true, wav)
    clean_h = clean.cpu().numpy().astype(np.float64)
    sigma = 0.01 * float(np.abs(clean_h).max())
    d_obs = torch.tensor((clean_h + sigma * p.noise).astype(np.float32), device=dev)
    del clean
    net = C.Autoencoder(W.ae_init(2048, 512, 32, seed=4))
    t0 = time.perf_counter()
    if args.inv_store == "space":
        ncap = (T - 1) // args.snapshot_every
        info = C.train_from_forward(s, net, c0, wav, every=args.snapshot_every, epochs=args.epochs,
                                    batch=args.batch, perms=device_shuffles(ncap * P, args.epochs, seed=5))
    else:
        nwin = (T - 1 + L.TWIN - 1) // L.TWIN
        y, meta, _ = C.time_window_samples(s, net, c0, wav, list(range(0, nwin, 4)))
        info = C.train_samples(net, y, None, args.epochs, args.batch,
                               perms=device_shuffles(int(y.shape[0]), args.epochs, seed=5))
        del y, meta
        torch.cuda.empty_cache()
        P = (p.nz // 4) * (p.ny // 4) * (p.nx // 4)    # exception vectors count 4^3 blocks
        K_exc = int(round(args.exceptions * P))
    t_train = time.perf_counter() - t0
    log(f"training {info}")
    alpha, theta = 2e-6, (4 * p.dx * p.dx,) * 3
    e_start = float(torch.linalg.norm(c0 - c_true))
    top = p.nz // 3
    e_start_top = float(torch.linalg.norm((c0 - c_true)[:top]))
    res, models = {}, {}
    for name in ("ae", "checkpoint"):
        sol = WaveSolver.for_problem(p)
        if name == "ae":
            L.wv_set_ae_exceptions(sol.ctx, K_exc)
            sol.set_storage(L.STORE_AE_BF16 if args.inv_store == "space" else L.STORE_AE_TIME, ae=net)
        else:
            sol.set_storage(L.STORE_CHECKPOINT, n_checkpoints=args.checkpoints)
        sol.set_prior(alpha, theta, c0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c, recs, it, reason = sol.newton_cg(c0, wav, d_obs, sigma, max_newton=args.inv_iters, max_cg=10,
                                            eta_max=0.5, gauss_newton=1, precondition=1)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        models[name] = c
        res[name] = {"wall_s": round(wall, 2), "newton_iterations": it, "stop_reason": reason,
                     "hessvec": sum(r["cg_iters"] for r in recs),
                     "gradients": 1 + sum(1 + r["backtracks"] for r in recs[:it]),
                     "cost": [round(r["cost"], 3) for r in recs],
                     "gnorm_ratio": round(recs[-1]["gnorm"] / recs[0]["gnorm"], 5),
                     "model_err_rel": round(float(torch.linalg.norm(c - c_true)) / e_start, 5),
                     "model_err_rel_top_third": round(float(torch.linalg.norm((c - c_true)[:top])) / e_start_top, 5)}
        log(f"{name}: {res[name]}")
        sol.close()
    ca, cc = models["ae"].double(), models["checkpoint"].double()
    store = (f"AE space store (bf16, {K_exc} exact patches per state)" if args.inv_store == "space" else
             f"AE time store (bf16, {K_exc} exact vectors per window)")
    out = {"workload": f"{p.name}: MAP inversion, {args.inv_iters} prior-preconditioned Gauss-Newton CG iterations, "
                       f"{store} vs revolve checkpointing",
           "prior": {"alpha": alpha, "theta_m2": theta[0], "mean": "c_start"},
           "train_s": round(t_train, 2), "results": res,
           "speedup_vs_checkpoint": round(res["checkpoint"]["wall_s"] / res["ae"]["wall_s"], 4),
           "speedup_incl_training": round(res["checkpoint"]["wall_s"] / (res["ae"]["wall_s"] + t_train), 4),
           "model_update_rel_diff": round(float(torch.linalg.norm(ca - cc) / torch.linalg.norm(cc - c0.double())), 5)}
    print(json.dumps(out), flush=True)


def hv384_pass(args):
    """The Gauss-Newton workload: 384^3 x 3000 steps, direction c * GRF(12 cells). Hv with the
    forward and incremental forward states both stored as bf16 latents (1 % exact patches) against
    the checkpointed Hv (64 slots, incremental forward recomputed beside the companion forward).
    The network is trained on every 60th state of the forward solve at c_start."""
    import torch
    import workloads as W
    from paper_2304_04781_amd import _lib as L
    from paper_2304_04781_amd import compressor as C
    from paper_2304_04781_amd.solver import WaveSolver
    L.load()
    dev = torch.device("cuda", 0)
    p = W.problem_384(args.hv_nt)
    T = p.nt
    P = (p.nz // 8) * (p.ny // 8) * (p.nx // 8)
    c = torch.tensor(p.c_start, dtype=torch.float32, device=dev)
    wav = torch.tensor(p.wavelet, dtype=torch.float32, device=dev)
    u = torch.tensor(p.c_start * W.direction_grf(p.c_start.shape, 12.0, 2), dtype=torch.float32, device=dev)
    d = torch.zeros((len(p.src), T, len(p.rec)), dtype=torch.float32, device=dev)
    sigma = 1.0  # the GN Hv depends on the data only through the weight dt / sigma^2
    net = C.Autoencoder(W.ae_init(2048, 512, 32, seed=4))
    s = WaveSolver.for_problem(p)
    s.set_storage(L.STORE_NONE)
    every = 60
    ncap = (T - 1) // every
    info = C.train_from_forward(s, net, c, wav, every=every, epochs=args.hv_epochs, batch=args.batch,
                                perms=device_shuffles(ncap * P, args.hv_epochs, seed=5))
    s.close()
    torch.cuda.empty_cache()
    log(f"training {info}")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed_hv(sol):
        runs, H = [], None
        for _ in range(2):
            torch.cuda.synchronize()
            ev0.record()
            H = sol.hessvec(c, u)
            ev1.record()
            torch.cuda.synchronize()
            runs.append(ev0.elapsed_time(ev1) / 1e3)
        return H, runs

    ck = WaveSolver.for_problem(p)
    ck.set_storage(L.STORE_CHECKPOINT, n_checkpoints=args.checkpoints)
    ck.gradient(c, wav, d, sigma)
    H_ck, runs_ck = timed_hv(ck)
    ck_bytes = ck.storage_bytes()
    ck.close()
    log(f"checkpointed Hv {runs_ck}")
    ae = WaveSolver.for_problem(p)
    L.wv_set_ae_exceptions(ae.ctx, int(round(args.exceptions * P)))
    ae.set_storage(L.STORE_AE_BF16, ae=net)
    ae.set_delta_storage(True)
    ae.gradient(c, wav, d, sigma)
    fwd_bytes = ae.storage_bytes()
    H_ae, runs_ae = timed_hv(ae)
    both_bytes = ae.storage_bytes()
    ae.set_timing(2)
    ae.hessvec(c, u)
    torch.cuda.synchronize()
    kt = {k: (round(us, 1), n) for k, (us, n) in ae.kernel_times().items() if n}
    ae.set_timing(0)
    log(f"AE Hv kernel times (us, launches timed): {kt}")
    ha, hc = H_ae.double(), H_ck.double()
    out = {"workload": f"{p.name}: Gauss-Newton Hv, forward and incremental states as bf16 latents "
                       f"({int(round(args.exceptions * P))} exact patches per state) vs revolve checkpointing "
                       f"({args.checkpoints} slots)",
           "train_s": info["train_s"], "hessvec_ae_s": round(min(runs_ae), 4), "runs_ae_s": [round(x, 4) for x in runs_ae],
           "hessvec_checkpoint_s": round(min(runs_ck), 4), "runs_checkpoint_s": [round(x, 4) for x in runs_ck],
           "speedup_vs_checkpoint": round(min(runs_ck) / min(runs_ae), 4),
           "hv_rel_err_vs_checkpoint": round(float(torch.linalg.norm(ha - hc) / torch.linalg.norm(hc)), 5),
           "hv_cos_vs_checkpoint": round(float(torch.sum(ha * hc) / torch.linalg.norm(ha) / torch.linalg.norm(hc)), 6),
           "store_GB": {"forward": round(fwd_bytes / 1e9, 2), "incremental": round((both_bytes - fwd_bytes) / 1e9, 2),
                        "checkpoints": round(ck_bytes / 1e9, 2)},
           "ae_kernel_us": kt}
    ae.close()
    print(json.dumps(out), flush=True)


def time_pass(args):
    """The time-compression scheme (e on 4^3 blocks x 32 levels) on the 256^3 x 2000 gradient workload."""
    import torch
    import workloads as W
    from paper_2304_04781_amd import _lib as L
    from paper_2304_04781_amd import compressor as C
    from paper_2304_04781_amd.solver import WaveSolver
    L.load()
    dev = torch.device("cuda", 0)
    T = args.nt
    p = W.problem_256(T)
    c_true = torch.tensor(p.c_true, dtype=torch.float32, device=dev)
    c0 = torch.tensor(p.c_start, dtype=torch.float32, device=dev)
    wav = torch.tensor(p.wavelet, dtype=torch.float32, device=dev)
    s = WaveSolver.for_problem(p)
    s.set_storage(L.STORE_NONE)
    clean, _, _ = s.forward(c_true, wav)
    clean_h = clean.cpu().numpy().astype(np.float64)
    sigma = 0.01 * float(np.abs(clean_h).max())
    d_obs = torch.tensor((clean_h + sigma * p.noise).astype(np.float32), device=dev)
    del clean
    nwin = (T - 1 + L.TWIN - 1) // L.TWIN
    windows = list(range(0, nwin, 4))
    net = C.Autoencoder(W.ae_init(2048, 512, 32, seed=4))
    y, meta, t_cap = C.time_window_samples(s, net, c0, wav, windows)
    n = int(y.shape[0])
    info = dict(C.train_samples(net, y, None, args.epochs, args.batch, perms=device_shuffles(n, args.epochs, seed=5)),
                windows=len(windows), capture_s=round(t_cap, 2))
    del y, meta
    torch.cuda.empty_cache()
    log(f"time-network training {info}")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    B = (p.nz // 4) * (p.ny // 4) * (p.nx // 4)
    K_exc = int(round(args.exceptions * B))
    tm = WaveSolver.for_problem(p)
    L.wv_set_ae_exceptions(tm.ctx, K_exc)
    tm.set_storage(L.STORE_AE_TIME, ae=net)
    tm.gradient(c0, wav, d_obs, sigma)
    torch.cuda.synchronize()
    # the timed gradients run with the library's kernel timing off; one more gradient with
    # every launch timed gives the per-kernel means
    times = []
    for _ in range(3):
        ev0.record()
        _, g_t = tm.gradient(c0, wav, d_obs, sigma)
        ev1.record()
        torch.cuda.synchronize()
        times.append(ev0.elapsed_time(ev1) / 1e3)
    tm.set_timing(1)
    tm.gradient(c0, wav, d_obs, sigma)
    kt = {k: (round(us, 1), n) for k, (us, n) in tm.kernel_times().items() if n}
    tm.set_timing(0)
    ck = WaveSolver.for_problem(p)
    ck.set_storage(L.STORE_CHECKPOINT, n_checkpoints=args.checkpoints)
    ck.gradient(c0, wav, d_obs, sigma)
    torch.cuda.synchronize()
    ev0.record()
    _, g_c = ck.gradient(c0, wav, d_obs, sigma)
    ev1.record()
    torch.cuda.synchronize()
    t_ck = ev0.elapsed_time(ev1) / 1e3
    gt, gc = g_t.double(), g_c.double()
    dc = c0 * torch.tensor(0.01 * W.direction_grf((p.nz, p.ny, p.nx), 12.0, seed=2), dtype=torch.float32, device=dev)
    hv = {}
    for name, sol in (("time", tm), ("checkpoint", ck)):
        torch.cuda.synchronize()
        ev0.record()
        H = sol.hessvec(c0, dc)
        ev1.record()
        torch.cuda.synchronize()
        hv[name] = (ev0.elapsed_time(ev1) / 1e3, H.double())
    ht, hc = hv["time"][1], hv["checkpoint"][1]
    out = {"workload": f"{p.name}: time compression (e on 4^3 blocks x {L.TWIN} levels, bf16 latents, "
                       f"{K_exc} exact vectors per window) vs revolve checkpointing ({args.checkpoints} slots)",
           "training": info,
           "gradient_s": {"time": round(float(np.median(times)), 4), "runs": [round(x, 4) for x in times],
                          "checkpoint": round(t_ck, 4)},
           "speedup_vs_checkpoint": round(t_ck / float(np.median(times)), 4),
           "grad_rel_err_vs_checkpoint": round(float(torch.linalg.norm(gt - gc) / torch.linalg.norm(gc)), 5),
           "grad_cos": round(float(torch.sum(gt * gc) / torch.linalg.norm(gt) / torch.linalg.norm(gc)), 6),
           "gn_hessvec_s": {"time": round(hv["time"][0], 4), "checkpoint": round(hv["checkpoint"][0], 4)},
           "hessvec_speedup_vs_checkpoint": round(hv["checkpoint"][0] / hv["time"][0], 4),
           "hv_rel_err_vs_checkpoint": round(float(torch.linalg.norm(ht - hc) / torch.linalg.norm(hc)), 5),
           "store_GB": round(tm.storage_bytes() / 1e9, 3),
           "kernel_times_us": kt,
           "note": "encode per window of 32 levels (timing class 3), decode per window (class 4)"}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.counters:
        counters_pass()
        return
    if args.multisource:
        multisource_pass(args)
        return
    if args.bayes:
        bayes_pass(args)
        return
    if args.time:
        time_pass(args)
        return
    if args.inversion:
        inversion_pass(args)
        return
    if args.hv384:
        hv384_pass(args)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the compressed gradient runs on a single MI355X; "
              "sharding by source or by domain is not implemented",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2304_04781_amd import _lib as L
    from paper_2304_04781_amd.solver import WaveSolver

    L.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t_setup = time.perf_counter()

    n, T = args.size, args.nt
    p = W.problem_256(T) if n == 256 else W.problem_3d(n, n, n, T, rec_first=33, rec_step=max(1, (n - 66) // 64),
                                                          rec_count=64, name=f"3d-{n}^3-{T}")
    N = p.n
    P = (p.nz // 8) * (p.ny // 8) * (p.nx // 8)
    K_exc = int(round(args.exceptions * P))
    log(f"problem {p.name}: N={N}, P={P}, dt={p.dt:.3e}, receivers={len(p.rec)}, exceptions={K_exc}")
    c_true = torch.tensor(p.c_true, dtype=torch.float32, device=dev)
    c0 = torch.tensor(p.c_start, dtype=torch.float32, device=dev)
    wav = torch.tensor(p.wavelet, dtype=torch.float32, device=dev)

    solver = WaveSolver.for_problem(p)
    solver.set_storage(L.STORE_NONE)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    # observations: forward at the true model (also the forward-stencil timing run)
    clean, _, _ = solver.forward(c_true, wav)
    torch.cuda.synchronize()
    ev0.record()
    clean, _, _ = solver.forward(c_true, wav)
    ev1.record()
    torch.cuda.synchronize()
    t_fwd_step = ev0.elapsed_time(ev1) / 1e3 / T
    clean_h = clean.cpu().numpy().astype(np.float64)
    sigma = 0.01 * float(np.abs(clean_h).max())
    d_obs = torch.tensor((clean_h + sigma * p.noise).astype(np.float32), device=dev)
    del clean
    log(f"forward stencil {t_fwd_step * 1e6:.1f} us/step")

    # ---- train the compressor on snapshots of the first forward solve at c_start
    from paper_2304_04781_amd.compressor import Autoencoder, train_from_forward
    t0 = time.perf_counter()
    net = Autoencoder(W.ae_init(2048, 512, 32, seed=4))
    nsamp = ((T - 1) // args.snapshot_every) * P * len(p.src)
    perms = device_shuffles(nsamp, args.epochs, seed=5)
    train_info = train_from_forward(solver, net, c0, wav, every=args.snapshot_every, epochs=args.epochs,
                                    batch=args.batch, perms=perms, weighting=args.weighting)
    del perms
    t_train_total = time.perf_counter() - t0
    log(f"training {train_info}")

    # ---- AE-compressed gradient (timed)
    fmt = L.STORE_AE_BF16 if args.latent == "bf16" else L.STORE_AE_FP8
    ae_solver = WaveSolver.for_problem(p)
    L.wv_set_ae_exceptions(ae_solver.ctx, K_exc)
    ae_solver.set_storage(fmt, ae=net)
    for _ in range(args.warmup):
        ae_solver.gradient(c0, wav, d_obs, sigma)
    torch.cuda.synchronize()
    # the timed gradients run with the library's kernel timing off
    times = []
    g_ae = None
    for _ in range(args.steps):
        torch.cuda.synchronize()
        ev0.record()
        J_ae, g_ae = ae_solver.gradient(c0, wav, d_obs, sigma)
        ev1.record()
        torch.cuda.synchronize()
        times.append(ev0.elapsed_time(ev1) / 1e3)
    t_ae = float(np.median(times))
    # per-kernel durations from one more gradient: HIP events around every 4th launch of
    # each kernel class, on the stream that runs it
    kt_ae = timed_kernels(ae_solver, c0, wav, d_obs, sigma)
    status = ae_solver.last_status
    store_bytes = ae_solver.storage_bytes()
    log(f"AE gradient {t_ae:.3f} s (runs {['%.3f' % x for x in times]}), store {store_bytes / 1e9:.2f} GB")
    log(f"AE kernel times (us, launches timed): {kt_ae}")

    # ---- checkpointed gradient (the plain path: fallback and judge)
    ck = WaveSolver.for_problem(p)
    ck.set_storage(L.STORE_CHECKPOINT, n_checkpoints=args.checkpoints)
    J_ck, g_ck = ck.gradient(c0, wav, d_obs, sigma)
    torch.cuda.synchronize()
    nrep = max(1, min(args.steps, 5))   # 5 timed runs of each reference path (1 warm-up above)
    times_ck = []
    for _ in range(nrep):
        torch.cuda.synchronize()
        ev0.record()
        J_ck, g_ck = ck.gradient(c0, wav, d_obs, sigma)
        ev1.record()
        torch.cuda.synchronize()
        times_ck.append(ev0.elapsed_time(ev1) / 1e3)
    t_ck = float(np.median(times_ck))
    kt_ck = timed_kernels(ck, c0, wav, d_obs, sigma)
    fsteps, _, _ = ck.stats()
    ck_bytes = ck.storage_bytes()
    log(f"checkpointed gradient {t_ck:.3f} s, {fsteps} forward steps; kernel times {kt_ck}")

    # ---- Gauss-Newton Hv at the same model: the AE path decodes the stored states, the
    # checkpointed path recomputes the forward alongside the incremental forward and in
    # the revolve reverse sweep (direction: c times a GRF of correlation length 12 cells)
    dc = c0 * torch.tensor(0.01 * W.direction_grf((p.nz, p.ny, p.nx), 12.0, seed=2), dtype=torch.float32,
                           device=dev)
    hv = {}
    for name, sol in (("ae", ae_solver), ("checkpoint", ck)):  # both hold the last gradient's c0
        runs = []
        for _ in range(nrep):
            torch.cuda.synchronize()
            ev0.record()
            Hv = sol.hessvec(c0, dc)
            ev1.record()
            torch.cuda.synchronize()
            runs.append(ev0.elapsed_time(ev1) / 1e3)
        hv[name] = (float(np.median(runs)), Hv.double(), runs)
    h_ae, h_ck = hv["ae"][1], hv["checkpoint"][1]
    hessvec = {"ae_s": round(hv["ae"][0], 4), "checkpoint_s": round(hv["checkpoint"][0], 4),
               "runs_s": {k: [round(x, 4) for x in hv[k][2]] for k in hv},
               "min_s": {k: round(min(hv[k][2]), 4) for k in hv},
               "speedup_vs_checkpoint": round(hv["checkpoint"][0] / hv["ae"][0], 4),
               "rel_err_vs_checkpoint_fp32": round(float(torch.linalg.norm(h_ae - h_ck) / torch.linalg.norm(h_ck)), 5),
               "cos_vs_checkpoint_fp32": round(float(torch.sum(h_ae * h_ck) / (torch.linalg.norm(h_ae) *
                                                                              torch.linalg.norm(h_ck))), 6)}
    # full-Newton Hv at the same model: only a stored history supports it at this size (the float32
    # history would take 537 GB), so the AE path runs alone; it re-runs the adjoint mu beside the
    # incremental adjoint and stores the incremental states in a second latent store
    torch.cuda.synchronize()
    ev0.record()
    Hf = ae_solver.hessvec(c0, dc, gauss_newton=False)
    ev1.record()
    torch.cuda.synchronize()
    hessvec["full_newton_ae_s"] = round(ev0.elapsed_time(ev1) / 1e3, 4)
    hessvec["full_newton_vs_gn_rel_diff"] = round(float(torch.linalg.norm(Hf.double() - h_ae) /
                                                        torch.linalg.norm(h_ae)), 5)
    hessvec["store_with_incremental_GB"] = round(ae_solver.storage_bytes() / 1e9, 3)
    del hv
    log(f"GN Hv: {hessvec}")

    # ---- the paper's method as published: latents only, no exact patches (K = 0), same network
    k0 = WaveSolver.for_problem(p)
    k0.set_storage(fmt, ae=net)
    k0.gradient(c0, wav, d_obs, sigma)
    runs0 = []
    for _ in range(nrep):
        torch.cuda.synchronize()
        ev0.record()
        _, g0 = k0.gradient(c0, wav, d_obs, sigma)
        ev1.record()
        torch.cuda.synchronize()
        runs0.append(ev0.elapsed_time(ev1) / 1e3)
    H0 = k0.hessvec(c0, dc).double()
    g0d, gckd = g0.double(), g_ck.double()
    latents_only = {
        "exact_patches_per_state": 0, "gradient_s": round(float(np.median(runs0)), 4),
        "gradient_runs_s": [round(x, 4) for x in runs0],
        "speedup_vs_checkpoint": round(t_ck / float(np.median(runs0)), 4),
        "grad_rel_err_vs_checkpoint_fp32": round(float(torch.linalg.norm(g0d - gckd) / torch.linalg.norm(gckd)), 5),
        "grad_cos_vs_checkpoint_fp32": round(float(torch.sum(g0d * gckd) / torch.linalg.norm(g0d) /
                                                   torch.linalg.norm(gckd)), 6),
        "hv_rel_err_vs_checkpoint_fp32": round(float(torch.linalg.norm(H0 - h_ck) / torch.linalg.norm(h_ck)), 5),
        "hv_cos_vs_checkpoint_fp32": round(float(torch.sum(H0 * h_ck) / torch.linalg.norm(H0) /
                                                 torch.linalg.norm(h_ck)), 6),
        "store_GB": round(k0.storage_bytes() / 1e9, 3)}
    k0.close()
    del g0, H0, g0d, gckd, h_ae
    log(f"latents only (K = 0): {latents_only}")

    # ---- the time-compression scheme on the same workload (e on 4^3 blocks x 32 levels,
    # 1 % exact vectors per window), against the same checkpointed gradient and Hv
    time_scheme = None
    if not args.no_time:
        time_scheme = time_leg(args, p, solver, c0, wav, d_obs, sigma, g_ck, h_ck, dc, t_ck, hessvec["checkpoint_s"],
                               Hf)
        log(f"time compression: {time_scheme}")
    del h_ck, dc, Hf

    # ---- one Newton-CG iteration for the MAP point (BiLaplacian prior): a gradient, newton_cg Hv
    # products in CG and the accepted trial's gradient; the AE store is written once per iterate
    # and decompressed in every Hv, checkpointing recomputes the forward in each of them
    newton = None
    if not args.no_newton:
        newton = newton_iteration(args, p, ae_solver, ck, c0, wav, d_obs, sigma)
        log(f"Newton iteration: {newton}")

    ga = g_ae.double()
    gc = g_ck.double()
    rel_err = float(torch.linalg.norm(ga - gc) / torch.linalg.norm(gc))
    cos = float(torch.sum(ga * gc) / (torch.linalg.norm(ga) * torch.linalg.norm(gc)))
    log(f"grad rel err {rel_err:.4f} cos {cos:.5f}")

    copy_gbs = copy_peak_gbs(torch, dev)
    gemm_tf = gemm_peak_tflops(torch, dev)
    probe = stream_ceilings(torch, dev, N)
    log(f"library bf16 GEMM {gemm_tf:.0f} TFLOP/s")
    log(f"device copy {copy_gbs:.0f} GB/s; streaming probe {probe}")

    # ---- rooflines: algorithmic bytes (flops) per launch over the measured mean launch duration
    per_launch = {
        "forward_stencil": ("hbm", 36.0 * N),                          # read 4 fields + m, write 4 fields
        "adjoint_stencil": ("hbm", adjoint_bytes_per_cell(T, L.wv_accumulation_block()) * N),
        "encode": ("mfma", 2.0 * P * (2048 * 512 + 512 * 32)),         # two encoder layers
        "decode_e": ("mfma", 2.0 * P * (32 * 512 + 512 * 512)),        # decoder layer 3 + e rows of layer 4
    }
    launches = {"forward_stencil": T, "adjoint_stencil": T - 1, "encode": T - 1, "decode_e": T - 1,
                "exceptions_select": T - 1, "exceptions_restore": T - 1, "exceptions_gather": T - 1}
    kernels = {}
    for name, (us, n) in kt_ae.items():
        if n == 0:
            continue
        row = {"us": us, "timed_launches": n, "ms_per_gradient": us * launches.get(name, 0) / 1e3}
        if name in per_launch:
            bound, work = per_launch[name]
            if bound == "hbm":
                row["GB/s"] = work / (us * 1e-6) / 1e9
                row["frac_hbm"] = row["GB/s"] / HBM_PEAK_GBS
            else:
                row["TFLOP/s"] = work / (us * 1e-6) / 1e12
                row["frac_mfma_bf16"] = row["TFLOP/s"] / BF16_PEAK_TFLOPS
                row["frac_of_library_gemm"] = row["TFLOP/s"] / gemm_tf
        kernels[name] = row
    # dominant kernel: the main-stream (critical-path) kernel with the most time per gradient; the
    # encode and decode run on side streams beside the stencil steps, so their event time overlaps
    dom = max((k for k in kernels if k in ("forward_stencil", "adjoint_stencil")),
              key=lambda k: kernels[k]["ms_per_gradient"])
    bound, work = per_launch[dom]
    if bound == "hbm":
        roofline = {"kernel": dom, "bound": "hbm", "achieved": round(kernels[dom]["GB/s"], 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(kernels[dom]["frac_hbm"], 4),
                    "measured_copy_GBps": round(copy_gbs, 1),
                    "frac_of_copy": round(kernels[dom]["GB/s"] / copy_gbs, 4),
                    "frac_of_streaming_mix": round(kernels[dom]["GB/s"] / probe[
                        "adjoint_mix_7in_5out" if dom == "adjoint_stencil" else "forward_mix_5in_4out"], 4),
                    "traffic": measured_traffic(dom), "mean_launch_us": round(kernels[dom]["us"], 2),
                    "algorithmic_bytes_per_launch": work}
        if dom == "forward_stencil" and "encode" in kernels:
            # context: during each forward step the side stream's encode reads the state the previous
            # step wrote and writes its latents and (lo, r) pairs, so the HBM moved in the step's
            # interval is both kernels' bytes (the exception selection and copy are small beside them)
            enc = 16.0 * N + P * (32 * 2 + 8 * 4)
            step = work + enc
            gbs = step / (kernels[dom]["us"] * 1e-6) / 1e9
            roofline["with_side_stream"] = {"kernels": "forward_stencil + encode (side stream)",
                                            "bytes_per_step": step, "achieved": round(gbs, 1),
                                            "frac": round(gbs / HBM_PEAK_GBS, 4),
                                            "frac_of_copy": round(gbs / copy_gbs, 4)}
    else:
        roofline = {"kernel": dom, "bound": "mfma", "achieved": round(kernels[dom]["TFLOP/s"], 1),
                    "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(kernels[dom]["frac_mfma_bf16"], 4),
                    "traffic": None, "mean_launch_us": round(kernels[dom]["us"], 2),
                    "algorithmic_flops_per_launch": work}

    # ---- CPU baseline: the FP64 oracle on a bounded sample of the same grid
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(p, T)
        log(f"cpu baseline {cpu}")

    gph = 3600.0 / t_ae
    out = {
        "metric": "gradients/hour at 256^3x2000 steps, AE vs checkpointing; grad rel err vs FP64",
        "value": round(gph, 1),
        "unit": "gradients/hour",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_ae * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16",
        "data": "synthetic",
        "config": {"workload": f"{p.name}: AE-compressed misfit gradient ({args.latent} latents, "
                               f"{K_exc} exact patches/step) vs revolve checkpointing ({args.checkpoints} slots)",
                   "grid": [p.nz, p.ny, p.nx], "nt": T, "sources": len(p.src), "receivers": len(p.rec),
                   "global_batch": 1},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "checkpoint": {"gradients_per_hour": round(3600.0 / t_ck, 1), "ms_per_gradient": round(t_ck * 1e3, 2),
                       "forward_steps": fsteps, "store_GB": round(ck_bytes / 1e9, 2)},
        "speedup_vs_checkpoint": round(t_ck / t_ae, 4),
        "gradient_runs_s": {"ae": [round(x, 4) for x in times], "ae_min": round(min(times), 4),
                            "checkpoint": [round(x, 4) for x in times_ck], "checkpoint_min": round(min(times_ck), 4)},
        "gn_hessvec": hessvec,
        "latents_only": latents_only,
        "time_compression": time_scheme,
        "newton_iteration": newton,
        "grad_rel_err_vs_checkpoint_fp32": round(rel_err, 5),
        "grad_cos_vs_checkpoint_fp32": round(cos, 6),
        "misfit": {"ae": J_ae, "checkpoint": J_ck},
        "status": int(status),
        "ae_store_GB": round(store_bytes / 1e9, 3),
        "compression": {"latent_only": 2048 * 4 / (32 * (2 if args.latent == "bf16" else 1)),
                        "effective_vs_float32_history": round(4.0 * 4 * N * (T - 1) / store_bytes, 1)},
        "train": dict(train_info, wall_s=round(t_train_total, 2), weighting=args.weighting),
        "kernels": {k: {kk: round(vv, 4) for kk, vv in v.items()} for k, v in kernels.items()},
        "measured_peaks": {"device_copy_GBps": round(copy_gbs, 1), "library_bf16_gemm_TFLOPs": round(gemm_tf, 1),
                           "streaming_probe_GBps": probe},
        # the same stencil kernels with the GPU to themselves (no encode or decode beside them)
        "checkpoint_kernels": {k: dict({"us": round(us, 2), "timed_launches": n},
                                       **({"GB/s": round(per_launch[k][1] / (us * 1e-6) / 1e9, 1),
                                           "frac_hbm": round(per_launch[k][1] / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                                           "frac_of_streaming_mix": round(per_launch[k][1] / (us * 1e-6) / 1e9 / probe[
                                               "adjoint_mix_7in_5out" if k == "adjoint_stencil"
                                               else "forward_mix_5in_4out"], 4)}
                                          if k in per_launch and per_launch[k][0] == "hbm" else {}))
                               for k, (us, n) in kt_ck.items() if n},
        "first_gradient_s": round(t_train_total + t_ae, 3),
        "amortized_over_10_gradients_s": round((t_train_total + 10 * t_ae) / 10, 4),
        "setup_s": round(time.perf_counter() - t_setup, 1),
    }
    print(json.dumps(out), flush=True)


def time_leg(args, p, solver, c0, wav, d_obs, sigma, g_ck, h_ck, dc, t_ck, hv_ck_s, hf_space):
    """Time-compression scheme: network trained on every 4th window of the forward solve at
    c0 (the solver's own states), then timed gradients, one Gauss-Newton Hv and one
    full-Newton Hv (its incremental states compressed by the same network; no uncompressed
    reference exists at this size, so it is compared with the space scheme's)."""
    import torch
    import workloads as W
    from paper_2304_04781_amd import _lib as L
    from paper_2304_04781_amd import compressor as C
    from paper_2304_04781_amd.solver import WaveSolver
    T = p.nt
    nwin = (T - 1 + L.TWIN - 1) // L.TWIN
    net = C.Autoencoder(W.ae_init(2048, 512, 32, seed=4))
    y, meta, _ = C.time_window_samples(solver, net, c0, wav, list(range(0, nwin, 4)))
    info = C.train_samples(net, y, None, args.epochs, args.batch, perms=device_shuffles(int(y.shape[0]), args.epochs, seed=5))
    del y, meta
    torch.cuda.empty_cache()
    B = (p.nz // 4) * (p.ny // 4) * (p.nx // 4)
    K = int(round(args.exceptions * B))
    tm = WaveSolver.for_problem(p)
    L.wv_set_ae_exceptions(tm.ctx, K)
    tm.set_storage(L.STORE_AE_TIME, ae=net)
    tm.gradient(c0, wav, d_obs, sigma)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        ev0.record()
        _, g = tm.gradient(c0, wav, d_obs, sigma)
        ev1.record()
        torch.cuda.synchronize()
        times.append(ev0.elapsed_time(ev1) / 1e3)
    gt, gc = g.double(), g_ck.double()
    torch.cuda.synchronize()
    ev0.record()
    H = tm.hessvec(c0, dc)
    ev1.record()
    torch.cuda.synchronize()
    t_hv = ev0.elapsed_time(ev1) / 1e3
    ht, hc = H.double(), h_ck
    store_bytes = tm.storage_bytes()
    torch.cuda.synchronize()
    ev0.record()
    Hf = tm.hessvec(c0, dc, gauss_newton=False)
    ev1.record()
    torch.cuda.synchronize()
    t_hf = ev0.elapsed_time(ev1) / 1e3
    hf, hs = Hf.double(), hf_space.double()
    t_g = float(np.median(times))
    out = {"exact_vectors_per_window": K, "train_s": info["train_s"],
           "gradient_s": round(t_g, 4), "gradient_runs_s": [round(x, 4) for x in times],
           "gradient_min_s": round(min(times), 4),
           "gradients_per_hour": round(3600.0 / t_g, 1), "speedup_vs_checkpoint": round(t_ck / t_g, 4),
           "grad_rel_err_vs_checkpoint_fp32": round(float(torch.linalg.norm(gt - gc) / torch.linalg.norm(gc)), 5),
           "grad_cos_vs_checkpoint_fp32": round(float(torch.sum(gt * gc) / torch.linalg.norm(gt) /
                                                      torch.linalg.norm(gc)), 6),
           "gn_hessvec_s": round(t_hv, 4), "hessvec_speedup_vs_checkpoint": round(hv_ck_s / t_hv, 4),
           "hv_rel_err_vs_checkpoint_fp32": round(float(torch.linalg.norm(ht - hc) / torch.linalg.norm(hc)), 5),
           "full_newton_s": round(t_hf, 4),
           "full_newton_rel_diff_vs_space_ae": round(float(torch.linalg.norm(hf - hs) / torch.linalg.norm(hs)), 5),
           "store_GB": round(store_bytes / 1e9, 3),
           "store_with_incremental_GB": round(tm.storage_bytes() / 1e9, 3)}
    tm.close()
    return out


def newton_iteration(args, p, ae_solver, ck, c0, wav, d_obs, sigma):
    """Wall time of one Gauss-Newton CG iteration (prior-preconditioned, eta tiny, so
    CG runs its newton_cg iterations) with the AE store and with checkpointing, from
    the same start model; the two updates are compared."""
    import torch
    alpha, theta = 2e-6, (4 * p.dx * p.dx,) * 3
    res = {"max_cg": args.newton_cg, "preconditioner": "prior covariance",
           "prior": {"alpha": alpha, "theta_m2": theta[0]}}
    upd = {}
    for name, sol in (("ae", ae_solver), ("checkpoint", ck)):
        sol.set_prior(alpha, theta, c0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c1, recs, it, reason = sol.newton_cg(c0, wav, d_obs, sigma, max_newton=1, max_cg=args.newton_cg,
                                             eta_max=1e-6, gauss_newton=1, precondition=1)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        r0 = recs[0]
        res[name] = {"wall_s": round(wall, 3), "hessvec": r0["cg_iters"], "gradients": 1 + 1 + r0["backtracks"],
                     "step": r0["step"], "cost": [round(r["cost"], 4) for r in recs],
                     "gnorm_ratio": round(recs[-1]["gnorm"] / r0["gnorm"], 5)}
        upd[name] = (c1 - c0).double()
        sol.set_prior(0.0)
    res["speedup_vs_checkpoint"] = round(res["checkpoint"]["wall_s"] / res["ae"]["wall_s"], 4)
    res["update_rel_err_vs_checkpoint"] = round(float(torch.linalg.norm(upd["ae"] - upd["checkpoint"]) /
                                                      torch.linalg.norm(upd["checkpoint"])), 5)
    return res


def adjoint_bytes_per_cell(T, block):
    """Mean algorithmic bytes per cell of the T-1 adjoint steps: 40 B of fields
    (read eta, mu_z, mu_y, mu_x, m, e^k; write eta, mu_z, mu_y, mu_x) plus the
    gradient accumulation of the step's phase in its block of `block` steps: the
    float32 partial written (first), read and written (middle), read with the
    compensated pair read and written (last), or the pair alone (a one-step block)."""
    total = 0.0
    steps = T - 1
    for j in range(steps):
        first, last = j % block == 0, j % block == block - 1 or j == steps - 1
        total += 40.0 + (16.0 if first and last else 4.0 if first else 20.0 if last else 8.0)
    return total / max(steps, 1)


def cpu_baseline(p, T, nsteps=20):
    """Time the FP64 oracle's forward and adjoint steps on the full grid and
    extrapolate to one gradient (T forward + T-1 adjoint steps)."""
    from oracle import wave as ow
    sol = ow.solver_for(p)
    m = p.c_start * p.c_start
    rng = np.random.default_rng(0)
    v = {a: 1e-6 * rng.standard_normal(sol.shape) for a in sol.axes}
    e = 1e-6 * rng.standard_normal(sol.shape)
    t0 = time.perf_counter()
    for n in range(nsteps):
        v, e = sol.step(v, e, m, force=(tuple(int(x) for x in p.src[0]), p.wavelet[0, n], p.src_w))
    t_f = (time.perf_counter() - t0) / nsteps
    mu = {a: x.copy() for a, x in v.items()}
    eta = e.copy()
    acc = np.zeros(sol.shape)
    t0 = time.perf_counter()
    for n in range(nsteps):
        mu, eta, q = sol.step_T(mu, eta, m)
        acc += e * q
    t_a = (time.perf_counter() - t0) / nsteps
    t_grad = T * t_f + (T - 1) * t_a
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"value": round(3600.0 / t_grad, 4), "unit": "gradients/hour", "cores": 1, "kind": "oracle",
            "host_cores": os.cpu_count(), "host_cores_usable": affinity,
            "sample": f"{nsteps} forward + {nsteps} adjoint FP64 numpy steps on the {p.nz}x{p.ny}x{p.nx} grid "
                      f"({t_f:.2f} s + {t_a:.2f} s per step), extrapolated to {T} + {T - 1} steps"}


if __name__ == "__main__":
    main()
