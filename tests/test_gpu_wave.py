"""GPU parity of the plain (uncompressed) path against the FP64 oracle.

Inputs are the seeded workloads rounded to float32; the oracle runs on the
same rounded values in float64, so differences are the kernels' FP32
arithmetic only. Tolerances: forward states and traces 1e-5 relative L2,
gradient and Hv 1e-4 relative L2 (float32 leapfrog over a few hundred
steps stays near 1e-6; the adjoint accumulation is Kahan-compensated)."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import wave as ow
from paper_2304_04781_amd import _lib as L
from paper_2304_04781_amd.solver import WaveSolver

pytestmark = pytest.mark.gpu


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rounded(p):
    """The problem with every array input rounded to float32."""
    p.c_true = f32(p.c_true)
    p.c_start = f32(p.c_start)
    p.wavelet = f32(p.wavelet)
    return p


def small3d(nt=300, shape=(40, 36, 70), sponge=6, nsrc=1):
    p = W.problem_3d(*shape, nt, f0=15.0, sponge=sponge, name="ragged3d")
    if nsrc == 2:
        p.src = np.array([[4, 18, 35], [6, 12, 50]], dtype=np.int32)
        p.wavelet = np.stack([p.wavelet[0], 0.6 * W.ricker(11.0, p.dt, nt) / p.dx ** 3])
        p.noise = np.random.default_rng(1).standard_normal((2, nt, len(p.rec)))
    return rounded(p)


def oracle_data(p):
    sol = ow.solver_for(p)
    d, sigma, _ = ow.observed_data(sol, p)
    return sol, f32(d), sigma


def solver_for(p, mode=L.STORE_FULL, nslots=16):
    s = WaveSolver.for_problem(p)
    s.set_storage(mode, n_checkpoints=nslots)
    return s


# ----- forward ---------------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["2d", "3d"])
def test_forward_states_and_traces(which):
    p = rounded(W.problem_2d_small()) if which == "2d" else small3d()
    print("case", which, p.name, flush=True)
    sol = ow.solver_for(p)
    tr_o, e_hist, finals, v_hist = ow.forward(sol, p.c_start, p.wavelet, p.src, p.rec, store_v=True, src_w=p.src_w)
    s = solver_for(p, L.STORE_NONE)
    tr, fin, cap = s.forward(p.c_start, p.wavelet, final_state=True, capture_every=1)
    torch.cuda.synchronize()
    cap = cap.cpu().numpy()          # [T-1, S, 4, nz, ny, nx]
    assert rel(tr.cpu().numpy(), tr_o) < 1e-5
    # all stored states: e and every velocity field
    fields = {0: e_hist[0, 1:p.nt]}
    axes_map = {0: 1, 1: 2, 2: 3}
    for a in sol.axes:
        fields[axes_map[a]] = np.stack([v_hist[0][n][a] for n in range(p.nt - 1)])
    for f, ref in fields.items():
        assert rel(cap[:, 0, f], ref) < 1e-5, f
    if p.ny == 1:
        assert np.all(cap[:, 0, 2] == 0.0)           # no y velocity in 2D
    fin = fin.cpu().numpy()
    assert rel(fin[0, 0], finals[0][1]) < 1e-5


# ----- gradient ---------------------------------------------------------------------------------
@pytest.mark.parametrize("which,mode", [("2d", L.STORE_FULL), ("3d", L.STORE_FULL),
                                        ("3d", L.STORE_CHECKPOINT), ("2d", L.STORE_CHECKPOINT)])
def test_gradient_matches_oracle(which, mode):
    p = rounded(W.problem_2d_small()) if which == "2d" else small3d()
    print("case", which, mode, flush=True)
    sol, d, sigma = oracle_data(p)
    J_o, g_o, _, _ = ow.gradient(sol, p.c_start, p.wavelet, p.src, p.rec, d, sigma, src_w=p.src_w)
    s = solver_for(p, mode, nslots=8)
    J, g = s.gradient(p.c_start, p.wavelet, d, sigma)
    g = g.cpu().numpy()
    assert abs(J - J_o) / J_o < 1e-5
    assert rel(g, g_o) < 1e-4
    cos = float(np.sum(g * g_o) / (np.linalg.norm(g) * np.linalg.norm(g_o)))
    assert cos > 0.9999999
    if mode == L.STORE_CHECKPOINT:
        from oracle import revolve as orv
        steps, _, _ = s.stats()
        assert steps == orv.closed_form(p.nt, 8) + 1


def test_receivers_at_depth_chunk_edges_and_shared_cells():
    """Receivers inside the volume: on the z-chunk edges (8-level chunks here), on
    the tile edges in y and x, at the first and last levels, and several on one cell.
    Traces, incremental traces and the gradient (whose residual injection sums the
    receivers sharing a cell) against the oracle."""
    p = small3d(nt=160)
    rec = []
    for q, k in enumerate([0, 2, 7, 8, 15, 16, 23, 24, 31, 32, 39]):
        for j, i in ((7, 63), (8, 64), (3 + q, 10 + 5 * q), (35, 69)):
            rec.append((k, j, i))
    rec += [(8, 8, 64), (8, 8, 64), (20, 17, 33), (20, 17, 33), (20, 17, 33)]
    p.rec = np.asarray(rec, dtype=np.int32)
    p.noise = np.random.default_rng(7).standard_normal((1, p.nt, len(rec)))
    print("case receivers", len(rec), flush=True)
    sol, d, sigma = oracle_data(p)
    tr_o, e_hist, _, _ = ow.forward(sol, p.c_start, p.wavelet, p.src, p.rec, src_w=p.src_w)
    J_o, g_o, _, _ = ow.gradient(sol, p.c_start, p.wavelet, p.src, p.rec, d, sigma, src_w=p.src_w)
    s = solver_for(p, L.STORE_FULL)
    tr = s.forward(p.c_start, p.wavelet)[0].cpu().numpy()
    assert rel(tr, tr_o) < 1e-5
    J, g = s.gradient(p.c_start, p.wavelet, d, sigma)
    assert abs(J - J_o) / J_o < 1e-5
    assert rel(g.cpu().numpy(), g_o) < 1e-4
    dc = f32(p.c_start * 0.01 * W.direction_grf(p.c_start.shape, 6.0, 2))
    dp_o, _ = ow.inc_forward(sol, p.c_start, dc, e_hist[0], p.rec)
    dp = s.inc_forward(p.c_start, dc).cpu().numpy()
    assert rel(dp[0], dp_o) < 1e-5


def test_checkpoint_gradient_bitwise_equals_full_storage():
    p = small3d(nt=200)
    sol, d, sigma = oracle_data(p)
    out = []
    for mode, ns in ((L.STORE_FULL, 0), (L.STORE_CHECKPOINT, 5), (L.STORE_CHECKPOINT, 1)):
        s = solver_for(p, mode, nslots=max(ns, 1))
        J, g = s.gradient(p.c_start, p.wavelet, d, sigma)
        out.append((J, g.cpu().numpy()))
    for J, g in out[1:]:
        assert J == out[0][0]
        assert np.array_equal(g, out[0][1])


def test_gradient_multisource():
    p = small3d(nt=250, nsrc=2)
    sol, d, sigma = oracle_data(p)
    J_o, g_o, _, _ = ow.gradient(sol, p.c_start, p.wavelet, p.src, p.rec, d, sigma, src_w=p.src_w)
    s = solver_for(p, L.STORE_FULL)
    J, g = s.gradient(p.c_start, p.wavelet, d, sigma)
    assert abs(J - J_o) / J_o < 1e-5
    assert rel(g.cpu().numpy(), g_o) < 1e-4


def test_gradient_deterministic():
    p = small3d(nt=150)
    sol, d, sigma = oracle_data(p)
    s = solver_for(p, L.STORE_FULL)
    J1, g1 = s.gradient(p.c_start, p.wavelet, d, sigma)
    J2, g2 = s.gradient(p.c_start, p.wavelet, d, sigma)
    assert J1 == J2 and torch.equal(g1, g2)


def test_zero_residual_gives_zero_gradient():
    p = small3d(nt=120)
    s = solver_for(p, L.STORE_FULL)
    tr, _, _ = s.forward(p.c_start, p.wavelet)
    J, g = s.gradient(p.c_start, p.wavelet, tr, 1.0)
    assert J == 0.0 and torch.count_nonzero(g).item() == 0


# ----- linearisation, adjoint identity and Hv --------------------------------------------------
def test_inc_forward_and_jacobian_dot_test():
    p = small3d(nt=200)
    sol = ow.solver_for(p)
    _, e_hist, _, _ = ow.forward(sol, p.c_start, p.wavelet, p.src, p.rec, src_w=p.src_w)
    rng = np.random.default_rng(3)
    dc = f32(p.c_start * 0.01 * W.direction_grf(p.c_start.shape, 6.0, 2))
    w = f32(rng.standard_normal((1, p.nt, len(p.rec))))
    dp_o, _ = ow.inc_forward(sol, p.c_start, dc, e_hist[0], p.rec)
    s = solver_for(p, L.STORE_FULL)
    s.forward(p.c_start, p.wavelet)
    dp = s.inc_forward(p.c_start, dc).cpu().numpy()
    assert rel(dp[0], dp_o) < 1e-5
    JTw = s.adjoint(p.c_start, w).cpu().numpy()
    lhs = float(np.sum(dp.astype(np.float64) * w))
    rhs = float(np.sum(dc * JTw.astype(np.float64)))
    assert abs(lhs - rhs) / abs(lhs) < 1e-4


@pytest.mark.parametrize("mode", [L.STORE_FULL, L.STORE_CHECKPOINT])
def test_gn_hessvec_matches_oracle(mode):
    p = small3d(nt=200)
    sol, d, sigma = oracle_data(p)
    _, e_hist, _, _ = ow.forward(sol, p.c_start, p.wavelet, p.src, p.rec, src_w=p.src_w)
    dc = f32(p.c_start * W.direction_grf(p.c_start.shape, 6.0, 2))
    H_o = ow.hessvec_gn(sol, p.c_start, dc, e_hist, p.rec, sigma)
    s = solver_for(p, mode, nslots=6)
    s.gradient(p.c_start, p.wavelet, d, sigma)
    H = s.hessvec(p.c_start, dc).cpu().numpy()
    assert rel(H, H_o) < 1e-4
    H2 = s.hessvec(p.c_start, dc).cpu().numpy()     # history reused by every Hv
    assert np.array_equal(H, H2)


def test_full_newton_hessvec_matches_oracle():
    """Full-Newton Hessian action (derivative of the gradient along dc: the
    incremental forward keeps de, then mu and dmu step together backwards) against
    the oracle's, which is pinned to finite differences of the FP64 gradient; the
    full Hessian is symmetric; it differs from the Gauss-Newton one."""
    p = small3d(nt=160)
    sol, d, sigma = oracle_data(p)
    traces, e_hist, _, _ = ow.forward(sol, p.c_start, p.wavelet, p.src, p.rec, src_w=p.src_w)
    _, resid = ow.misfit(sol, traces, d, sigma)
    u = f32(p.c_start * 0.01 * W.direction_grf(p.c_start.shape, 6.0, 2))
    w = f32(p.c_start * 0.01 * W.direction_grf(p.c_start.shape, 6.0, 9))
    Hf_o = ow.hessvec_full(sol, p.c_start, u, e_hist, resid, p.rec, sigma)
    s = solver_for(p, L.STORE_FULL)
    s.gradient(p.c_start, p.wavelet, d, sigma)
    Hu = s.hessvec(p.c_start, u, gauss_newton=False).cpu().numpy()
    print("full Newton rel err", rel(Hu, Hf_o), flush=True)
    assert rel(Hu, Hf_o) < 1e-4
    Hw = s.hessvec(p.c_start, w, gauss_newton=False).cpu().numpy()
    a, b = float(np.sum(w * Hu)), float(np.sum(u * Hw))
    assert abs(a - b) / abs(a) < 1e-4
    Hg = s.hessvec(p.c_start, u).cpu().numpy()
    assert rel(Hg, Hf_o) > 1e-3
    # the gradient residual survives the Gauss-Newton product
    assert np.array_equal(s.hessvec(p.c_start, u, gauss_newton=False).cpu().numpy(), Hu)
    ck = solver_for(p, L.STORE_CHECKPOINT, nslots=6)
    ck.gradient(p.c_start, p.wavelet, d, sigma)
    with pytest.raises(L.WvError):
        ck.hessvec(p.c_start, u, gauss_newton=False)


def test_autograd_gradient_and_double_backward():
    from paper_2304_04781_amd.autograd import WaveMisfit
    p = small3d(nt=150)
    sol, d, sigma = oracle_data(p)
    s = solver_for(p, L.STORE_FULL)
    c = torch.tensor(p.c_start, dtype=torch.float32, device="cuda", requires_grad=True)
    J = WaveMisfit.apply(c, s, torch.tensor(p.wavelet, dtype=torch.float32, device="cuda"),
                         torch.tensor(d, dtype=torch.float32, device="cuda"), sigma)
    (g,) = torch.autograd.grad(J, c, create_graph=True)
    J_o, g_o, _, _ = ow.gradient(sol, p.c_start, p.wavelet, p.src, p.rec, d, sigma, src_w=p.src_w)
    assert rel(g.detach().cpu().numpy(), g_o) < 1e-4
    v = torch.tensor(f32(W.direction_grf(p.c_start.shape, 6.0, 2)), dtype=torch.float32, device="cuda")
    (Hv,) = torch.autograd.grad(g, c, grad_outputs=v)
    H_direct = s.hessvec(c.detach(), v)
    assert torch.equal(Hv, H_direct)


# ----- error paths --------------------------------------------------------------------------------
def test_error_codes():
    p = small3d(nt=20)
    s = solver_for(p, L.STORE_FULL)
    c = np.array(p.c_start)
    bad = c.copy()
    bad[3, 4, 5] = np.nan
    with pytest.raises(L.WvError) as e:
        s.forward(bad, p.wavelet)
    assert e.value.code == -1
    with pytest.raises(L.WvError) as e:
        s.forward(c * 10.0, p.wavelet)
    assert e.value.code == -5
    s2 = solver_for(p, L.STORE_FULL)
    with pytest.raises(L.WvError) as e:
        s2.hessvec(c, c)
    assert e.value.code == -4
    s3 = WaveSolver.for_problem(p)
    with pytest.raises(L.WvError) as e:
        s3.set_storage(L.STORE_CHECKPOINT, n_checkpoints=8, mem_budget_bytes=1000)
    assert e.value.code == -2


# ----- kernel timing ------------------------------------------------------------------------------
@pytest.mark.gpu
def test_kernel_timing_counts_and_durations():
    """Sampled event timing: every 2nd launch of each stencil class is timed on the
    context's stream; the counts follow from the step counts of the solve."""
    p = small3d(nt=21)
    s = solver_for(p, L.STORE_CHECKPOINT, nslots=4)
    d = torch.zeros((len(p.src), p.nt, len(p.rec)), dtype=torch.float32, device="cuda")
    s.set_timing(2)
    s.gradient(p.c_start, p.wavelet, d, 1.0)
    kt = s.kernel_times()
    fsteps, _, _ = s.stats()
    assert kt["forward_stencil"][1] == (fsteps + 1) // 2
    assert kt["adjoint_stencil"][1] == (p.nt - 1 + 1) // 2
    assert kt["forward_stencil"][0] > 0 and kt["adjoint_stencil"][0] > 0
    assert kt["encode"][1] == 0 and kt["decode_e"][1] == 0
    s.set_timing(0)
    assert s.kernel_times()["forward_stencil"][1] == 0
    with pytest.raises(L.WvError) as e:
        L.wv_kernel_time(s.ctx, 8)
    assert e.value.code == -1
