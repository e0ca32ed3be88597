"""GPU parity of the MAP layer against the FP64 oracle: the BiLaplacian prior
(paper Sec. 2) and the Newton-CG loop (Sec. 4) built on the gradient and the
Hessian actions.

Inputs are float32-rounded and the oracle runs on them in float64. The prior
is a 7-point float32 stencil, so cost, gradient and Hessian action agree to
1e-5 relative. Newton-CG takes its branch decisions (CG stop, curvature sign,
Armijo acceptance) from float64 dot products of float32 vectors. The cases
keep them away from their thresholds: the CG iteration cap binds and full
steps are accepted. So the iteration records must match exactly, and costs,
gradient norms and the model update agree to 1e-3 relative (a few float32
Hessian actions compounded through CG)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import inverse as oi
from oracle import wave as ow
from paper_2304_04781_amd import _lib as L
from paper_2304_04781_amd.solver import WaveSolver

pytestmark = pytest.mark.gpu

ALPHA, THETA = 2e-6, (1600.0, 1600.0, 1600.0)


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rounded(p):
    p.c_true, p.c_start, p.wavelet = f32(p.c_true), f32(p.c_start), f32(p.wavelet)
    return p


@pytest.mark.parametrize("which", ["3d", "2d"])
def test_prior_cost_gradient_hessvec(which):
    p = rounded(W.problem_3d(20, 18, 22, 10, sponge=3) if which == "3d" else W.problem_2d_small(nt=10))
    print("case", which, p.name, flush=True)
    u = f32(p.c_start * (1.0 + 0.02 * W.direction_grf(p.c_start.shape, 3.0, 5)))
    v = f32(p.c_start * 0.01 * W.direction_grf(p.c_start.shape, 3.0, 6))
    R_o, g_o = oi.prior_cost_grad(u, p.c_start, ALPHA, THETA, p.dx)
    H_o = oi.prior_hessvec(v, ALPHA, THETA, p.dx)
    s = WaveSolver.for_problem(p)
    s.set_prior(ALPHA, THETA, p.c_start)
    R, g = s.prior(u)
    assert abs(R - R_o) < 1e-5 * R_o
    assert rel(g.cpu().numpy(), g_o) < 1e-5
    assert rel(s.prior_hessvec(v).cpu().numpy(), H_o) < 1e-5
    # accumulation into the output, as the Newton loop uses it
    H = torch.as_tensor(np.float32(H_o), device="cuda")
    L.wv_prior_hessvec(s.ctx, s._f32(v), H)
    assert rel(H.cpu().numpy(), 2 * H_o) < 1e-5
    # no prior: zero cost, output untouched
    s.set_prior(0.0)
    R0, g0 = s.prior(u)
    assert R0 == 0.0 and not torch.any(g0)


def newton_case():
    p = rounded(W.problem_3d(24, 20, 28, 120, f0=15.0, sponge=5, name="newton3d-24x20x28-120"))
    sol = ow.solver_for(p)
    d, sigma, _ = ow.observed_data(sol, p)
    return p, sol, f32(d), sigma


@pytest.mark.parametrize("gauss_newton,precondition", [(1, 0), (0, 0), (1, 1), (0, 1)])
def test_newton_cg_matches_oracle(gauss_newton, precondition):
    """Three Newton iterations with at most 4 CG iterations each (full storage),
    without and with the prior-covariance preconditioner (on the GPU two CG solves
    of the elliptic operator to 1e-6, in the oracle the exact cosine-mode solve):
    iteration records, costs, gradient norms and the final model against the
    oracle's Newton-CG on the same problem."""
    p, sol, d, sigma = newton_case()
    print("case", p.name, "gauss_newton", gauss_newton, "precondition", precondition, flush=True)
    cfg = dict(max_newton=3, max_cg=4, eta_max=0.5, rel_tol=1e-8, c_armijo=1e-4, max_backtrack=10)
    cost_grad, hv = oi.wave_map_problem(sol, p.wavelet, p.src, p.rec, d, sigma, p.c_start, ALPHA, THETA,
                                        gauss_newton=bool(gauss_newton), src_w=p.src_w)
    prec = (lambda r: oi.prior_covariance(r, ALPHA, THETA, p.dx)) if precondition else None
    c_o, log_o, reason_o = oi.newton_cg(cost_grad, hv, p.c_start, oi.NewtonConfig(**cfg), prec=prec)
    s = WaveSolver.for_problem(p)
    s.set_storage(L.STORE_FULL)
    s.set_prior(ALPHA, THETA, p.c_start)
    c, log, it, reason = s.newton_cg(p.c_start, p.wavelet, d, sigma, gauss_newton=gauss_newton,
                                     precondition=precondition, **cfg)
    for r_o, r in zip(log_o, log):
        print("oracle", r_o, "\ngpu   ", r, flush=True)
    assert reason == reason_o and it == len(log_o) - 1
    for r_o, r in zip(log_o, log):
        assert (r["cg_iters"], bool(r["neg_curv"]), r["backtracks"]) == (r_o.cg_iters, r_o.neg_curv, r_o.backtracks)
        assert r["step"] == r_o.step
        assert abs(r["cost"] - r_o.cost) < 1e-3 * r_o.cost
        assert abs(r["gnorm"] - r_o.gnorm) < 1e-3 * r_o.gnorm
    # misfit and prior both fall over the run; the update agrees with the oracle's
    assert log[-1]["cost"] < log[0]["cost"]
    assert rel(c.cpu().numpy() - p.c_start, c_o - p.c_start) < 1e-3


def test_newton_cg_checkpointing_equals_full_storage():
    """The Gauss-Newton loop on revolve checkpointing (forward recomputed in every
    Hessian action) takes the same path as with full storage, bit for bit."""
    p, sol, d, sigma = newton_case()
    cfg = dict(max_newton=2, max_cg=3)
    out = []
    for mode in (L.STORE_FULL, L.STORE_CHECKPOINT):
        s = WaveSolver.for_problem(p)
        s.set_storage(mode, n_checkpoints=8)
        s.set_prior(ALPHA, THETA, p.c_start)
        out.append(s.newton_cg(p.c_start, p.wavelet, d, sigma, **cfg))
    (c0, log0, _, _), (c1, log1, _, _) = out
    assert torch.equal(c0, c1)
    assert [r["cost"] for r in log0] == [r["cost"] for r in log1]


def test_newton_cg_argument_checks():
    p, sol, d, sigma = newton_case()
    s = WaveSolver.for_problem(p)
    with pytest.raises(L.WvError):   # no storage mode
        s.newton_cg(p.c_start, p.wavelet, d, sigma)
    s.set_storage(L.STORE_FULL)
    for bad in (dict(max_cg=0), dict(eta_max=1.0), dict(c_armijo=0.0), dict(gauss_newton=2), dict(max_newton=-1),
                dict(precondition=2), dict(precondition=1)):   # the last: no prior set
        with pytest.raises(L.WvError):
            s.newton_cg(p.c_start, p.wavelet, d, sigma, **bad)
    with pytest.raises(L.WvError):
        s.set_prior(-1.0, THETA, p.c_start)
    # zero iterations: the record of the starting point only
    c, log, it, reason = s.newton_cg(p.c_start, p.wavelet, d, sigma, max_newton=0)
    assert it == 0 and reason == 0 and len(log) == 1
    assert np.array_equal(c.cpu().numpy(), np.float32(p.c_start))


@pytest.mark.parametrize("which", ["3d", "2d"])
def test_prior_sample_matches_oracle(which):
    """A prior draw by conjugate gradients on the GPU against the oracle's exact
    cosine-mode solve for the same white noise (float32 CG to 1e-6 residual,
    condition number of A about 1 + 12 theta / dx^2 = 49)."""
    p = rounded(W.problem_3d(24, 20, 28, 10, sponge=3) if which == "3d" else W.problem_2d_small(nt=10))
    print("case", which, p.name, flush=True)
    w = f32(W.white_noise(p.c_start.shape, 7))
    ref = oi.prior_sample(w, p.c_start, ALPHA, THETA, p.dx)
    s = WaveSolver.for_problem(p)
    with pytest.raises(L.WvError):   # no prior set
        s.prior_sample(w)
    s.set_prior(ALPHA, THETA, p.c_start)
    c, it, rr = s.prior_sample(w, rtol=1e-6)
    print("CG iterations", it, "relative residual", rr, flush=True)
    assert rr <= 1e-6 and it < 2000
    assert rel(c.cpu().numpy() - p.c_start, ref - p.c_start) < 1e-4


@pytest.mark.parametrize("gauss_newton", [True, False])
def test_autograd_map_objective(gauss_newton):
    """The MAP objective through torch.autograd (misfit + BiLaplacian prior): value,
    gradient and the double-backward Hessian action against the oracle's (Gauss-
    Newton or full-Newton misfit Hessian plus the exact prior Hessian)."""
    from paper_2304_04781_amd.autograd import BiLaplacianPrior, WaveMisfit
    p, sol, d, sigma = newton_case()
    cost_grad, hv = oi.wave_map_problem(sol, p.wavelet, p.src, p.rec, d, sigma, p.c_start, ALPHA, THETA,
                                        gauss_newton=gauss_newton, src_w=p.src_w)
    cm = f32(p.c_start * (1.0 + 0.01 * W.direction_grf(p.c_start.shape, 3.0, 4)))
    J_o, g_o, st = cost_grad(cm)
    v = f32(p.c_start * 0.01 * W.direction_grf(p.c_start.shape, 3.0, 8))
    H_o = hv(st, v)
    s = WaveSolver.for_problem(p)
    s.set_storage(L.STORE_FULL)
    s.set_prior(ALPHA, THETA, p.c_start)
    c = torch.tensor(cm, dtype=torch.float32, device="cuda", requires_grad=True)
    J = WaveMisfit.apply(c, s, s._f32(p.wavelet), s._f32(d), sigma, gauss_newton) + BiLaplacianPrior.apply(c, s)
    assert abs(float(J.detach()) - J_o) < 1e-5 * J_o
    (g,) = torch.autograd.grad(J, c, create_graph=True)
    assert rel(g.detach().cpu().numpy(), g_o) < 1e-4
    (Hv,) = torch.autograd.grad(g, c, grad_outputs=torch.tensor(v, dtype=torch.float32, device="cuda"))
    assert rel(Hv.cpu().numpy(), H_o) < 1e-4
