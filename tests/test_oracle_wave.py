"""Pins of the FP64 wave oracle against closed forms, invariants and
identities that hold independently of its code (paper Sec. 2 model and
MAP objective; the adjoint is the exact transpose of the discrete step)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import wave as ow


def small_2d(nt=150, nz=48, nx=64, sponge=8):
    rng = np.random.default_rng(11)
    c = 2000.0 + 600.0 * (np.arange(nz)[:, None, None] / nz) + 50.0 * rng.random((nz, 1, nx))
    dx = 10.0
    dt = 0.4 * dx / c.max()
    sol = ow.Solver(nz, 1, nx, dx, dt, nt, sponge=sponge, c_ref=float(c.max()))
    wav = W.ricker(25.0, dt, nt)[None, :] / dx ** 2
    src = np.array([[4, 0, nx // 2]], dtype=np.int32)
    rec = np.array([[2, 0, i] for i in range(sponge + 1, nx - sponge - 1, 3)], dtype=np.int32)
    return sol, c, wav, src, rec


def small_3d(nt=80, shape=(20, 18, 22), sponge=5):
    nz, ny, nx = shape
    rng = np.random.default_rng(12)
    c = 2000.0 + 400.0 * rng.random(shape)
    dx = 10.0
    dt = 0.4 * dx / c.max()
    sol = ow.Solver(nz, ny, nx, dx, dt, nt, sponge=sponge, c_ref=float(c.max()))
    wav = W.ricker(40.0, dt, nt)[None, :] / dx ** 3
    src = np.array([[3, ny // 2, nx // 2]], dtype=np.int32)
    rec = np.array([[2, j, i] for j in range(6, 12, 2) for i in range(6, 16, 3)], dtype=np.int32)
    return sol, c, wav, src, rec


# ----- operators -------------------------------------------------------------------
def test_gradient_is_minus_divergence_transpose():
    """G_a = -D_a^T for the one-sided boundary closures (brute-force matrices)."""
    sol = ow.Solver(4, 3, 5, 1.0, 0.1, 1, sponge=0)
    n = 4 * 3 * 5
    for a in sol.axes:
        Gm = np.zeros((n, n))
        Dm = np.zeros((n, n))
        for col in range(n):
            unit = np.zeros(n)
            unit[col] = 1.0
            Gm[:, col] = sol.G(unit.reshape(sol.shape), a).ravel()
            v = {b: np.zeros(sol.shape) for b in sol.axes}
            v[a] = unit.reshape(sol.shape)
            Dm[:, col] = sol.D(v).ravel()
        assert np.array_equal(Gm, -Dm.T)


# ----- closed form: exact discrete plane wave ---------------------------------------
@pytest.mark.parametrize("shape,modes", [((16, 12, 20), (1, 2, 3)), ((24, 1, 32), (2, 0, 3))])
def test_plane_wave_exact(shape, modes):
    """Periodic homogeneous medium: e = A cos(k.x - w n dt) and
    v_a = -c A sin(k_a dx/2)/S cos(k.x_a - w (n - 1/2) dt) with
    sin(w dt / 2) = (c dt/dx) S, S^2 = sum_a sin^2(k_a dx/2), solve the
    leapfrog scheme exactly (discrete dispersion relation)."""
    nz, ny, nx = shape
    dx, c0, A = 5.0, 1800.0, 0.7
    sol0 = ow.Solver(nz, ny, nx, dx, 1.0, 1, periodic=True)
    axes = sol0.axes
    dt = 0.45 * dx / c0
    nsteps = 400
    sol = ow.Solver(nz, ny, nx, dx, dt, nsteps, periodic=True)
    k = np.array([2 * math.pi * modes[a] / (shape[a] * dx) for a in range(3)])
    S = math.sqrt(sum(math.sin(k[a] * dx / 2) ** 2 for a in axes))
    w = 2.0 / dt * math.asin(c0 * dt / dx * S)
    idx = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
    xc = [(idx[a] + 0.5) * dx for a in range(3)]

    def phase_c():
        return sum(k[a] * xc[a] for a in axes)

    def phase_f(b):
        return sum(k[a] * (xc[a] - (0.5 * dx if a == b else 0.0)) for a in axes)

    def exact(n):
        e = A * np.cos(phase_c() - w * n * dt)
        v = {b: -c0 * A * math.sin(k[b] * dx / 2) / S * np.cos(phase_f(b) - w * (n - 0.5) * dt)
             for b in axes}
        return v, e

    m = np.full(shape, c0 * c0)
    v, e = exact(0)
    for _ in range(nsteps):
        v, e = sol.step(v, e, m)
    ve, ee = exact(nsteps)
    assert np.max(np.abs(e - ee)) / A < 1e-11
    for b in axes:
        assert np.max(np.abs(v[b] - ve[b])) / (c0 * A) < 1e-11


# ----- invariant: discrete energy ------------------------------------------------------
@pytest.mark.parametrize("shape", [(18, 14, 22), (30, 1, 26)])
def test_energy_conserved_without_layer(shape):
    sol = ow.Solver(*shape, 10.0, 1.2e-3, 1, sponge=0)
    rng = np.random.default_rng(3)
    m = (2000.0 + 800.0 * rng.random(shape)) ** 2
    v = {a: rng.standard_normal(shape) for a in sol.axes}
    e = 1e-3 * rng.standard_normal(shape)
    E0 = ow.energy(sol, v, e, m)
    for _ in range(500):
        v, e = sol.step(v, e, m)
    assert abs(ow.energy(sol, v, e, m) - E0) / E0 < 1e-13


def test_energy_decays_with_layer():
    shape = (30, 26, 28)
    sol = ow.Solver(*shape, 10.0, 1.2e-3, 1, sponge=8, c_ref=2800.0)
    rng = np.random.default_rng(4)
    m = (2000.0 + 800.0 * rng.random(shape)) ** 2
    v = {a: rng.standard_normal(shape) for a in sol.axes}
    e = 1e-3 * rng.standard_normal(shape)
    E = [ow.energy(sol, v, e, m)]
    for _ in range(150):
        v, e = sol.step(v, e, m)
        E.append(ow.energy(sol, v, e, m))
    assert np.all(np.diff(E) <= 1e-12 * E[0])
    assert E[-1] < 0.5 * E[0]


def test_layer_is_identity_inside_and_on_free_surface():
    sol = ow.Solver(40, 36, 44, 10.0, 1e-3, 1, sponge=8, c_ref=3000.0)
    assert np.all(sol.S_e[:32, 8:28, 8:36] == 1.0)
    assert np.all(sol.S_v[0][:32, 8:28, 8:36] == 1.0)
    assert sol.S_e[0, 20, 20] == 1.0 and sol.S_v[0][0, 20, 20] == 1.0   # top: free surface
    assert sol.S_e[39, 20, 20] < 1.0 and sol.S_e[20, 0, 20] < 1.0 and sol.S_e[20, 20, 43] < 1.0
    assert np.all((sol.S_e > 0) & (sol.S_e <= 1))


# ----- adjoint identities ----------------------------------------------------------------
@pytest.mark.parametrize("mk", [small_2d, small_3d])
def test_one_step_dot_test(mk):
    sol, c, _, _, _ = mk()
    m = c * c
    rng = np.random.default_rng(5)
    v = {a: rng.standard_normal(sol.shape) for a in sol.axes}
    e = rng.standard_normal(sol.shape)
    mu = {a: rng.standard_normal(sol.shape) for a in sol.axes}
    eta = rng.standard_normal(sol.shape)
    v1, e1 = sol.step(v, e, m)
    mu0, eta0, _ = sol.step_T(mu, eta, m)
    lhs = sum(np.sum(v1[a] * mu[a]) for a in sol.axes) + np.sum(e1 * eta)
    rhs = sum(np.sum(v[a] * mu0[a]) for a in sol.axes) + np.sum(e * eta0)
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


@pytest.mark.parametrize("mk", [small_2d, small_3d])
def test_jacobian_dot_test(mk):
    """<J dc, w> = <dc, J^T w>: incremental forward against the adjoint."""
    sol, c, wav, src, rec = mk()
    rng = np.random.default_rng(6)
    _, e_hist, _, _ = ow.forward(sol, c, wav, src, rec)
    dc = rng.standard_normal(sol.shape)
    w = rng.standard_normal((sol.nt, len(rec)))
    dp, _ = ow.inc_forward(sol, c, dc, e_hist[0], rec)
    JTw = -2.0 * sol.dt * c * ow.adjoint_acc(sol, c, e_hist[0], w, rec)
    lhs = float(np.sum(dp * w))
    rhs = float(np.sum(dc * JTw))
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


def test_inc_forward_matches_fd_of_forward():
    sol, c, wav, src, rec = small_2d(nt=120)
    rng = np.random.default_rng(7)
    dc = c * 0.01 * rng.standard_normal(sol.shape)
    _, e_hist, _, _ = ow.forward(sol, c, wav, src, rec)
    dp, _ = ow.inc_forward(sol, c, dc, e_hist[0], rec)
    h = 1e-3
    tp = ow.forward(sol, c + h * dc, wav, src, rec, store_e=False)[0][0]
    tm = ow.forward(sol, c - h * dc, wav, src, rec, store_e=False)[0][0]
    fd = (tp - tm) / (2 * h)
    assert np.linalg.norm(fd - dp) / np.linalg.norm(dp) < 1e-5


# ----- gradient --------------------------------------------------------------------------
def test_gradient_taylor_2d_workload():
    """Central FD of J along a smooth direction on the 128^2 x 500 workload:
    second-order convergence and agreement to 1e-8 at h = 1e-4."""
    p = W.problem_2d_small()
    sol = ow.solver_for(p)
    d, sigma, _ = ow.observed_data(sol, p)
    J, g, _, _ = ow.gradient(sol, p.c_start, p.wavelet, p.src, p.rec, d, sigma, src_w=p.src_w)
    assert J > 0
    dc = p.c_start * 0.01 * W.direction_grf(p.c_start.shape, 8.0, 7)
    an = float(np.sum(g * dc))
    errs = []
    for h in (1e-2, 1e-3, 1e-4):
        Jp = ow.gradient(sol, p.c_start + h * dc, p.wavelet, p.src, p.rec, d, sigma, src_w=p.src_w)[0]
        Jm = ow.gradient(sol, p.c_start - h * dc, p.wavelet, p.src, p.rec, d, sigma, src_w=p.src_w)[0]
        errs.append(abs((Jp - Jm) / (2 * h) - an) / abs(an))
    assert errs[2] < 1e-8
    assert errs[0] / errs[1] > 50.0       # slope ~2 (ratio 100)


def test_gradient_fd_3d_multisource():
    sol, c, wav, src, rec = small_3d(nt=70)
    src = np.array([[3, 9, 11], [5, 7, 8]], dtype=np.int32)
    wav = np.stack([wav[0], 0.7 * np.roll(wav[0], 5)])
    d = ow.forward(sol, c * 1.02, wav, src, rec, store_e=False)[0]
    sigma = 0.05 * float(np.max(np.abs(d)))
    J, g, _, _ = ow.gradient(sol, c, wav, src, rec, d, sigma)
    rng = np.random.default_rng(8)
    dc = c * 0.01 * rng.standard_normal(sol.shape)
    h = 1e-3
    Jp = ow.gradient(sol, c + h * dc, wav, src, rec, d, sigma)[0]
    Jm = ow.gradient(sol, c - h * dc, wav, src, rec, d, sigma)[0]
    an = float(np.sum(g * dc))
    assert abs((Jp - Jm) / (2 * h) - an) / abs(an) < 1e-6


def test_zero_residual_gives_zero_gradient():
    sol, c, wav, src, rec = small_2d(nt=60)
    d = ow.forward(sol, c, wav, src, rec, store_e=False)[0]
    J, g, _, _ = ow.gradient(sol, c, wav, src, rec, d, 1.0)
    assert J == 0.0 and np.all(g == 0.0)


# ----- Hessian-vector products ---------------------------------------------------------------
def _hess_setup(zero_residual):
    sol, c, wav, src, rec = small_2d(nt=100, nz=40, nx=48, sponge=6)
    c_true = c * (1.0 + 0.15 * np.exp(-((np.arange(40)[:, None, None] - 20) ** 2
                                          + (np.arange(48)[None, None, :] - 24) ** 2) / 50.0))
    d = ow.forward(sol, c if zero_residual else c_true, wav, src, rec, store_e=False)[0]
    sigma = 0.01 * float(np.max(np.abs(d)))
    return sol, c, wav, src, rec, d, sigma


def test_gn_hessian_symmetric():
    sol, c, wav, src, rec, d, sigma = _hess_setup(False)
    _, e_hist, _, _ = ow.forward(sol, c, wav, src, rec)
    rng = np.random.default_rng(9)
    x = rng.standard_normal(sol.shape)
    y = rng.standard_normal(sol.shape)
    Hx = ow.hessvec_gn(sol, c, x, e_hist, rec, sigma)
    Hy = ow.hessvec_gn(sol, c, y, e_hist, rec, sigma)
    a, b = float(np.sum(y * Hx)), float(np.sum(x * Hy))
    assert abs(a - b) / abs(a) < 1e-12
    assert float(np.sum(x * Hx)) > 0.0          # GN is positive semi-definite


def _fd_hess(sol, c, wav, src, rec, d, sigma, dc, h=1e-3):
    gp = ow.gradient(sol, c + h * dc, wav, src, rec, d, sigma)[1]
    gm = ow.gradient(sol, c - h * dc, wav, src, rec, d, sigma)[1]
    return (gp - gm) / (2 * h)


def test_gn_hessvec_matches_fd_at_zero_residual():
    """At a zero-residual point the Gauss-Newton and full Hessians coincide,
    so GN Hv equals the FD of the gradient (step 1e-3)."""
    sol, c, wav, src, rec, d, sigma = _hess_setup(True)
    _, e_hist, _, _ = ow.forward(sol, c, wav, src, rec)
    dc = c * 0.01 * W.direction_grf(sol.shape, 6.0, 2)
    H = ow.hessvec_gn(sol, c, dc, e_hist, rec, sigma)
    fd = _fd_hess(sol, c, wav, src, rec, d, sigma, dc)
    assert np.linalg.norm(H - fd) / np.linalg.norm(fd) < 1e-6


def test_full_hessvec_matches_fd_and_differs_from_gn():
    sol, c, wav, src, rec, d, sigma = _hess_setup(False)
    traces, e_hist, _, _ = ow.forward(sol, c, wav, src, rec)
    _, resid = ow.misfit(sol, traces, d, sigma)
    dc = c * 0.01 * W.direction_grf(sol.shape, 6.0, 2)
    Hf = ow.hessvec_full(sol, c, dc, e_hist, resid, rec, sigma)
    Hg = ow.hessvec_gn(sol, c, dc, e_hist, rec, sigma)
    fd = _fd_hess(sol, c, wav, src, rec, d, sigma, dc)
    assert np.linalg.norm(Hf - fd) / np.linalg.norm(fd) < 1e-6
    assert np.linalg.norm(Hg - fd) / np.linalg.norm(fd) > 1e-3


def test_unit_box_source_equals_point_force_and_is_linear():
    sol, c, wav, src, rec = small_3d(nt=40)
    tp, _, _, _ = ow.forward(sol, c, wav, src, rec, store_e=False)
    w = np.zeros((5, 5, 5))
    w[2, 2, 2] = 1.0
    tb, _, _, _ = ow.forward(sol, c, wav, src, rec, store_e=False, src_w=w)
    assert np.array_equal(tp, tb)
    # a box straddling the top surface is truncated, and the response is linear in the weights
    w1 = W.source_weights(10.0, 3, 20.0)
    w2 = np.random.default_rng(3).random(w1.shape)
    t1 = ow.forward(sol, c, wav, src, rec, store_e=False, src_w=w1)[0]
    t2 = ow.forward(sol, c, wav, src, rec, store_e=False, src_w=w2)[0]
    t12 = ow.forward(sol, c, wav, src, rec, store_e=False, src_w=2.0 * w1 - w2)[0]
    assert np.allclose(t12, 2.0 * t1 - t2, rtol=1e-12, atol=1e-12 * np.abs(t1).max())
    assert abs(w1.sum() - 1.0) < 1e-14 and w1.shape[0] == 2 * 6 + 1
