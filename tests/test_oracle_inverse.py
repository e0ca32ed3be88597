"""Pins of the FP64 inverse-problem oracle (BiLaplacian prior of Sec. 2, the
Newton-CG loop of Sec. 4) against closed forms, brute force and problems whose
minimiser is known, independently of its code."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import inverse as oi
from oracle import wave as ow


def dct_mode(shape, modes):
    """Product of cos(pi (i + 1/2) m / n) along each axis: the cell-centred
    cosine modes, eigenvectors of the zero-flux second difference."""
    out = np.ones(shape)
    for axis, (n, m) in enumerate(zip(shape, modes)):
        i = np.arange(n) + 0.5
        sh = [1, 1, 1]
        sh[axis] = n
        out = out * np.cos(math.pi * i * m / n).reshape(sh)
    return out


@pytest.mark.parametrize("shape,modes", [((6, 5, 7), (1, 2, 3)), ((6, 5, 7), (0, 4, 6)), ((8, 1, 9), (3, 0, 5))])
def test_prior_cosine_modes_are_eigenvectors(shape, modes):
    """A u = alpha (1 + sum_a theta_a / dx^2 (2 - 2 cos(pi m_a / n_a))) u for the
    cosine modes: the closed-form spectrum of the zero-flux (Neumann) Laplacian.
    A wrong boundary closure, coefficient or axis order fails it; in the 2D mode
    (ny == 1) the y term is absent whatever theta_y says."""
    alpha, dx = 0.7, 12.5
    theta = (300.0, 500.0, 900.0)
    u = dct_mode(shape, modes)
    lam = 1.0
    for axis, (n, m) in enumerate(zip(shape, modes)):
        if n > 1:
            lam += theta[axis] / dx ** 2 * (2.0 - 2.0 * math.cos(math.pi * m / n))
    Au = oi.prior_operator(u, alpha, theta, dx)
    np.testing.assert_allclose(Au, alpha * lam * u, rtol=1e-12, atol=1e-12)


def test_prior_matrix_symmetric_positive_with_known_extremes():
    """Brute-force matrix of A on a 3 x 4 x 5 grid: symmetric; its smallest
    eigenvalue is alpha (the constant vector, no flux anywhere) and its largest
    is the highest cosine mode's."""
    shape, alpha, dx, theta = (3, 4, 5), 1.3, 2.0, (0.5, 1.5, 2.5)
    n = int(np.prod(shape))
    M = np.zeros((n, n))
    for col in range(n):
        e = np.zeros(n)
        e[col] = 1.0
        M[:, col] = oi.prior_operator(e.reshape(shape), alpha, theta, dx).ravel()
    np.testing.assert_array_equal(M, M.T)
    ev = np.linalg.eigvalsh(M)
    assert abs(ev[0] - alpha) < 1e-12
    top = alpha * (1 + sum(th / dx ** 2 * (2 - 2 * math.cos(math.pi * (k - 1) / k)) for th, k in zip(theta, shape)))
    assert abs(ev[-1] - top) < 1e-11
    # row sums: alpha (constant vector is an eigenvector with eigenvalue alpha)
    np.testing.assert_allclose(M.sum(axis=1), alpha, rtol=0, atol=1e-12)


def test_prior_cost_constant_offset_and_derivatives():
    """R(c0 + kappa) = 1/2 dx^3 alpha^2 kappa^2 N; grad and Hessian against
    central differences of the cost (exact for a quadratic up to rounding)."""
    rng = np.random.default_rng(3)
    shape, alpha, dx, theta = (5, 6, 7), 0.01, 10.0, (400.0, 400.0, 900.0)
    c0 = 2000 + 100 * rng.random(shape)
    R, g = oi.prior_cost_grad(c0 + 3.0, c0, alpha, theta, dx)
    assert abs(R - 0.5 * dx ** 3 * alpha ** 2 * 9.0 * np.prod(shape)) < 1e-9 * R
    c = c0 + 20 * rng.standard_normal(shape)
    R, g = oi.prior_cost_grad(c, c0, alpha, theta, dx)
    v = rng.standard_normal(shape)
    h = 1e-2
    fd = (oi.prior_cost_grad(c + h * v, c0, alpha, theta, dx)[0] - oi.prior_cost_grad(c - h * v, c0, alpha, theta, dx)[0]) / (2 * h)
    assert abs(fd - np.sum(g * v)) < 1e-7 * abs(fd)
    Hv = oi.prior_hessvec(v, alpha, theta, dx)
    fdg = (oi.prior_cost_grad(c + h * v, c0, alpha, theta, dx)[1] - oi.prior_cost_grad(c - h * v, c0, alpha, theta, dx)[1]) / (2 * h)
    np.testing.assert_allclose(Hv, fdg, rtol=1e-7, atol=1e-9 * np.abs(Hv).max())
    # the 2D mode weights by dx^2
    c2 = c0[:, :1, :]
    R2, _ = oi.prior_cost_grad(c2 + 1.0, c2, alpha, theta, dx)
    assert abs(R2 - 0.5 * dx ** 2 * alpha ** 2 * c2.size) < 1e-9 * R2


@pytest.mark.parametrize("shape", [(6, 5, 7), (9, 1, 8)])
def test_prior_sample_inverts_the_operator(shape):
    """c = c0 + A^-1 w / sqrt(vol): applying A (the finite-volume stencil, not the
    spectral form the sampler uses) to c - c0 returns w / sqrt(vol); and the
    sample covariance over many draws on a tiny grid approaches (vol A A)^-1."""
    rng = np.random.default_rng(8)
    alpha, dx, theta = 0.05, 20.0, (1600.0, 900.0, 2500.0)
    c0 = 2000.0 + 10 * rng.random(shape)
    w = rng.standard_normal(shape)
    vol = oi.cell_volume(shape, dx)
    c = oi.prior_sample(w, c0, alpha, theta, dx)
    np.testing.assert_allclose(oi.prior_operator(c - c0, alpha, theta, dx) * np.sqrt(vol), w, rtol=1e-10, atol=1e-10)
    if shape[1] == 1:
        return
    small = (2, 2, 3)
    n = int(np.prod(small))
    M = np.zeros((n, n))
    for col in range(n):
        e = np.zeros(n)
        e[col] = 1.0
        M[:, col] = oi.prior_operator(e.reshape(small), alpha, theta, dx).ravel()
    cov = np.linalg.inv(oi.cell_volume(small, dx) * M @ M)
    draws = np.stack([oi.prior_sample(rng.standard_normal(small), np.zeros(small), alpha, theta, dx).ravel()
                      for _ in range(20000)])
    emp = draws.T @ draws / len(draws)
    assert np.abs(emp - cov).max() < 0.05 * np.abs(cov).max()


def test_cg_solves_spd_system_and_stops_on_negative_curvature():
    rng = np.random.default_rng(5)
    n = 12
    Q = rng.standard_normal((n, n))
    H = Q @ Q.T + n * np.eye(n)
    g = rng.standard_normal(n)
    p, its, neg, rel = oi.cg_steihaug(lambda v: H @ v, g, 1e-14, 4 * n)
    np.testing.assert_allclose(p, np.linalg.solve(H, -g), rtol=1e-10, atol=1e-12)
    assert not neg and rel <= 1e-14
    # the forcing stops it early with ||r|| <= eta ||g||
    p, its, neg, rel = oi.cg_steihaug(lambda v: H @ v, g, 0.3, 4 * n)
    assert rel <= 0.3 and its < n and np.linalg.norm(H @ p + g) <= 0.3 * np.linalg.norm(g) * (1 + 1e-12)
    # max_cg bounds the iterations
    assert oi.cg_steihaug(lambda v: H @ v, g, 1e-14, 3)[1] == 3
    # non-positive curvature along -g at the first iteration: steepest descent
    Hn = np.diag([-1.0, 2.0, 3.0])
    p, its, neg, _ = oi.cg_steihaug(lambda v: Hn @ v, np.array([1.0, 0.0, 0.0]), 1e-8, 10)
    assert neg and its == 1 and np.array_equal(p, [-1.0, 0.0, 0.0])
    # later: the iterate before the direction of non-positive curvature is kept
    Hn = np.diag([3.0, -1.0])
    p, its, neg, _ = oi.cg_steihaug(lambda v: Hn @ v, np.array([1.0, 0.5]), 1e-8, 10)
    a = (1.25) / (3.0 - 0.25)
    assert neg and its == 2
    np.testing.assert_allclose(p, [-a, -0.5 * a], rtol=1e-14)


def test_preconditioned_cg():
    """With any SPD preconditioner CG still solves the SPD system exactly; with
    M = H^-1 it needs one iteration; the prior covariance (spectral solve) is the
    inverse of dx^dims A A (finite-volume stencil)."""
    rng = np.random.default_rng(9)
    n = 12
    Q = rng.standard_normal((n, n))
    H = Q @ Q.T + n * np.eye(n)
    g = rng.standard_normal(n)
    Md = rng.uniform(0.1, 3.0, n)
    p, its, neg, rel = oi.cg_steihaug(lambda v: H @ v, g, 1e-14, 4 * n, prec=lambda v: Md * v)
    np.testing.assert_allclose(p, np.linalg.solve(H, -g), rtol=1e-10, atol=1e-12)
    Hinv = np.linalg.inv(H)
    p, its, neg, rel = oi.cg_steihaug(lambda v: H @ v, g, 1e-8, 10, prec=lambda v: Hinv @ v)
    assert its == 1 and rel < 1e-10
    np.testing.assert_allclose(p, -Hinv @ g, rtol=1e-10)
    # first-iteration negative curvature returns the preconditioned direction -M g
    Hn = np.diag([-1.0, 2.0])
    p, its, neg, _ = oi.cg_steihaug(lambda v: Hn @ v, np.array([1.0, 0.0]), 1e-8, 5, prec=lambda v: 2.0 * v)
    assert neg and its == 1 and np.array_equal(p, [-2.0, 0.0])
    shape, alpha, dx, theta = (6, 5, 7), 0.03, 20.0, (1600.0, 900.0, 2500.0)
    r = rng.standard_normal(shape)
    z = oi.prior_covariance(r, alpha, theta, dx)
    back = oi.cell_volume(shape, dx) * oi.prior_operator(oi.prior_operator(z, alpha, theta, dx), alpha, theta, dx)
    np.testing.assert_allclose(back, r, rtol=1e-9, atol=1e-9)


def test_newton_one_step_on_a_quadratic():
    """J = 1/2 x.Qx - b.x: one Newton step with CG to high accuracy lands on
    Q^-1 b with the full step accepted; the next test of the gradient stops."""
    rng = np.random.default_rng(7)
    n = 10
    Q = rng.standard_normal((n, n))
    Q = Q @ Q.T + np.eye(n)
    b = rng.standard_normal(n)
    cg = lambda x: (0.5 * x @ Q @ x - b @ x, Q @ x - b, None)
    hv = lambda st, v: Q @ v
    cfg = oi.NewtonConfig(max_newton=5, max_cg=50, eta_max=1e-13, rel_tol=1e-9)
    # a forcing this small needs eta_max to bind at the first step only
    x, log, reason = oi.newton_cg(cg, hv, np.zeros(n), cfg)
    np.testing.assert_allclose(x, np.linalg.solve(Q, b), rtol=1e-9, atol=1e-10)
    assert log[0].step == 1.0 and log[0].backtracks == 0
    assert reason == 1 and len(log) == 2
    # the same with a diagonal preconditioner
    x, log, reason = oi.newton_cg(cg, hv, np.zeros(n), cfg, prec=lambda v: v / np.diag(Q))
    np.testing.assert_allclose(x, np.linalg.solve(Q, b), rtol=1e-9, atol=1e-10)
    assert reason == 1 and len(log) == 2


def test_newton_rosenbrock_reaches_known_minimiser():
    """Rosenbrock's function, minimiser (1, 1): the full-Hessian Newton-CG with
    backtracking converges from the classic start (-1.2, 1); on the way the
    Hessian is indefinite, so the negative-curvature and backtracking branches run."""
    def cg(x):
        a, b = x
        J = (1 - a) ** 2 + 100 * (b - a * a) ** 2
        g = np.array([-2 * (1 - a) - 400 * a * (b - a * a), 200 * (b - a * a)])
        return J, g, x.copy()

    def hv(x, v):
        a, b = x
        H = np.array([[2 - 400 * (b - 3 * a * a), -400 * a], [-400 * a, 200.0]])
        return H @ v

    cfg = oi.NewtonConfig(max_newton=100, max_cg=2, eta_max=0.5, rel_tol=1e-10, max_backtrack=30)
    x, log, reason = oi.newton_cg(cg, hv, np.array([-1.2, 1.0]), cfg)
    assert reason == 1
    np.testing.assert_allclose(x, [1.0, 1.0], atol=1e-7)
    assert all(r1.cost < r0.cost for r0, r1 in zip(log, log[1:]))
    assert any(r.backtracks > 0 for r in log)


def _wave_case():
    nz, ny, nx, nt = 14, 12, 16, 60
    rng = np.random.default_rng(21)
    c_true = 2000.0 + 300.0 * rng.random((nz, ny, nx))
    c0 = np.full((nz, ny, nx), 2150.0)
    dx = 10.0
    dt = 0.4 * dx / 2600.0
    sol = ow.Solver(nz, ny, nx, dx, dt, nt, sponge=3, c_ref=2600.0)
    wav = W.ricker(45.0, dt, nt)[None, :] / dx ** 3
    src = np.array([[3, ny // 2, nx // 2]], dtype=np.int32)
    rec = np.array([[2, j, i] for j in range(4, 9, 2) for i in range(4, 13, 2)], dtype=np.int32)
    d, _, _, _ = ow.forward(sol, c_true, wav, src, rec)
    sigma = 0.01 * float(np.abs(d).max())
    return sol, c_true, c0, wav, src, rec, d, sigma


def test_map_objective_gradient_and_hessian_by_differences():
    """The MAP objective (misfit + prior): its gradient and its Gauss-Newton and
    full Hv against central differences; the full Hv is the derivative of the
    gradient, the GN one only at zero residual (here the residual is not zero)."""
    sol, c_true, c0, wav, src, rec, d, sigma = _wave_case()
    alpha, theta = 1e-6, (400.0, 400.0, 400.0)
    cost_grad, hv_gn = oi.wave_map_problem(sol, wav, src, rec, d, sigma, c0, alpha, theta, True)
    _, hv_full = oi.wave_map_problem(sol, wav, src, rec, d, sigma, c0, alpha, theta, False)
    rng = np.random.default_rng(2)
    c = c0 + 30 * rng.standard_normal(c0.shape)
    v = rng.standard_normal(c0.shape)
    J, g, st = cost_grad(c)
    h = 0.05
    Jp, gp, _ = cost_grad(c + h * v)
    Jm, gm, _ = cost_grad(c - h * v)
    fd = (Jp - Jm) / (2 * h)
    assert abs(fd - np.sum(g * v)) < 1e-6 * abs(fd)
    fdg = (gp - gm) / (2 * h)
    Hf = hv_full(st, v)
    assert np.linalg.norm(Hf - fdg) < 1e-5 * np.linalg.norm(fdg)
    assert np.linalg.norm(hv_gn(st, v) - fdg) > 1e-3 * np.linalg.norm(fdg)


def test_wave_newton_decreases_cost():
    """Two Gauss-Newton iterations on the small wave problem: every accepted step
    satisfies the Armijo condition, and the cost and gradient fall."""
    sol, c_true, c0, wav, src, rec, d, sigma = _wave_case()
    cost_grad, hv = oi.wave_map_problem(sol, wav, src, rec, d, sigma, c0, 1e-6, (400.0, 400.0, 400.0), True)
    cfg = oi.NewtonConfig(max_newton=2, max_cg=4)
    c, log, reason = oi.newton_cg(cost_grad, hv, c0, cfg)
    assert reason == 0 and len(log) == 3
    assert log[2].cost < log[1].cost < log[0].cost
    assert log[2].gnorm < log[0].gnorm
