"""FP64 oracle of the inverse-problem layer: the BiLaplacian prior and the
inexact Newton-CG loop that computes the MAP point.

TEST INFRASTRUCTURE ONLY (see the package docstring).

MAP objective (paper Sec. 2):
    min_c  1/2 ||F(c) - d||^2_{noise^-1} + 1/2 ||c - c0||^2_{prior^-1},
with c0 the initial guess (prior mean). The prior is the PDE-based
BiLaplacian of Sec. 2: the elliptic operator
    A u = alpha (u - div(Theta grad u))   in the domain,
    (Theta grad u) . n = 0               on the boundary,
whose square is the inverse prior covariance. Theta = diag(theta_z, theta_y,
theta_x) (m^2) carries the anisotropy.

Discretisation (cell-centred, the grid of the wave solver): the divergence of
the flux Theta grad u is the sum over the 2 dims faces of each cell of
theta_a (u_nb - u) / dx^2, where faces on the domain boundary carry zero flux
(the Neumann condition). With the lumped mass dx^dims I the prior term is
    R(c) = 1/2 dx^dims ||A (c - c0)||^2,  grad R = dx^dims A A (c - c0),
    Hess R = dx^dims A A    (A is symmetric).

Prior draws (Sec. 3.3.1, Algorithm 1 trains the compressor on forward solves at
draws from the prior): c = c0 + A^-1 w / sqrt(dx^dims), w white noise.

Newton-CG (Sec. 4; the method of its references on inexact Newton-CG for
wave inversion):
  * CG on H p = -g from p = 0, optionally preconditioned by the prior
    covariance (dx^dims A A)^-1, stopped when ||r||_M <= eta ||g||_M with the
    Eisenstat-Walker forcing eta = min(eta_max, sqrt(||g|| / ||g_0||)), after
    max_cg iterations, or at the first direction of non-positive curvature
    (then the iterate so far is kept; at the first iteration the
    (preconditioned) steepest-descent direction -M g is taken);
  * Armijo backtracking: the step length starts at 1 and halves until
    J(c + a p) <= J(c) + c_armijo a g.p;
  * stop when ||g|| <= rel_tol ||g_0|| or after max_newton iterations.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, List, Sequence

import numpy as np


def prior_operator(u: np.ndarray, alpha: float, theta: Sequence[float], dx: float) -> np.ndarray:
    """A u = alpha (u - div(Theta grad u)) with zero flux on every boundary face
    (Sec. 2, BiLaplacian prior). u is [nz, ny, nx]; ny == 1 drops the y term."""
    u = np.asarray(u, dtype=np.float64)
    out = u.copy()
    for axis in range(3):
        if u.shape[axis] == 1:
            continue
        th = float(theta[axis]) / (dx * dx)
        n = u.shape[axis]
        # flux through each interior face f between cells f and f+1
        lo = np.take(u, np.arange(n - 1), axis=axis)
        hi = np.take(u, np.arange(1, n), axis=axis)
        flux = th * (hi - lo)
        div = np.zeros_like(u)
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[axis] = slice(0, n - 1)
        sl_hi[axis] = slice(1, n)
        div[tuple(sl_lo)] += flux   # the face above cell f brings +flux
        div[tuple(sl_hi)] -= flux   # the same face below cell f+1 brings -flux
        out -= div
    return alpha * out


def cell_volume(shape, dx: float) -> float:
    """dx^dims: dx^2 in the 2D (z, x) mode (ny == 1), dx^3 otherwise."""
    return dx ** 2 if shape[1] == 1 else dx ** 3


def prior_cost_grad(c, c0, alpha, theta, dx):
    """R = 1/2 dx^dims ||A (c - c0)||^2 and grad R = dx^dims A A (c - c0)."""
    vol = cell_volume(c.shape, dx)
    w = prior_operator(np.asarray(c, np.float64) - c0, alpha, theta, dx)
    return 0.5 * vol * float(np.sum(w * w)), vol * prior_operator(w, alpha, theta, dx)


def prior_hessvec(dc, alpha, theta, dx):
    """dx^dims A A dc."""
    vol = cell_volume(dc.shape, dx)
    return vol * prior_operator(prior_operator(dc, alpha, theta, dx), alpha, theta, dx)


def prior_solve(b, alpha, theta, dx):
    """A^-1 b, exactly: the cell-centred cosine modes diagonalise A (the
    orthonormal type-II DCT along each axis), with eigenvalues
    alpha (1 + sum_a theta_a / dx^2 (2 - 2 cos(pi k_a / n_a)))."""
    from scipy.fft import dctn, idctn

    b = np.asarray(b, np.float64)
    lam = np.full(b.shape, 1.0)
    for axis, n in enumerate(b.shape):
        if n == 1:
            continue
        sh = [1, 1, 1]
        sh[axis] = n
        k = np.arange(n).reshape(sh)
        lam = lam + float(theta[axis]) / dx ** 2 * (2.0 - 2.0 * np.cos(np.pi * k / n))
    return idctn(dctn(b, type=2, norm="ortho") / (alpha * lam), type=2, norm="ortho")


def prior_covariance(r, alpha, theta, dx):
    """The prior covariance applied to r: (dx^dims A A)^-1 r, the preconditioner
    of the Newton system."""
    return prior_solve(prior_solve(r, alpha, theta, dx), alpha, theta, dx) / cell_volume(r.shape, dx)


def prior_sample(w, c0, alpha, theta, dx):
    """A draw from the prior N(c0, (dx^dims A A)^-1) for white noise w ~ N(0, I):
    c = c0 + A^-1 w / sqrt(dx^dims) (covariance A^-1 A^-1 / dx^dims, A symmetric)."""
    w = np.asarray(w, np.float64)
    return c0 + prior_solve(w / np.sqrt(cell_volume(w.shape, dx)), alpha, theta, dx)


@dataclass
class NewtonConfig:
    max_newton: int = 5
    max_cg: int = 10
    eta_max: float = 0.5
    rel_tol: float = 1e-6
    c_armijo: float = 1e-4
    max_backtrack: int = 10


@dataclass
class NewtonRecord:
    cost: float
    gnorm: float
    cg_iters: int = 0
    neg_curv: bool = False
    backtracks: int = 0
    step: float = 0.0
    cg_rel_res: float = 0.0


def cg_steihaug(hv: Callable[[np.ndarray], np.ndarray], g: np.ndarray, eta: float, max_cg: int,
                prec: Callable[[np.ndarray], np.ndarray] = None):
    """Approximate solve of H p = -g from p = 0: conjugate gradients, preconditioned
    by prec (symmetric positive definite, M ~ H^-1; None: M = I), with the forcing
    eta on the M-norm of the residual, ||r||_M = sqrt(r.Mr), and the
    negative-curvature stop (at the first iteration the direction d = -M g itself
    is taken). Returns p, iterations, whether non-positive curvature ended it, and
    ||r||_M / ||g||_M."""
    M = prec if prec is not None else (lambda v: v)
    p = np.zeros_like(g)
    r = -g
    z = M(r)
    d = z.copy()
    rz = float(np.sum(r * z))
    r0 = np.sqrt(rz)
    if r0 == 0.0:
        return p, 0, False, 0.0
    it = 0
    while it < max_cg:
        Hd = hv(d)
        dHd = float(np.sum(d * Hd))
        it += 1
        if dHd <= 0.0:
            if it == 1:
                p = d.copy()
            return p, it, True, np.sqrt(rz) / r0
        a = rz / dHd
        p = p + a * d
        r = r - a * Hd
        z = M(r)
        rz_new = float(np.sum(r * z))
        if np.sqrt(rz_new) <= eta * r0:
            return p, it, False, np.sqrt(rz_new) / r0
        d = z + (rz_new / rz) * d
        rz = rz_new
    return p, it, False, np.sqrt(rz) / r0


def newton_cg(cost_grad: Callable, hessvec: Callable, c: np.ndarray, cfg: NewtonConfig,
              prec: Callable[[np.ndarray], np.ndarray] = None):
    """Inexact Newton-CG with Armijo backtracking. cost_grad(c) -> (J, g, state);
    hessvec(state, v) -> H v at the point whose state it is; prec: the CG
    preconditioner (None: none). Returns the final c, the per-iteration records
    and the reason it stopped (0: iteration limit, 1: gradient tolerance, 2: line
    search failed)."""
    c = np.asarray(c, np.float64).copy()
    J, g, st = cost_grad(c)
    g0 = np.sqrt(float(np.sum(g * g)))
    log: List[NewtonRecord] = [NewtonRecord(J, g0)]
    for _ in range(cfg.max_newton):
        gn = log[-1].gnorm
        if gn <= cfg.rel_tol * g0:
            return c, log, 1
        eta = min(cfg.eta_max, np.sqrt(gn / g0))
        p, its, neg, rel = cg_steihaug(lambda v: hessvec(st, v), g, eta, cfg.max_cg, prec)
        gp = float(np.sum(g * p))
        a = 1.0
        for bt in range(cfg.max_backtrack + 1):
            ct = c + a * p
            Jt, gt, stt = cost_grad(ct)
            if Jt is not None and Jt <= J + cfg.c_armijo * a * gp:
                break
            a *= 0.5
        else:
            rec = log[-1]
            rec.cg_iters, rec.neg_curv, rec.backtracks, rec.cg_rel_res = its, neg, cfg.max_backtrack + 1, rel
            return c, log, 2
        rec = log[-1]
        rec.cg_iters, rec.neg_curv, rec.backtracks, rec.step, rec.cg_rel_res = its, neg, bt, a, rel
        c, J, g, st = ct, Jt, gt, stt
        log.append(NewtonRecord(J, np.sqrt(float(np.sum(g * g)))))
    return c, log, 0


def wave_map_problem(sol, wavelet, src, rec, d_obs, sigma, c0, alpha, theta, gauss_newton=True,
                     src_w=None):
    """cost_grad and hessvec of the MAP objective for the wave solver of
    oracle.wave (misfit + BiLaplacian prior); a trial speed that leaves the
    leapfrog stability range or is not positive costs None (rejected)."""
    from . import wave as ow

    dims = 2 if sol.shape[1] == 1 else 3

    def cost_grad(c):
        if not np.all(c > 0) or np.max(c) * sol.dt / sol.dx >= 1.0 / np.sqrt(dims):
            return None, None, None
        Jm, gm, traces, e_hist = ow.gradient(sol, c, wavelet, src, rec, d_obs, sigma, src_w=src_w)
        R, gR = prior_cost_grad(c, c0, alpha, theta, sol.dx)
        _, resid = ow.misfit(sol, traces, d_obs, sigma)
        return Jm + R, gm + gR, (c, e_hist, resid)

    def hessvec(state, v):
        c, e_hist, resid = state
        if gauss_newton:
            Hm = ow.hessvec_gn(sol, c, v, e_hist, rec, sigma)
        else:
            Hm = ow.hessvec_full(sol, c, v, e_hist, resid, rec, sigma)
        return Hm + prior_hessvec(v, alpha, theta, sol.dx)

    return cost_grad, hessvec
