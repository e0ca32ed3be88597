"""FP64 reference solver: forward, misfit, exact discrete adjoint, gradient,
incremental forward and Hessian-vector products.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Continuous model (paper Sec. 2, Eq. (model), density 1):
    dv/dt - grad(c^2 e) = b,    de/dt - div v = 0,
zero initial state, traction-free (e = 0) top surface; the PtO map samples
the vertical velocity at receivers (Sec. 2, F = B A); the data-misfit part
of the MAP objective is (1/2) ||F(c) - d||^2 with noise covariance
sigma^2 I (Sec. 2, MAP objective).

Discretisation (the paper's DG/RK4 solver is replaced by a 2nd-order
staggered grid with leapfrog; its derivation of the discrete adjoint is
deferred to its references, so the adjoint here is the exact transpose of
the discrete forward map, the "discretely exact" choice Sec. 2 cites):
  * cells (k, j, i), k = depth index with k = 0 at the free surface;
    e at cell centres, v_z[k] on the face between cells k-1 and k, v_y and
    v_x likewise in j and i. All arrays are [nz, ny, nx]; ny == 1 is the
    2D (z, x) mode, which has no y terms at all.
  * (G_a q)[i] = (q[i] - q[i-1]) / dx with q[-1] = 0 (e = 0 outside the low
    faces), (D v)[i] = sum_a (v_a[i+1] - v_a[i]) / dx with v_a[n_a] = 0;
    G_a = -D_a^T. Periodic mode wraps both.
  * one step n -> n+1 (v^n lives at t_{n-1/2}, e^n at t_n):
        v_a <- S_va * (v_a + dt G_a(m e) + dt b_a^n),  m = c^2
        e   <- S_e  * (e + dt D v)
        p^{n+1}_r = v_z[rec_r]
  * absorbing layer: S = exp(-dt * sum of axis profiles); each absorbing
    side adds sigma_max ((N - w)/N)^2 where w < N is the node's distance in
    cells from the outer edge (cell centre for e, face for v_a along a),
    sigma_max = 3 c_ref ln(1/R) / (2 N dx), R = 1e-3. The top (k = 0) side
    is the free surface and has no layer.
  * misfit J = dt / (2 sigma^2) sum_{n=1..T} sum_r (p^n_r - d^n_r)^2.
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

R_TARGET = 1e-3


class Solver:
    """Grid, time step and absorbing-layer factors of one discretisation."""

    def __init__(self, nz: int, ny: int, nx: int, dx: float, dt: float, nt: int,
                 sponge: int = 16, c_ref: float = 1.0, periodic: bool = False):
        self.shape = (nz, ny, nx)
        self.dx, self.dt, self.nt = float(dx), float(dt), int(nt)
        self.periodic = bool(periodic)
        self.sponge = 0 if periodic else int(sponge)
        self.c_ref = float(c_ref)
        self.axes: Tuple[int, ...] = (0, 2) if ny == 1 else (0, 1, 2)
        self._build_sponge()

    # ----- absorbing layer -------------------------------------------------
    def _axis_sigma(self, axis: int, faces: bool) -> np.ndarray:
        n = self.shape[axis]
        ns = self.sponge
        out = np.zeros(n)
        if ns == 0 or axis not in self.axes:
            return out
        smax = 3.0 * self.c_ref * math.log(1.0 / R_TARGET) / (2.0 * ns * self.dx)
        pos = np.arange(n, dtype=np.float64) + (0.0 if faces else 0.5)
        sides = []
        if axis != 0:                 # low side of y and x absorbs; low z is the free surface
            sides.append(pos)
        sides.append(n - pos)         # high side of every axis absorbs
        for w in sides:
            inside = w < ns
            out[inside] += smax * ((ns - w[inside]) / ns) ** 2
        return out

    def _build_sponge(self):
        dt = self.dt
        centre = [self._axis_sigma(a, False) for a in range(3)]
        face = [self._axis_sigma(a, True) for a in range(3)]

        def total(prof):
            return (prof[0][:, None, None] + prof[1][None, :, None] + prof[2][None, None, :])

        self.S_e = np.exp(-dt * total(centre))
        self.S_v = {}
        for a in self.axes:
            prof = [face[b] if b == a else centre[b] for b in range(3)]
            self.S_v[a] = np.exp(-dt * total(prof))

    # ----- difference operators --------------------------------------------
    def G(self, q: np.ndarray, a: int) -> np.ndarray:
        if self.periodic:
            return (q - np.roll(q, 1, axis=a)) / self.dx
        out = q.copy()
        sl_hi = [slice(None)] * 3
        sl_lo = [slice(None)] * 3
        sl_hi[a] = slice(1, None)
        sl_lo[a] = slice(None, -1)
        out[tuple(sl_hi)] -= q[tuple(sl_lo)]
        return out / self.dx

    def D(self, v: dict) -> np.ndarray:
        out = np.zeros(self.shape)
        for a in self.axes:
            va = v[a]
            if self.periodic:
                out += np.roll(va, -1, axis=a) - va
            else:
                out -= va
                sl_hi = [slice(None)] * 3
                sl_lo = [slice(None)] * 3
                sl_hi[a] = slice(1, None)
                sl_lo[a] = slice(None, -1)
                out[tuple(sl_lo)] += va[tuple(sl_hi)]
        return out / self.dx

    # ----- one step and its transpose ---------------------------------------
    def zero_v(self) -> dict:
        return {a: np.zeros(self.shape) for a in self.axes}

    def step(self, v: dict, e: np.ndarray, m: np.ndarray, force: Optional[Tuple] = None,
             extra: Optional[np.ndarray] = None):
        """One leapfrog step. `force` = ((k, j, i), b, w) adds dt*b*w to v_z on
        the faces of the box of half-width R = (w.shape[0]-1)/2 centred at
        (k, j, i), truncated at the grid boundary (w = None: point force);
        `extra` is an additional field inside G (used by the incremental
        forward for the dm * e term)."""
        q = m * e if extra is None else m * e + extra
        vn = {}
        for a in self.axes:
            g = self.G(q, a)
            if a == 0 and force is not None:
                (k, j, i), b, w = force
                if w is None:
                    g[k, j, i] += b
                else:
                    self._add_box(g, (k, j, i), b * w)
            vn[a] = self.S_v[a] * (v[a] + self.dt * g)
        en = self.S_e * (e + self.dt * self.D(vn))
        return vn, en

    def _add_box(self, g: np.ndarray, centre, vals: np.ndarray):
        lo, src = [], []
        for ax in range(3):
            r = (vals.shape[ax] - 1) // 2
            a0 = centre[ax] - r
            s0 = max(0, -a0)
            s1 = vals.shape[ax] - max(0, a0 + vals.shape[ax] - self.shape[ax])
            lo.append(slice(a0 + s0, a0 + s1))
            src.append(slice(s0, s1))
        g[tuple(lo)] += vals[tuple(src)]

    def step_T(self, mu: dict, eta: np.ndarray, m: np.ndarray):
        """Transpose of the linear map (v^n, e^n) -> (v^{n+1}, e^{n+1}) of
        `step`: takes adjoints (mu, eta) of (v^{n+1}, e^{n+1}) and returns the
        adjoints of (v^n, e^n) together with q = D(S_v muhat), where muhat is
        the total adjoint of v^{n+1}; the m-derivative of the step paired
        with w is -dt * e^n * q."""
        se_eta = self.S_e * eta
        muhat = {a: mu[a] - self.dt * self.G(se_eta, a) for a in self.axes}
        svmu = {a: self.S_v[a] * muhat[a] for a in self.axes}
        q = self.D(svmu)
        eta_n = se_eta - self.dt * m * q
        return svmu, eta_n, q


def _rec_index(rec: np.ndarray):
    rec = np.asarray(rec)
    return (rec[:, 0], rec[:, 1], rec[:, 2])


def forward(sol: Solver, c: np.ndarray, wavelet: np.ndarray, src: np.ndarray, rec: np.ndarray,
            store_e: bool = True, store_v: bool = False, src_w: Optional[np.ndarray] = None):
    """Forward solve for every source. Returns traces [S, T, R] (traces[s, n]
    = p^{n+1}) and, if requested, e history [S, T+1, ...] (index n = e^n) and
    the final states. src_w: spatial weights of every source (None: point)."""
    m = c * c
    T = sol.nt
    S = len(src)
    ri = _rec_index(rec)
    traces = np.zeros((S, T, len(rec)))
    e_hist = np.zeros((S, T + 1) + sol.shape) if store_e else None
    v_hist = [] if store_v else None
    finals = []
    for s in range(S):
        v, e = sol.zero_v(), np.zeros(sol.shape)
        ks, js, is_ = (int(x) for x in src[s])
        vs = [] if store_v else None
        for n in range(T):
            v, e = sol.step(v, e, m, force=((ks, js, is_), wavelet[s, n], src_w))
            traces[s, n] = v[0][ri]
            if store_e:
                e_hist[s, n + 1] = e
            if store_v:
                vs.append({a: v[a].copy() for a in sol.axes})
        finals.append((v, e))
        if store_v:
            v_hist.append(vs)
    return traces, e_hist, finals, v_hist


def misfit(sol: Solver, traces: np.ndarray, d_obs: np.ndarray, sigma: float):
    """J = dt/(2 sigma^2) sum (p - d)^2 and the adjoint source dt/sigma^2 (p - d)."""
    diff = traces - d_obs
    J = sol.dt / (2.0 * sigma * sigma) * float(np.sum(diff * diff))
    return J, (sol.dt / (sigma * sigma)) * diff


def adjoint_acc(sol: Solver, c: np.ndarray, e_hist_s: np.ndarray, resid_s: np.ndarray,
                rec: np.ndarray, de_hist_s: Optional[np.ndarray] = None,
                dresid_s: Optional[np.ndarray] = None, dm: Optional[np.ndarray] = None):
    """Backward sweep k = T..1 for one source. Returns acc = sum_n e^n * q^n
    (so dJ/dm = -dt acc). With the incremental arguments it also runs the
    linearised adjoint and returns dacc = sum_n (de^n q^n + e^n dq^n)."""
    m = c * c
    T = sol.nt
    ri = _rec_index(rec)
    mu, eta = sol.zero_v(), np.zeros(sol.shape)
    acc = np.zeros(sol.shape)
    second = de_hist_s is not None
    if second:
        dmu, deta = sol.zero_v(), np.zeros(sol.shape)
        dacc = np.zeros(sol.shape)
    for k in range(T, 0, -1):
        np.add.at(mu[0], ri, resid_s[k - 1])
        mu, eta_new, q = sol.step_T(mu, eta, m)
        acc += e_hist_s[k - 1] * q
        if second:
            np.add.at(dmu[0], ri, dresid_s[k - 1])
            dmu, deta_new, dq = sol.step_T(dmu, deta, m)
            deta_new -= sol.dt * dm * q
            dacc += de_hist_s[k - 1] * q + e_hist_s[k - 1] * dq
            deta = deta_new
        eta = eta_new
    return (acc, dacc) if second else acc


def gradient(sol: Solver, c: np.ndarray, wavelet: np.ndarray, src, rec, d_obs, sigma: float,
             src_w: Optional[np.ndarray] = None):
    """Misfit J and dJ/dc = -2 dt c * sum_s acc_s (summed over sources)."""
    traces, e_hist, _, _ = forward(sol, c, wavelet, src, rec, src_w=src_w)
    J, resid = misfit(sol, traces, d_obs, sigma)
    acc = np.zeros(sol.shape)
    for s in range(len(src)):
        acc += adjoint_acc(sol, c, e_hist[s], resid[s], rec)
    return J, -2.0 * sol.dt * c * acc, traces, e_hist


def inc_forward(sol: Solver, c: np.ndarray, dc: np.ndarray, e_hist_s: np.ndarray, rec,
                store_e: bool = False):
    """Linearised forward in direction dc (dm = 2 c dc): returns dp [T, R]
    and optionally the de history."""
    m = c * c
    dm = 2.0 * c * dc
    T = sol.nt
    ri = _rec_index(rec)
    dv, de = sol.zero_v(), np.zeros(sol.shape)
    dp = np.zeros((T, len(rec)))
    de_hist = np.zeros((T + 1,) + sol.shape) if store_e else None
    for n in range(T):
        dv, de = sol.step(dv, de, m, extra=dm * e_hist_s[n])
        dp[n] = dv[0][ri]
        if store_e:
            de_hist[n + 1] = de
    return dp, de_hist


def hessvec_gn(sol: Solver, c, dc, e_hist, rec, sigma: float):
    """Gauss-Newton H dc = J_F^T (dt/sigma^2) J_F dc, summed over sources."""
    acc = np.zeros(sol.shape)
    for s in range(e_hist.shape[0]):
        dp, _ = inc_forward(sol, c, dc, e_hist[s], rec)
        acc += adjoint_acc(sol, c, e_hist[s], (sol.dt / sigma ** 2) * dp, rec)
    return -2.0 * sol.dt * c * acc


def hessvec_full(sol: Solver, c, dc, e_hist, resid, rec, sigma: float):
    """Full-Newton H dc: derivative of the gradient along dc,
    -2 dt (dc * acc + c * dacc)."""
    dm = 2.0 * c * dc
    acc = np.zeros(sol.shape)
    dacc = np.zeros(sol.shape)
    for s in range(e_hist.shape[0]):
        dp, de_hist = inc_forward(sol, c, dc, e_hist[s], rec, store_e=True)
        a, da = adjoint_acc(sol, c, e_hist[s], resid[s], rec, de_hist_s=de_hist,
                            dresid_s=(sol.dt / sigma ** 2) * dp, dm=dm)
        acc += a
        dacc += da
    return -2.0 * sol.dt * (dc * acc + c * dacc)


def solver_for(problem, periodic: bool = False) -> Solver:
    """Solver for a `workloads.Problem`."""
    return Solver(problem.nz, problem.ny, problem.nx, problem.dx, problem.dt, problem.nt,
                  sponge=problem.sponge, c_ref=problem.c_ref, periodic=periodic)


def observed_data(sol: Solver, problem, noise_level: Optional[float] = None):
    """d = F(c_true) + sigma xi, sigma = noise_level * max|F(c_true)| (per run)."""
    lvl = problem.noise_level if noise_level is None else noise_level
    clean, _, _, _ = forward(sol, problem.c_true, problem.wavelet, problem.src, problem.rec,
                             store_e=False, src_w=problem.src_w)
    sigma = lvl * float(np.max(np.abs(clean)))
    if sigma == 0.0:
        sigma = 1.0
    return clean + sigma * problem.noise, sigma, clean


def energy(sol: Solver, v: dict, e: np.ndarray, m: np.ndarray) -> float:
    """Discrete energy |v|^2 + e^T M e - dt e^T M D v, conserved exactly by
    the leapfrog step without source and absorbing layer."""
    dv = sol.D(v)
    return float(sum(np.sum(v[a] * v[a]) for a in sol.axes) + np.sum(m * e * e)
                 - sol.dt * np.sum(m * e * dv))
