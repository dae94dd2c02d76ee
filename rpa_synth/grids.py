"""Non-uniform imaginary time / frequency grids and cosine-transform weights.

The paper takes its minimax grids and L2-fitted transform coefficients from an
external library (Sec. 2, RPA correlation energy).  That library is not
available here, so the grids are generated from their defining fits:

* tau grid: tau_j, sigma_j such that sum_j sigma_j exp(-x tau_j) approximates 1/x
  with small relative error on x in [1, R] (R = E_max / E_min);
* omega grid: omega_k, w_k such that (4/pi) sum_k w_k x^3/(x^2+omega_k^2)^2
  approximates 1 with small relative error on [1, R] (the integrand of the
  second-order term of the frequency integral, whose exact integral is pi/4);
* cosine weights: Gamma_kj = gamma_kj cos(omega_k tau_j) from a linear L2 fit of
  sum_j Gamma_kj exp(-x tau_j) to 2x/(x^2+omega_k^2) uniformly in ln x.

Each fit starts from a sinc (trapezoid in log variable) quadrature and is
refined by nonlinear least squares.  The grids are inputs shared by every
code path, so their quality changes the answer but never the parity between
paths; their errors are returned for reporting.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import least_squares


def _xs(R, n=2400):
    return np.exp(np.linspace(0.0, np.log(R), n))


def _tau_init(n, R):
    # 1/x = int_0^inf exp(-x t) dt, t = exp(s): trapezoid in s
    smin, smax = np.log(0.02 / R), np.log(20.0)
    s = np.linspace(smin, smax, n)
    h = s[1] - s[0]
    t = np.exp(s)
    return t, h * t


def fit_tau(n, R):
    x = _xs(R, 500)
    t0, w0 = _tau_init(n, R)

    def res(p):
        with np.errstate(over="ignore", invalid="ignore"):
            t, w = np.exp(p[:n]), np.exp(p[n:])
            r = x * (np.exp(-np.outer(x, t)) @ w) - 1.0
        return np.nan_to_num(r, nan=1e6, posinf=1e6, neginf=-1e6)

    p0 = np.concatenate([np.log(t0), np.log(w0)])
    # tau <= 30 / E_min: beyond it exp(-x tau) < 1e-13 for every transition energy, so a point
    # there would only carry rounding noise
    lo = np.concatenate([np.full(n, np.log(1e-4 / R)), np.full(n, np.log(1e-8 / R))])
    hi = np.concatenate([np.full(n, np.log(30.0)), np.full(n, np.log(100.0))])
    sol = least_squares(res, np.clip(p0, lo + 1e-9, hi - 1e-9), bounds=(lo, hi), method="trf",
                        xtol=1e-12, ftol=1e-12, gtol=1e-12, max_nfev=400)
    t, w = np.exp(sol.x[:n]), np.exp(sol.x[n:])
    order = np.argsort(t)
    t, w = t[order], w[order]
    x = _xs(R)
    err = np.max(np.abs(x * (np.exp(-np.outer(x, t)) @ w) - 1.0))
    return t, w, err


def _omega_init(n, R):
    # (4/pi) int_0^inf x^3/(x^2+w^2)^2 dw = 1 ; w = exp(s)
    smin, smax = np.log(0.05), np.log(20.0 * R)
    s = np.linspace(smin, smax, n)
    h = s[1] - s[0]
    om = np.exp(s)
    return om, h * om


def fit_omega(n, R):
    x = _xs(R, 500)
    o0, w0 = _omega_init(n, R)

    def model(o, w):
        X = x[:, None]
        return (4.0 / np.pi) * ((X ** 3) / (X ** 2 + o[None, :] ** 2) ** 2) @ w

    def res(p):
        with np.errstate(over="ignore", invalid="ignore"):
            r = model(np.exp(p[:n]), np.exp(p[n:])) - 1.0
        return np.nan_to_num(r, nan=1e6, posinf=1e6, neginf=-1e6)

    p0 = np.concatenate([np.log(o0), np.log(w0)])
    lo = np.concatenate([np.full(n, np.log(1e-3)), np.full(n, np.log(1e-6))])
    hi = np.concatenate([np.full(n, np.log(1e3 * R)), np.full(n, np.log(1e3 * R))])
    sol = least_squares(res, np.clip(p0, lo + 1e-9, hi - 1e-9), bounds=(lo, hi), method="trf",
                        xtol=1e-12, ftol=1e-12, gtol=1e-12, max_nfev=400)
    o, w = np.exp(sol.x[:n]), np.exp(sol.x[n:])
    order = np.argsort(o)
    o, w = o[order], w[order]
    x = _xs(R)
    err = np.max(np.abs(model(o, w) - 1.0))
    return o, w, err


def fit_cosine_weights(tau, omega, R, nx=2400, ridge=1e-6):
    """Gamma[k, j] minimising int d(ln x) [sum_j Gamma_kj e^{-x tau_j} - 2x/(x^2+omega_k^2)]^2
    over x in [1, R] (all quantities in units of E_min), plus ridge^2 |Gamma_k|^2.

    The unregularised fit is ill-conditioned (sum_j |Gamma_kj| reaches 1e5 at 16
    points); the small ridge term keeps it near 10 at a slightly larger fit error,
    so that rounding errors of chi0(tau) are not amplified by the transform."""
    x = _xs(R, nx)
    E = np.exp(-np.outer(x, tau))                        # (nx, ntau)
    n = len(tau)
    A = np.vstack([E, ridge * np.sqrt(nx) * np.eye(n)])
    Gam = np.empty((len(omega), n))
    for k, om in enumerate(omega):
        f = 2.0 * x / (x ** 2 + om ** 2)
        Gam[k], *_ = np.linalg.lstsq(A, np.concatenate([f, np.zeros(n)]), rcond=None)
    return Gam


def transform_error_bound(tau, omega, Gam, emin, emax, nx=20000):
    """eta_k = max over x in [emin, emax] of |sum_j Gam_kj e^{-x tau_j} - 2x/(x^2+omega_k^2)|
    (physical units)."""
    x = np.exp(np.linspace(np.log(emin), np.log(emax), nx))
    E = np.exp(-np.outer(x, tau))
    target = 2.0 * x[None, :] / (x[None, :] ** 2 + omega[:, None] ** 2)
    return np.max(np.abs(Gam @ E.T - target), axis=1)


def make_grids(n, emin, emax):
    """Grids for n points on transition energies [emin, emax] (Hartree).

    Returns dict with tau (1/Ha), omega (Ha), womega (Ha; the frequency quadrature
    weights), gamma_cos (Gamma_kj, 1/Ha... dimension of 1/energy), and the fit errors."""
    R = emax / emin
    t, sig, et = fit_tau(n, R)
    o, w, eo = fit_omega(n, R)
    Gam = fit_cosine_weights(t, o, R)
    tau = t / emin
    omega = o * emin
    womega = w * emin
    gamma_cos = Gam / emin
    eta = transform_error_bound(tau, omega, gamma_cos, emin, emax)
    return dict(tau=tau, omega=omega, womega=womega, gamma_cos=gamma_cos,
                tau_fit_err=et, omega_fit_err=eo, eta=eta, emin=emin, emax=emax)
