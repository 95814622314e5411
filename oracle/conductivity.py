"""Steady-state conductivity on patterns (oracle; test infrastructure only).

Sec. 3 names the steady-state heat equation as the other typical
homogenization problem beside quasi-static elasticity (its Sec. 3.1
construction follows the integral formulation first derived for the heat
equation) and then writes the scheme out for elasticity only.  The scalar
problem used here is the same construction one tensor order lower (a reading:
the paper prints no formula for it): the unknown is the gradient field
e = grad(theta) of a periodic potential plus a prescribed mean e_bar, the flux
is q = k(x) e, and equilibrium is div q = 0.  With a reference conductivity k0
the Lippmann-Schwinger equation reads
e = e_bar - Gamma0 * ((k - k0) e), where the Green operator of the scalar
problem acts per frequency h != 0 as
    Gamma0(h) tau_hat = h (h . tau_hat) / (h^T k0 h),
the projection of tau_hat / k0 onto the direction of h; it is homogeneous of
degree 0 in h.  Collocation at the pattern points and the Basic Scheme
(Algorithm 1) carry over unchanged: the same transform F(M), the same
generating set G(M^T) and the same Hermitian rule for unpaired classes
(``elasticity.active_classes``).

Readings (as for elasticity): the reference k0 is the mean of the extreme
phase conductivities; the stop is the equilibrium residual
    r(n) = sqrt(sum_{h active, h != 0} |q_hat(n)_h . xi_h|^2) / |q_hat(n)_0|,
xi = h / |h|; the effective conductivity K_eff has columns <q> for the unit
mean gradients; 2-D is the in-plane problem.

Everything is FP64 on full d-vectors through the oracle's own transforms;
K is solved as a scalar h^T k0 h per frequency (no shortcut).
"""
from __future__ import annotations

import math

import numpy as np

from .dft import make_transform
from .elasticity import SchemeResult, active_classes, wave_vectors
from .lattice import as_int_matrix


def flux(kvals, phase, e):
    """q_y = k_{phase(y)} e_y for e shaped (d, m)."""
    return np.asarray(kvals, dtype=np.float64)[np.asarray(phase)][None, :] * e


def gamma0_scalar(k0, H, tau_hat):
    """-Gamma0(h) tau_hat per frequency: -h (h . tau_hat) / (h^T k0 h); tau_hat (d, n), H (n, d)."""
    Hf = np.asarray(H, dtype=np.float64)
    K0 = np.eye(Hf.shape[1]) * float(k0)
    denom = np.einsum("ni,ij,nj->n", Hf, K0, Hf)
    proj = np.einsum("ni,in->n", Hf, tau_hat) / denom
    return -(Hf.T * proj[None, :])


def flux_residual(q_hat, K, active, zero):
    """r = sqrt(sum_{active, h != 0} |q_hat_h . xi_h|^2) / |q_hat_0|."""
    sel = active.copy()
    sel[zero] = False
    Hf = np.asarray(K[sel], dtype=np.float64)
    xi = Hf / np.linalg.norm(Hf, axis=1)[:, None]
    t = np.einsum("in,ni->n", q_hat[:, sel], xi)
    return math.sqrt(float(np.sum(np.abs(t) ** 2))) / float(np.linalg.norm(q_hat[:, zero]))


class ThermalProblem:
    """Pattern, phases and the per-frequency data of the conductivity problem."""

    def __init__(self, M, phase, kvals, k0, transform=None, rule="hermitian", cell=None):
        self.T = transform or make_transform(M)
        self.d = len(as_int_matrix(M))
        H = np.asarray(self.T.freqs, dtype=np.int64)
        self.K = wave_vectors(H, cell)
        self.zero = np.flatnonzero(np.all(H == 0, axis=1))[0]
        self.active = active_classes(M, H, rule)
        self.upd = self.active.copy()
        self.upd[self.zero] = False
        self.kvals = np.asarray(kvals, dtype=np.float64)
        self.k0 = float(k0)
        self.phase = np.asarray(phase)

    def ls_map(self, e, e_bar):
        """e_new = F^{-1}[ e_bar at h = 0; -Gamma0(h) ((k - k0) e)^_h on active h != 0; 0 else ]."""
        tau_hat = self.T.forward(flux(self.kvals, self.phase, e) - self.k0 * e)
        e_hat = np.zeros_like(tau_hat)
        e_hat[:, self.upd] = gamma0_scalar(self.k0, self.K[self.upd], tau_hat[:, self.upd])
        e_hat[:, self.zero] = e_bar
        new = self.T.inverse(e_hat)
        assert np.max(np.abs(new.imag)) <= 1e-9 * max(1.0, np.max(np.abs(new.real)))
        return new.real

    def residual(self, e):
        q = flux(self.kvals, self.phase, e)
        return flux_residual(self.T.forward(q), self.K, self.active, self.zero), q.sum(axis=1) / self.T.m

    # conjugate gradients: A x = Gamma0 * (k x) on compatible zero-mean fields, k0 inner product
    def gamma(self, tau):
        th = self.T.forward(tau)
        out = np.zeros_like(th)
        out[:, self.upd] = -gamma0_scalar(self.k0, self.K[self.upd], th[:, self.upd])
        g = self.T.inverse(out)
        assert np.max(np.abs(g.imag)) <= 1e-9 * max(1.0, np.max(np.abs(g.real)))
        return g.real

    def apply(self, x):
        return self.gamma(flux(self.kvals, self.phase, x))

    def project(self, w):
        return self.gamma(self.k0 * w)

    def inner(self, u, v):
        return float(self.k0 * np.sum(u * v))


def basic_scheme_thermal(M, phase, kvals, k0, e_bar, tol=1e-8, max_iter=1000, transform=None, rule="hermitian",
                         fixed_iters=None, cell=None, prob=None):
    """Algorithm 1 for the conductivity problem: Picard iteration of ``ThermalProblem.ls_map``
    from e(0) = e_bar, stopped on the flux residual of the current iterate."""
    pr = prob or ThermalProblem(M, phase, kvals, k0, transform=transform, rule=rule, cell=cell)
    e_bar = np.asarray(e_bar, dtype=np.float64)
    e = np.broadcast_to(e_bar[:, None], (pr.d, pr.T.m)).copy()
    norm0 = float(np.linalg.norm(e))
    hist, cauchy = [], []
    n = 0
    r0 = None
    while True:
        r, mean = pr.residual(e)
        hist.append(r)
        r0 = r if r0 is None else r0
        if not math.isfinite(r) or (r0 > 0 and r > 1e3 * r0):
            return SchemeResult(e, n, r, 2, mean, hist, cauchy)
        if fixed_iters is None and r <= tol:
            return SchemeResult(e, n, r, 0, mean, hist, cauchy)
        if n == (fixed_iters if fixed_iters is not None else max_iter):
            return SchemeResult(e, n, r, 0 if fixed_iters is not None else 1, mean, hist, cauchy)
        new = pr.ls_map(e, e_bar)
        cauchy.append(float(np.linalg.norm(new - e)) / norm0)     # the Sec. 5.2 measure, reported
        e = new
        n += 1


def cg_thermal(M, phase, kvals, k0, e_bar, tol=1e-8, max_iter=1000, transform=None, rule="hermitian",
               fixed_iters=None, cell=None, prob=None):
    """Conjugate gradients for the conductivity problem (the scheme of
    ``accelerated.conjugate_gradient`` with the scalar Green operator and the
    inner product k0 sum u . v)."""
    pr = prob or ThermalProblem(M, phase, kvals, k0, transform=transform, rule=rule, cell=cell)
    e_bar = np.asarray(e_bar, dtype=np.float64)
    ebar = np.broadcast_to(e_bar[:, None], (pr.d, pr.T.m))
    x = np.zeros((pr.d, pr.T.m))
    r = -pr.apply(ebar)
    p = r.copy()
    rr = pr.inner(r, r)
    hist = []
    n = 0
    r0 = None
    while True:
        e = ebar + x
        res, mean = pr.residual(e)
        hist.append(res)
        r0 = res if r0 is None else r0
        if not math.isfinite(res) or (r0 > 0 and res > 1e3 * r0):
            return SchemeResult(e, n, res, 2, mean, hist)
        if fixed_iters is None and res <= tol:
            return SchemeResult(e, n, res, 0, mean, hist)
        if n == (fixed_iters if fixed_iters is not None else max_iter):
            return SchemeResult(e, n, res, 0 if fixed_iters is not None else 1, mean, hist)
        q = pr.apply(p)
        alpha = rr / pr.inner(p, q)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = pr.inner(r, r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        n += 1


def effective_conductivity(M, phase, kvals, k0, tol=1e-10, max_iter=5000, transform=None, scheme="basic"):
    """K_eff (d x d): column j is <q> for the unit mean gradient e_j."""
    pr = ThermalProblem(M, phase, kvals, k0, transform=transform)
    run = basic_scheme_thermal if scheme == "basic" else cg_thermal
    cols, runs = [], []
    for j in range(pr.d):
        res = run(M, phase, kvals, k0, np.eye(pr.d)[j], tol=tol, max_iter=max_iter, prob=pr)
        cols.append(res.mean_stress)
        runs.append(res)
    return np.array(cols).T, runs


def default_reference_conductivity(kvals):
    """Reading: k0 = mean of the extreme phase conductivities."""
    k = np.asarray(kvals, dtype=np.float64)
    return 0.5 * (k.min() + k.max())


def laminate_conductivity(k1, k2, f1, normal):
    """Closed form of a two-phase laminate: the arithmetic mean along the layers,
    the harmonic mean across them, K = k_a (I - n n^T) + k_h n n^T."""
    n = np.asarray(normal, dtype=np.float64)
    n = n / np.linalg.norm(n)
    f2 = 1.0 - f1
    ka = f1 * k1 + f2 * k2
    kh = 1.0 / (f1 / k1 + f2 / k2)
    return ka * (np.eye(len(n)) - np.outer(n, n)) + kh * np.outer(n, n)
