"""Conjugate gradients on the pattern Lippmann-Schwinger system (oracle; test infrastructure only).

The paper names accelerated FFT schemes beside the Basic Scheme (Sec. 1 and
the conclusion of Sec. 6) without writing one out.  This module states the
conjugate-gradient scheme on the same discrete problem as Algorithm 1, so
that its converged solution is the one the Basic Scheme converges to.

Discrete problem (Sec. 3.1-3.2, collocation on P(M)): find eps = eps_bar + x
with x a compatible strain field of zero mean (x = Gamma0 C0 x) such that the
stress sigma = C : eps is in equilibrium, i.e. Gamma0 * sigma = 0 (every
active frequency h != 0 has sigma_hat_h xi_h = 0).  With the operator
    A x = Gamma0 * (C : x)           (maps into compatible zero-mean fields)
this is the linear system A x = b, b = -Gamma0 * (C : eps_bar).

Inner product: <u, v>_C0 = sum_y u_y : C0 : v_y over the pattern points.
Gamma0 C0 is the C0-orthogonal projection onto compatible zero-mean fields
(Gamma0 C0 Gamma0 = Gamma0 per active frequency; the Hermitian rule keeps the
field-level operator a projection), hence for compatible u, v
    <u, A v>_C0 = <Gamma0 C0 u, C v> = sum_y u_y : C_y : v_y,
which is symmetric and positive definite when every C_y is: conjugate
gradients in the C0 inner product apply.

Iteration (textbook CG, x_0 = 0 or a given compatible start): r_0 = b - A x_0,
p_0 = r_0; for k = 0, 1, ...: evaluate the equilibrium residual of
eps_k = eps_bar + x_k (the same r(n) as the Basic Scheme, from the forward
transform of sigma_k); stop if r(k) <= tol; q = A p_k,
alpha = <r_k, r_k>_C0 / <p_k, q>_C0, x_{k+1} = x_k + alpha p_k,
r_{k+1} = r_k - alpha q, beta = <r_{k+1}, r_{k+1}>_C0 / <r_k, r_k>_C0,
p_{k+1} = r_{k+1} + beta p_k.  n = the number of updates performed.

All arithmetic is FP64 on full d x d tensors, through the oracle's own
transforms and Gamma0 (``elasticity.gamma0_apply``), no recurrence for the
residual or the mean stress.
"""
from __future__ import annotations

import math

import numpy as np

from .dft import make_transform
from .elasticity import (SchemeResult, active_classes, apply_phases, contract, equilibrium_residual, gamma0_apply,
                         iso_tensor, to_mandel, unit_loads, wave_vectors)
from .lattice import as_int_matrix


class LSOperator:
    """A x = Gamma0 * (C : x) on P(M) (or P_L(M)), with its C0 inner product."""

    def __init__(self, M, phase, lame, lame0, transform=None, rule="hermitian", cell=None):
        self.T = transform or make_transform(M)
        self.d = len(as_int_matrix(M))
        H = np.asarray(self.T.freqs, dtype=np.int64)
        self.K = wave_vectors(H, cell)
        self.zero = np.flatnonzero(np.all(H == 0, axis=1))[0]
        self.active = active_classes(M, H, rule)
        self.upd = self.active.copy()
        self.upd[self.zero] = False
        self.tensors = [iso_tensor(l, mu, self.d) for l, mu in np.asarray(lame, dtype=np.float64)]
        self.C0 = iso_tensor(lame0[0], lame0[1], self.d)
        self.phase = np.asarray(phase)

    def stress(self, eps):
        return apply_phases(self.tensors, self.phase, eps)

    def gamma(self, tau):
        """Gamma0 * tau (zero mean, zero on the unpaired classes), real field."""
        th = self.T.forward(tau)
        out = np.zeros_like(th)
        out[:, :, self.upd] = -gamma0_apply(self.C0, self.K[self.upd], th[:, :, self.upd])
        g = self.T.inverse(out)
        assert np.max(np.abs(g.imag)) <= 1e-9 * max(1.0, np.max(np.abs(g.real)))
        return g.real

    def apply(self, x):
        return self.gamma(self.stress(x))

    def project(self, w):
        """Gamma0 C0 w: the compatible zero-mean part of w."""
        return self.gamma(contract(self.C0, w))

    def inner(self, u, v):
        """<u, v>_C0 = sum over points of u : C0 : v."""
        return float(np.sum(u * contract(self.C0, v)))

    def residual(self, eps):
        """Equilibrium residual r of eps and its mean stress (as the Basic Scheme reports them)."""
        sigma = self.stress(eps)
        r = equilibrium_residual(self.T.forward(sigma), self.K, self.active, self.zero)
        return r, np.sum(sigma, axis=2) / self.T.m


def conjugate_gradient(M, phase, lame, lame0, eps_bar, tol=1e-8, max_iter=1000, init=None, transform=None,
                       rule="hermitian", fixed_iters=None, cell=None, op=None):
    """CG on A x = b (module docstring); returns a SchemeResult like ``elasticity.basic_scheme``.

    init: optional (d, d, m) start x_0, which must be compatible with zero
    mean (e.g. ``LSOperator.project`` of any field).  fixed_iters: run exactly
    this many updates, ignoring tol.
    """
    A = op or LSOperator(M, phase, lame, lame0, transform=transform, rule=rule, cell=cell)
    d, m = A.d, A.T.m
    ebar = np.broadcast_to(np.asarray(eps_bar, dtype=np.float64)[:, :, None], (d, d, m))
    x = np.zeros((d, d, m)) if init is None else np.array(init, dtype=np.float64)
    r = -A.apply(ebar) - A.apply(x)
    p = r.copy()
    rr = A.inner(r, r)
    hist = []
    n = 0
    r0 = None
    while True:
        eps = ebar + x
        res, mean = A.residual(eps)
        hist.append(res)
        r0 = res if r0 is None else r0
        if not math.isfinite(res) or (r0 > 0 and res > 1e3 * r0):
            return SchemeResult(eps, n, res, 2, mean, hist)
        if fixed_iters is None and res <= tol:
            return SchemeResult(eps, n, res, 0, mean, hist)
        if n == (fixed_iters if fixed_iters is not None else max_iter):
            return SchemeResult(eps, n, res, 0 if fixed_iters is not None else 1, mean, hist)
        q = A.apply(p)
        alpha = rr / A.inner(p, q)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = A.inner(r, r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        n += 1


def effective_stiffness_cg(M, phase, lame, lame0, tol=1e-10, max_iter=2000, transform=None, rule="hermitian", cell=None):
    """C_eff in Mandel form from CG solves of the unit loads (Def. 3.1)."""
    A = LSOperator(M, phase, lame, lame0, transform=transform, rule=rule, cell=cell)
    cols, runs = [], []
    for E in unit_loads(A.d):
        res = conjugate_gradient(M, phase, lame, lame0, E, tol=tol, max_iter=max_iter, op=A)
        cols.append(to_mandel(res.mean_stress))
        runs.append(res)
    return np.array(cols).T, runs


def krylov_galerkin(op, eps_bar, k):
    """The minimiser of the energy J(x) = 1/2 <x, A x>_C0 - <b, x>_C0 over the
    Krylov space span{b, A b, ..., A^{k-1} b}, from an explicit C0-orthonormal
    basis (Gram-Schmidt twice) and a dense k x k solve: what the k-th CG
    iterate from x_0 = 0 equals in exact arithmetic."""
    d, m = op.d, op.T.m
    ebar = np.broadcast_to(np.asarray(eps_bar, dtype=np.float64)[:, :, None], (d, d, m))
    b = -op.apply(ebar)
    basis = []
    v = b
    for _ in range(k):
        w = v.copy()
        for _ in range(2):
            for u in basis:
                w = w - op.inner(u, w) * u
        nrm = math.sqrt(op.inner(w, w))
        basis.append(w / nrm)
        v = op.apply(basis[-1])
    G = np.array([[op.inner(u, op.apply(v)) for v in basis] for u in basis])
    rhs = np.array([op.inner(u, b) for u in basis])
    c = np.linalg.solve(G, rhs)
    return sum(ci * u for ci, u in zip(c, basis))
