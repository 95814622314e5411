"""Linear elasticity on patterns and Algorithm 1 (oracle; test infrastructure only).

Sec. 3.1: isotropic stiffness C_ijkl = lambda d_ij d_kl + mu (d_ik d_jl + d_il d_jk);
the Fourier multiplier of the symmetric gradient, Gsym_k u = (i/2)(k u^T + u k^T),
and the Lippmann-Schwinger equation in Fourier form.
Sec. 3.2: collocation at the pattern points and Algorithm 1 (fixed point on
patterns).  Def. 3.1: C_eff : eps0 is the mean stress.

All arithmetic is FP64 on full d x d tensors (no Voigt/Mandel packing inside
the iteration), so it is independent of any packing a fast implementation
uses.

Readings of the paper applied here
----------------------------------
* Green operator: Algorithm 1 and the collocation formula print the last
  factor as Gsym_h; it must be its adjoint Gsym_h^H (as in the continuous
  Fourier form).  With Gsym_h^H tau = -i tau h the operator becomes
      eps_hat = -1/2 (h v^T + v h^T),  v = K(h)^{-1} (tau_hat h),
      K(h)_ik = C0_ijkl h_j h_l,
  which is real and homogeneous of degree 0 in h.  K is solved as a general
  d x d system (no isotropic shortcut).
* Unpaired boundary frequencies (rule "hermitian", the default): a class c
  of G(M^T) is active when its representative satisfies rep(-c) = -rep(c)
  (ordinary pair) or rep(-c) = rep(c) (self-conjugate, 2c = 0).  On the
  remaining classes (some coordinate of M^{-T} h equal to -1/2 and c != -c),
  Gamma0 at rep(c) and at rep(-c) differ, so the update would not be real;
  eps_hat is set to 0 there.  Rule "literal" applies Gamma0 at every
  representative and keeps the real part of the result.
* Convergence criterion (Algorithm 1 leaves it open): the equilibrium
  residual
      r(n) = sqrt( sum_{h active, h != 0} |sigma_hat(n)_h xi_h|^2 ) / |sigma_hat(n)_0|_F,
  xi = h/|h|, with the 1/m-normalized F(M) and sigma(n) = C : eps(n).  The
  returned iterate is eps(n) for the first n with r(n) <= tol; n is the
  number of updates performed.  The Cauchy measure of Sec. 5.2,
  |eps(n+1) - eps(n)| / |eps(0)|, is reported beside it.
* Plane strain in 2-D: d = 2 tensors with the in-plane part of the 3-D
  isotropic law.
* Transformed patterns P_L(M) (Def. 3.3): the cell is L[-1/2,1/2)^d and the
  point y of P(M) sits at x = L y.  A function periodic on that cell is a
  sum of exp(2 pi i h^T L^{-1} x), so the wave vector of class h is L^{-T} h;
  Gamma0 and the residual's xi use it.  Everything else (transform, phases
  per point, means) is that of P(M).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .dft import make_transform
from .lattice import reduce_to_generating_set, transpose, as_int_matrix


# --------------------------------------------------------------------------
# material laws
# --------------------------------------------------------------------------

def lame_from_young(E, nu):
    """(lambda, mu) of an isotropic material with Young's modulus E, Poisson nu."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def iso_tensor(lam, mu, d):
    """Full 4th-order isotropic stiffness tensor (Sec. 3.1)."""
    I = np.eye(d)
    return (lam * np.einsum("ij,kl->ijkl", I, I)
            + mu * (np.einsum("ik,jl->ijkl", I, I) + np.einsum("il,jk->ijkl", I, I)))


def contract(C, eps):
    """C : eps = (C_ijkl eps_kl)_ij for eps shaped (d, d, ...)."""
    return np.einsum("ijkl,kl...->ij...", C, eps)


def apply_phases(tensors, phase, eps):
    """sigma_y = C_{phase(y)} : eps_y for eps shaped (d, d, m)."""
    out = np.zeros_like(eps)
    for p, C in enumerate(tensors):
        sel = phase == p
        if np.any(sel):
            out[:, :, sel] = contract(C, eps[:, :, sel])
    return out


# --------------------------------------------------------------------------
# Mandel notation (only for C_eff in/out)
# --------------------------------------------------------------------------

def mandel_pairs(d):
    return [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)] if d == 3 else [(0, 0), (1, 1), (0, 1)]


def to_mandel(t):
    d = t.shape[0]
    return np.array([t[i, j] * (1.0 if i == j else math.sqrt(2.0)) for i, j in mandel_pairs(d)])


def from_mandel(v, d):
    t = np.zeros((d, d))
    for k, (i, j) in enumerate(mandel_pairs(d)):
        if i == j:
            t[i, i] = v[k]
        else:
            t[i, j] = t[j, i] = v[k] / math.sqrt(2.0)
    return t


def tensor4_to_mandel(C):
    d = C.shape[0]
    pr = mandel_pairs(d)
    w = [1.0 if i == j else math.sqrt(2.0) for i, j in pr]
    return np.array([[C[i, j, k, l] * w[a] * w[b] for b, (k, l) in enumerate(pr)]
                     for a, (i, j) in enumerate(pr)])


# --------------------------------------------------------------------------
# Gamma0 on the generating set (Sec. 3.1, 3.2)
# --------------------------------------------------------------------------

def active_classes(M, H, rule="hermitian"):
    """Boolean mask over frequencies H (rows of G(M^T)) where Gamma0 is applied."""
    if rule == "literal":
        return np.ones(H.shape[0], dtype=bool)
    MT = transpose(as_int_matrix(M))
    neg = reduce_to_generating_set(MT, -np.asarray(H, dtype=object))
    return np.all(neg == -H, axis=1) | np.all(neg == H, axis=1)


def gamma0_apply(C0, H, tau_hat):
    """eps_hat = -Gsym_h (Gsym_h^H C0 Gsym_h)^{-1} Gsym_h^H tau_hat per frequency.

    tau_hat: (d, d, n) complex, H: (n, d) nonzero frequencies.
    """
    Hf = np.asarray(H, dtype=np.float64)
    K = np.einsum("ijkl,nj,nl->nik", C0, Hf, Hf)
    t = np.einsum("ijn,nj->ni", tau_hat, Hf)
    v = np.linalg.solve(K, t[..., None])[..., 0]
    out = -0.5 * (np.einsum("ni,nj->ijn", Hf, v) + np.einsum("ni,nj->ijn", v, Hf))
    return out


def equilibrium_residual(sig_hat, H, active, zero):
    """r = sqrt(sum_{active, h != 0} |sigma_hat_h xi_h|^2) / |sigma_hat_0|_F."""
    sel = active.copy()
    sel[zero] = False
    Hf = np.asarray(H[sel], dtype=np.float64)
    xi = Hf / np.linalg.norm(Hf, axis=1)[:, None]
    t = np.einsum("ijn,nj->ni", sig_hat[:, :, sel], xi)
    num = math.sqrt(float(np.sum(np.abs(t) ** 2)))
    den = float(np.linalg.norm(sig_hat[:, :, zero]))
    return num / den


# --------------------------------------------------------------------------
# Algorithm 1
# --------------------------------------------------------------------------

@dataclass
class SchemeResult:
    eps: np.ndarray            # (d, d, m) strain in the transform's point order
    iters: int                 # number of updates performed
    resid: float               # r(iters)
    status: int                # 0 converged, 1 not converged, 2 diverged
    mean_stress: np.ndarray    # (d, d) <sigma(iters)>
    history: list = field(default_factory=list)
    cauchy: list = field(default_factory=list)


def wave_vectors(H, cell=None):
    """Rows L^{-T} h of the integer frequencies H (Def. 3.3); H itself for P(M)."""
    Hf = np.asarray(H, dtype=np.float64)
    if cell is None:
        return Hf
    return Hf @ np.linalg.inv(np.asarray(cell, dtype=np.float64))


def lippmann_schwinger_map(T, C0, K, upd, zero, eps_bar, eps, sigma, rule="hermitian"):
    """The fixed-point map of the collocated Lippmann-Schwinger equation (Sec. 3.1-3.2).

    With the polarization tau = sigma - C0 : eps = (C - C0) : eps, the
    equation eps = eps_bar - Gamma0 * tau holds at the solution; evaluated on
    the pattern, the convolution is a product per frequency of G(M^T):
        eps_new = F(M)^{-1} [ eps_bar at h = 0;  -Gamma0(k_h) tau_hat_h on the
                  active h != 0 (rows `upd`);  0 on the unpaired classes ].
    K: the wave vectors of the frequencies (L^{-T} h on P_L(M)).
    Returns the real field eps_new (its imaginary part vanishes under the
    Hermitian rule and is dropped).
    """
    tau_hat = T.forward(sigma - contract(C0, eps))
    eps_hat = np.zeros_like(tau_hat)
    eps_hat[:, :, upd] = gamma0_apply(C0, K[upd], tau_hat[:, :, upd])
    eps_hat[:, :, zero] = eps_bar
    new = T.inverse(eps_hat)
    if rule == "hermitian":
        assert np.max(np.abs(new.imag)) <= 1e-9 * max(1.0, np.max(np.abs(new.real)))
    return new.real


def basic_scheme(M, phase, lame, lame0, eps_bar, tol=1e-8, max_iter=1000, init=None,
                 transform=None, rule="hermitian", fixed_iters=None, cell=None, stop="residual", on_iteration=None):
    """The Basic Scheme (Algorithm 1, Sec. 3.2) on P(M), or on P_L(M) with cell = L.

    Picard iteration of ``lippmann_schwinger_map`` from eps(0) = eps_bar
    (+ init), stopped on the equilibrium residual of the current iterate.

    phase: (m,) ints in the transform's point order; lame: (n_phase, 2) rows
    (lambda, mu); lame0 = (lambda0, mu0); eps_bar: (d, d) macroscopic strain;
    init: optional (d, d, m) fluctuation added to eps_bar in eps(0).
    fixed_iters: run exactly this many updates, ignoring tol.
    stop="cauchy": the Sec. 5.2 criterion instead, |eps(n+1) - eps(n)| / |eps(0)|
    <= tol; the result is eps(n) for the first such n (n updates performed).
    on_iteration: optional callable(n), called after each update (timing only).
    """
    T = transform or make_transform(M)
    d = len(as_int_matrix(M))
    m = T.m
    H = np.asarray(T.freqs, dtype=np.int64)
    K = wave_vectors(H, cell)
    zero = np.flatnonzero(np.all(H == 0, axis=1))[0]
    active = active_classes(M, H, rule)
    upd = active.copy()
    upd[zero] = False
    tensors = [iso_tensor(l, mu, d) for l, mu in np.asarray(lame, dtype=np.float64)]
    C0 = iso_tensor(lame0[0], lame0[1], d)
    phase = np.asarray(phase)

    eps = np.broadcast_to(np.asarray(eps_bar, dtype=np.float64)[:, :, None], (d, d, m)).copy()
    if init is not None:
        eps = eps + np.asarray(init, dtype=np.float64)
    norm0 = float(np.linalg.norm(eps))
    hist, cauchy = [], []
    r0 = None
    n = 0
    while True:
        sigma = apply_phases(tensors, phase, eps)
        sig_hat = T.forward(sigma)
        r = equilibrium_residual(sig_hat, K, active, zero)
        hist.append(r)
        r0 = r if r0 is None else r0
        mean = np.sum(sigma, axis=2) / m
        if not math.isfinite(r) or (r0 > 0 and r > 1e3 * r0):
            return SchemeResult(eps, n, r, 2, mean, hist, cauchy)
        if fixed_iters is None and stop == "residual" and r <= tol:
            return SchemeResult(eps, n, r, 0, mean, hist, cauchy)
        if n == (fixed_iters if fixed_iters is not None else max_iter):
            status = 0 if fixed_iters is not None else 1
            return SchemeResult(eps, n, r, status, mean, hist, cauchy)
        new = lippmann_schwinger_map(T, C0, K, upd, zero, eps_bar, eps, sigma, rule)
        cauchy.append(float(np.linalg.norm(new - eps)) / norm0)
        if fixed_iters is None and stop == "cauchy" and cauchy[-1] <= tol:
            return SchemeResult(eps, n, r, 0, mean, hist, cauchy)
        eps = new
        n += 1
        if on_iteration is not None:
            on_iteration(n)


def unit_loads(d):
    """Strain tensors of the Mandel unit vectors (6 in 3-D, 3 in 2-D)."""
    k = 6 if d == 3 else 3
    return [from_mandel(np.eye(k)[i], d) for i in range(k)]


def effective_stiffness(M, phase, lame, lame0, tol=1e-10, max_iter=5000, transform=None, rule="hermitian", cell=None):
    """C_eff in Mandel form: column k is Mandel(<sigma>) for unit load k (Def. 3.1)."""
    T = transform or make_transform(M)
    d = len(as_int_matrix(M))
    cols, runs = [], []
    for E in unit_loads(d):
        res = basic_scheme(M, phase, lame, lame0, E, tol=tol, max_iter=max_iter, transform=T, rule=rule, cell=cell)
        cols.append(to_mandel(res.mean_stress))
        runs.append(res)
    return np.array(cols).T, runs


def default_reference(lame):
    """Reading: C0 Lame constants = mean of the extreme phase values."""
    lame = np.asarray(lame, dtype=np.float64)
    return (0.5 * (lame[:, 0].min() + lame[:, 0].max()), 0.5 * (lame[:, 1].min() + lame[:, 1].max()))


def error_l2(eps, eps_ref):
    """e_l2 of Sec. 5.1: relative l2 error of the strain over the pattern."""
    return float(np.linalg.norm(eps - eps_ref) / np.linalg.norm(eps_ref))


def error_eff(ceff_eps0, ceff_eps0_ref):
    """e_eff of Sec. 5.1: relative 2-norm error of C_eff : eps0."""
    return float(np.linalg.norm(ceff_eps0 - ceff_eps0_ref) / np.linalg.norm(ceff_eps0_ref))
