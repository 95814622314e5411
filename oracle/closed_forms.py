"""Closed-form solutions of Sec. 4 (oracle; test infrastructure only).

Laminate (Sec. 4.1)
-------------------
Two isotropic phases alternating along the unit normal n with volume
fractions f1, f2.  Two independent routes:
* ``laminate_milton``: the formula quoted from Milton Sec. 9.5,
  (S - T)^{-1} = <(S~(x) - T)^{-1}>, S = s0 (s0 Id - C_eff)^{-1},
  S~ = s0 (s0 Id - C(x))^{-1}, T_ijkl = 1/2 (n_i d_jk n_l + n_i d_jl n_k
  + n_j d_ik n_l + n_j d_il n_k) - n_i n_j n_k n_l, evaluated on the Mandel
  space, s0 above the largest stiffness eigenvalue.
* ``laminate_jump``: the piecewise-constant strain eps1, eps2.  Reading: the
  second equation of the printed two-strain system is vacuous (it is the
  first multiplied by C_eff); the conditions used are the strain jump
  eps2 - eps1 = sym(a (x) n) and traction continuity (sigma2 - sigma1) n = 0
  together with f1 eps1 + f2 eps2 = eps0.

Generalized Hashin structure (Sec. 4.2)
---------------------------------------
Confocal coated ellipsoid, semi-axes l_j(rho) = sqrt(c_j^2 + rho), rotated by R.
Readings:
* depolarization factors: the printed spheroid forms are garbled (prolate
  d3 misses a "-1"; "d2 = 2 - 2 d3" must be (1 - d3)/2; oblate likewise).
  General ellipsoids use d_i = (l1 l2 l3 / 2) int_0^inf ds /
  ((l_i^2 + s) sqrt(prod_j (l_j^2 + s))) by quadrature; the corrected
  spheroid and cylinder forms are kept as pins of that quadrature.
* rotation: any rotation R with the shortest semi-axis along R e1; the
  printed Rodrigues form has the coefficient (1 - n1)/sqrt(n2^2 + n3^2) where
  (1 - n1)/(n2^2 + n3^2) is needed (``rotation_e1_to``).
* gradient of the ellipsoidal radius: the printed denominator uses index i
  and lacks squares; used: d rho / d x_i = (2 x_i / (c_i^2 + rho)) /
  sum_j x_j^2 / (c_j^2 + rho)^2.
* the formulas fix C_eff only along the special eps0 and require a neutral
  matrix: mu_m = mu_e and lambda_m chosen so that C_m : eps0 = C_eff : eps0
  (``hashin`` returns that matrix).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

from .elasticity import iso_tensor, tensor4_to_mandel, to_mandel, from_mandel, contract


# --------------------------------------------------------------------------
# laminate
# --------------------------------------------------------------------------

def laminate_T(n):
    n = np.asarray(n, dtype=np.float64)
    d = n.size
    I = np.eye(d)
    T = 0.5 * (np.einsum("i,jk,l->ijkl", n, I, n) + np.einsum("i,jl,k->ijkl", n, I, n)
               + np.einsum("j,ik,l->ijkl", n, I, n) + np.einsum("j,il,k->ijkl", n, I, n))
    return T - np.einsum("i,j,k,l->ijkl", n, n, n, n)


def laminate_milton(lame1, lame2, f1, n, s0=None):
    """C_eff (Mandel) of a two-phase laminate via the Milton formula."""
    n = np.asarray(n, dtype=np.float64)
    n = n / np.linalg.norm(n)
    d = n.size
    C1 = tensor4_to_mandel(iso_tensor(*lame1, d))
    C2 = tensor4_to_mandel(iso_tensor(*lame2, d))
    T = tensor4_to_mandel(laminate_T(n))
    Id = np.eye(C1.shape[0])
    if s0 is None:
        s0 = 2.0 * max(np.linalg.eigvalsh(C1).max(), np.linalg.eigvalsh(C2).max())
    S1 = s0 * np.linalg.inv(s0 * Id - C1)
    S2 = s0 * np.linalg.inv(s0 * Id - C2)
    avg = f1 * np.linalg.inv(S1 - T) + (1.0 - f1) * np.linalg.inv(S2 - T)
    S = T + np.linalg.inv(avg)
    return s0 * (Id - np.linalg.inv(S))


def laminate_jump(lame1, lame2, f1, n, eps0):
    """Piecewise-constant laminate strains and C_eff : eps0 from jump conditions."""
    n = np.asarray(n, dtype=np.float64)
    n = n / np.linalg.norm(n)
    d = n.size
    eps0 = np.asarray(eps0, dtype=np.float64)
    C1 = iso_tensor(*lame1, d)
    C2 = iso_tensor(*lame2, d)
    f2 = 1.0 - f1
    # eps1 = eps0 - f2 sym(a n), eps2 = eps0 + f1 sym(a n)
    # (C2 eps2 - C1 eps1) n = 0  ->  Kbar a = -((C2 - C1) eps0) n
    Kbar = np.einsum("ijkl,j,l->ik", f1 * C2 + f2 * C1, n, n)
    rhs = -contract(C2 - C1, eps0) @ n
    a = np.linalg.solve(Kbar, rhs)
    S = 0.5 * (np.outer(a, n) + np.outer(n, a))
    eps1 = eps0 - f2 * S
    eps2 = eps0 + f1 * S
    ceff_eps0 = f1 * contract(C1, eps1) + f2 * contract(C2, eps2)
    return eps1, eps2, ceff_eps0


def laminate_ceff_jump(lame1, lame2, f1, n):
    d = len(n)
    k = 6 if d == 3 else 3
    cols = []
    for i in range(k):
        E = from_mandel(np.eye(k)[i], d)
        cols.append(to_mandel(laminate_jump(lame1, lame2, f1, n, E)[2]))
    return np.array(cols).T


# --------------------------------------------------------------------------
# Hashin: geometry helpers
# --------------------------------------------------------------------------

def depolarization_quadrature(l):
    """d_i for an ellipsoid with semi-axes l (all finite), by quadrature."""
    l = np.asarray(l, dtype=np.float64)
    prod = float(np.prod(l))
    out = []
    for i in range(3):
        def f(s, i=i):
            return 1.0 / ((l[i] ** 2 + s) * math.sqrt(np.prod(l ** 2 + s)))
        # substitute s = t/(1-t) to map [0, inf) onto [0, 1)
        def g(t, f=f):
            if t >= 1.0:
                return 0.0  # the integrand decays like s^(-5/2)
            s = t / (1.0 - t)
            return f(s) / (1.0 - t) ** 2
        val, _ = integrate.quad(g, 0.0, 1.0, epsabs=0.0, epsrel=1e-13, limit=400)
        out.append(0.5 * prod * val)
    return np.array(out)


def depolarization_cylinder(l1, l2):
    """Elliptic cylinder (c3 -> infinity): d = (l2, l1, 0)/(l1 + l2)."""
    return np.array([l2 / (l1 + l2), l1 / (l1 + l2), 0.0])


def depolarization_prolate(l_short, l_long):
    """Prolate spheroid l1 = l2 = l_short < l3 = l_long (corrected form)."""
    delta = math.sqrt(1.0 - (l_short / l_long) ** 2)
    d3 = (1.0 - delta ** 2) / delta ** 2 * (math.log((1.0 + delta) / (1.0 - delta)) / (2.0 * delta) - 1.0)
    d1 = 0.5 * (1.0 - d3)
    return np.array([d1, d1, d3])


def depolarization_oblate(l_short, l_long):
    """Oblate spheroid l1 = l_short < l2 = l3 = l_long (corrected form)."""
    delta = math.sqrt(1.0 - (l_short / l_long) ** 2)
    d1 = (1.0 - math.sqrt(1.0 - delta ** 2) / delta * math.asin(delta)) / delta ** 2
    d2 = 0.5 * (1.0 - d1)
    return np.array([d1, d2, d2])


def depolarization(c, rho):
    """d_i(rho) for semi-axes l_j = sqrt(c_j^2 + rho); c3 = inf is a cylinder."""
    c = np.asarray(c, dtype=np.float64)
    if math.isinf(c[2]):
        l1, l2 = math.sqrt(c[0] ** 2 + rho), math.sqrt(c[1] ** 2 + rho)
        return depolarization_cylinder(l1, l2)
    return depolarization_quadrature(np.sqrt(c ** 2 + rho))


def g_fun(c, rho):
    c = np.asarray(c, dtype=np.float64)
    if math.isinf(c[2]):
        return (c[0] ** 2 + rho) * (c[1] ** 2 + rho)
    return float(np.prod(c ** 2 + rho))


def ellipsoidal_radius(c, xt):
    """Largest root rho of sum_i xt_i^2/(c_i^2 + rho) = 1 (rho > -c_1^2).

    phi(rho) = sum xt_i^2/(c_i^2+rho) - 1 decreases strictly on (-c1^2, inf),
    so the root is found by bisection to full precision.
    """
    c = np.asarray(c, dtype=np.float64)
    xt = np.asarray(xt, dtype=np.float64)
    k = 2 if math.isinf(c[2]) else 3
    cc = c[:k] ** 2
    x2 = xt[:k] ** 2
    lo = -cc.min()
    hi = max(1.0, float(x2.sum()))
    phi = lambda r: float(np.sum(x2 / (cc + r))) - 1.0
    lo_r = lo + 1e-300
    for _ in range(400):
        mid = 0.5 * (lo_r + hi)
        if mid == lo_r or mid == hi:
            break
        if phi(mid) > 0:
            lo_r = mid
        else:
            hi = mid
    return 0.5 * (lo_r + hi)


def ellipsoidal_radius_many(c, xt):
    """Vectorized ``ellipsoidal_radius`` for rows of xt (bisection, 200 steps)."""
    c = np.asarray(c, dtype=np.float64)
    k = 2 if math.isinf(c[2]) else 3
    cc = c[:k] ** 2
    x2 = np.asarray(xt, dtype=np.float64)[:, :k] ** 2
    lo = np.full(x2.shape[0], -cc.min())
    hi = np.maximum(1.0, x2.sum(axis=1))
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        with np.errstate(divide="ignore", invalid="ignore"):
            pos = np.sum(x2 / (cc[None, :] + mid[:, None]), axis=1) > 1.0
        lo = np.where(pos, mid, lo)
        hi = np.where(pos, hi, mid)
    return 0.5 * (lo + hi)


def rotation_e1_to(n):
    """Rotation taking e1 to the unit vector n (corrected Rodrigues form)."""
    n = np.asarray(n, dtype=np.float64)
    n = n / np.linalg.norm(n)
    s = n[1] ** 2 + n[2] ** 2
    if s == 0.0:
        return np.eye(3) if n[0] > 0 else np.diag([-1.0, -1.0, 1.0])
    A = np.array([[1.0, -n[1], -n[2]], [n[1], 1.0, 0.0], [n[2], 0.0, 1.0]])
    B = np.array([[-n[1] ** 2 - n[2] ** 2, 0.0, 0.0],
                  [0.0, -n[1] ** 2, -n[1] * n[2]],
                  [0.0, -n[1] * n[2], -n[2] ** 2]])
    return A + (1.0 - n[0]) / s * B


def bulk(lam, mu):
    return lam + 2.0 * mu / 3.0


# --------------------------------------------------------------------------
# Hashin: the closed form
# --------------------------------------------------------------------------

def hashin(c, rho_c, rho_e, lame_c, lame_e, R=None):
    """Generalized Hashin structure of Sec. 4.2.

    Returns dict with eps0, ceff_eps0 (3x3), the neutral matrix Lame pair,
    f = f(rho_e) and a callable strain(x) for points x (N, 3) in the cell.
    """
    c = np.asarray(c, dtype=np.float64)
    R = np.eye(3) if R is None else np.asarray(R, dtype=np.float64)
    lam_c, mu_c = lame_c
    lam_e, mu_e = lame_e
    kc, ke = bulk(lam_c, mu_c), bulk(lam_e, mu_e)
    g_c = g_fun(c, rho_c)
    f_e = math.sqrt(g_c) / math.sqrt(g_fun(c, rho_e))
    Dc = np.diag(depolarization(c, rho_c))
    De = np.diag(depolarization(c, rho_e))
    S_e = (Dc - f_e * De) / (1.0 - f_e)
    a = (3.0 * ke + 4.0 * mu_e) / (9.0 * (kc - ke))
    I = np.eye(3)
    eps0 = R @ (a * I + (1.0 - f_e) * S_e) @ R.T
    A = ke / (kc - ke) * (kc + 4.0 / 3.0 * mu_e) + 4.0 / 3.0 * mu_e * f_e
    ceff_eps0 = R @ (A * I) @ R.T + R @ (2.0 / 3.0 * mu_e * (1.0 - f_e) * (3.0 * S_e - I)) @ R.T
    # neutral isotropic matrix: mu_m = mu_e, lambda_m from the trace
    mu_m = mu_e
    lam_m = float(np.trace(ceff_eps0 - 2.0 * mu_m * eps0)) / (3.0 * float(np.trace(eps0)))
    eps_core = R @ (a * I) @ R.T
    is_cyl = math.isinf(c[2])

    def strain(x):
        x = np.atleast_2d(np.asarray(x, dtype=np.float64))
        if x.shape[1] == 2:
            x = np.concatenate([x, np.zeros((x.shape[0], 1))], axis=1)
        xt_all = x @ R  # rows: (R^{-1} x)^T = x^T R for orthogonal R
        rho = ellipsoidal_radius_many(c, xt_all)
        out = np.empty((x.shape[0], 3, 3))
        out[:] = eps0
        out[rho <= rho_c] = eps_core
        k = 2 if is_cyl else 3
        for n_ in np.flatnonzero((rho > rho_c) & (rho <= rho_e)):
            xt, r = xt_all[n_], rho[n_]
            cc = c[:k] ** 2 + r
            gsq = math.sqrt(g_fun(c, r))
            q = np.zeros(3)
            q[:k] = xt[:k] / (cc * gsq)
            grad = np.zeros(3)
            grad[:k] = (2.0 * xt[:k] / cc) / float(np.sum(xt[:k] ** 2 / cc ** 2))
            f_r = math.sqrt(g_c) / gsq
            Dr = np.diag(depolarization(c, r))
            inner = a * I + Dc - f_r * Dr + 0.5 * math.sqrt(g_c) * np.outer(q, grad)
            out[n_] = R @ inner @ R.T
        return out

    return dict(eps0=eps0, ceff_eps0=ceff_eps0, lame_m=(lam_m, mu_m), f=f_e, strain=strain,
                eps_core=eps_core)


def hashin_bulk_classic(lame_c, lame_e, f):
    """Hashin's coated-sphere effective bulk modulus (textbook formula)."""
    kc, ke = bulk(*lame_c), bulk(*lame_e)
    mu_e = lame_e[1]
    return ke + f * (kc - ke) / (1.0 + (1.0 - f) * (kc - ke) / (ke + 4.0 / 3.0 * mu_e))
