"""Seeded synthetic inputs shared by the oracle tests and the GPU harness.

This module holds geometry and random draws only: pattern matrices, phase
assignments at given points, material tables.  It contains none of the
method's arithmetic (no pattern DFT, no Green operator, no local law).  Point
coordinates come from the caller (the oracle's own enumeration or the
library's canonical order), always as exact integer numerators p = m * y.

Workload recipes (shapes of the paper's examples, Sec. 4-5):
* laminate_2d: layers normal to q = (1, 2), phase 0 iff frac(q . y) < 1/2;
* hashin_3d: coated confocal ellipsoid, semi-axes (0.15, 0.2, 0.3), rotated
  by seeded Euler angles, coating 0.1 of the cell;
* rank1_generator: Korobov vector z = (1, a, a^2 mod m) whose dual lattice
  has the longest shortest vector among seeded odd candidates;
* spheres_rsa: random sequential addition of periodic spheres;
* batch_2d_members: non-diagonal 2-D pattern matrices with 7-smooth
  elementary divisors and random elliptical inclusions.
"""
from __future__ import annotations

import functools
import math

import numpy as np


# --------------------------------------------------------------------------
# materials
# --------------------------------------------------------------------------

def lame(E, nu):
    """(lambda, mu) of an isotropic material (E, nu)."""
    return (E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu)))


def phase_mean_reference(lame_table):
    """Reference Lame pair: mean of the extreme phase values."""
    t = np.asarray(lame_table, dtype=np.float64)
    return (0.5 * (t[:, 0].min() + t[:, 0].max()), 0.5 * (t[:, 1].min() + t[:, 1].max()))


# --------------------------------------------------------------------------
# laminate (Sec. 4.1, configuration of the 2-D correctness case)
# --------------------------------------------------------------------------

def laminate_phase(points_num, m, q=(1, 2)):
    """Phase 0 iff frac(q . y) < 1/2 for y = p/m, decided with integers."""
    p = np.asarray(points_num, dtype=np.int64)
    s = (p.astype(object).dot(np.asarray(q, dtype=object))) % m
    s = np.array(s, dtype=np.int64)
    return np.where(2 * s < m, 0, 1).astype(np.uint8)


LAMINATE_LAME = (lame(1.0, 0.3), lame(10.0, 0.3))


# --------------------------------------------------------------------------
# rotations and ellipsoids
# --------------------------------------------------------------------------

def euler_zyz(seed):
    """R = Rz(alpha) Ry(beta) Rz(gamma), alpha, gamma ~ U[0, 2pi), cos beta ~ U[-1, 1]."""
    rng = np.random.default_rng(seed)
    a, g = rng.uniform(0.0, 2.0 * math.pi, size=2)
    b = math.acos(rng.uniform(-1.0, 1.0))

    def rz(t):
        return np.array([[math.cos(t), -math.sin(t), 0.0], [math.sin(t), math.cos(t), 0.0], [0.0, 0.0, 1.0]])

    def ry(t):
        return np.array([[math.cos(t), 0.0, math.sin(t)], [0.0, 1.0, 0.0], [-math.sin(t), 0.0, math.cos(t)]])

    return rz(a) @ ry(b) @ rz(g)


def coating_radius(c, volume):
    """rho_e with (4/3) pi (prod sqrt(c^2 + rho_e) - prod c) = volume (bisection)."""
    c = np.asarray(c, dtype=np.float64)
    base = float(np.prod(c))
    f = lambda r: 4.0 / 3.0 * math.pi * (float(np.prod(np.sqrt(c ** 2 + r))) - base) - volume
    lo, hi = 0.0, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def hashin_geometry(seed=2, c=(0.15, 0.2, 0.3), rho_c=0.0, coating_fraction=0.1):
    """Geometry of the 3-D coated-ellipsoid workload."""
    c = np.asarray(c, dtype=np.float64)
    return dict(c=c, rho_c=rho_c, rho_e=coating_radius(c, coating_fraction), R=euler_zyz(seed))


def hashin_phase(points_num, m, geom):
    """0 core, 1 coating, 2 matrix at y = p/m (closed inequalities).

    Core iff sum xt_i^2/(c_i^2 + rho_c) <= 1 with xt = R^T y, i.e. the
    ellipsoidal radius is at most rho_c (the defining function decreases
    in rho); likewise for the coating.
    """
    y = np.asarray(points_num, dtype=np.float64) / m
    if y.shape[1] == 2:
        y = np.concatenate([y, np.zeros((y.shape[0], 1))], axis=1)
    xt = y @ geom["R"]
    c2 = geom["c"] ** 2
    inner = np.sum(xt ** 2 / (c2 + geom["rho_c"]), axis=1) <= 1.0
    outer = np.sum(xt ** 2 / (c2 + geom["rho_e"]), axis=1) <= 1.0
    ph = np.full(y.shape[0], 2, dtype=np.uint8)
    ph[outer] = 1
    ph[inner] = 0
    return ph


# --------------------------------------------------------------------------
# rank-1 lattices
# --------------------------------------------------------------------------

def lll_reduce(B, delta=0.75):
    """LLL reduction of the rows of an integer basis B (exact rationals)."""
    from fractions import Fraction
    B = [list(map(int, r)) for r in B]
    n = len(B)

    def dot(u, v):
        return sum(a * b for a, b in zip(u, v))

    def gs(B):
        Bs, mu = [], [[Fraction(0)] * n for _ in range(n)]
        for i in range(n):
            v = [Fraction(x) for x in B[i]]
            for j in range(i):
                mu[i][j] = Fraction(dot(B[i], Bs[j])) / dot(Bs[j], Bs[j]) if dot(Bs[j], Bs[j]) else Fraction(0)
                v = [a - mu[i][j] * b for a, b in zip(v, Bs[j])]
            Bs.append(v)
        return Bs, mu

    k = 1
    Bs, mu = gs(B)
    while k < n:
        for j in range(k - 1, -1, -1):
            q = round(mu[k][j])
            if q:
                B[k] = [a - q * b for a, b in zip(B[k], B[j])]
                Bs, mu = gs(B)
        if dot(Bs[k], Bs[k]) >= (delta - mu[k][k - 1] ** 2) * dot(Bs[k - 1], Bs[k - 1]):
            k += 1
        else:
            B[k], B[k - 1] = B[k - 1], B[k]
            Bs, mu = gs(B)
            k = max(k - 1, 1)
    return B


def rank1_matrix(m, z):
    """Integer M with P(M) = {k z / m mod 1}: M^T = LLL basis of {h : h . z = 0 mod m}."""
    z = [int(v) for v in z]
    d = len(z)
    if math.gcd(z[0], m) != 1:
        raise ValueError("z_1 must be a unit modulo m")
    inv = pow(z[0], -1, m)
    rows = [[m] + [0] * (d - 1)]
    for j in range(1, d):
        r = [0] * d
        r[0] = (-z[j] * inv) % m
        r[j] = 1
        rows.append(r)
    red = lll_reduce(rows)
    MT = np.array(red, dtype=np.int64).T  # columns = reduced dual basis
    M = MT.T.copy()
    return M


def rank1_generator(m, seed=2, candidates=4096, d=3):
    """Korobov a maximizing the shortest LLL vector of the dual lattice."""
    rng = np.random.default_rng(seed)
    best = None
    for a in rng.integers(0, m // 2, size=candidates) * 2 + 1:
        a = int(a)
        z = [1, a, (a * a) % m][:d]
        M = rank1_matrix(m, z)
        short = min(float(np.linalg.norm(r)) for r in M)
        if best is None or short > best[0]:
            best = (short, a, M)
    return best[1], best[2]


# --------------------------------------------------------------------------
# random sequential addition of periodic spheres (3-D precision workload)
# --------------------------------------------------------------------------

def spheres_rsa(seed=3, rmin=0.03, rmax=0.08, target=0.3, max_tries=200000):
    rng = np.random.default_rng(seed)
    centres, radii = [], []
    vol = 0.0
    tries = 0
    while vol < target and tries < max_tries:
        tries += 1
        c = rng.uniform(-0.5, 0.5, size=3)
        r = rng.uniform(rmin, rmax)
        ok = True
        for c2, r2 in zip(centres, radii):
            dv = c - c2
            dv -= np.round(dv)
            if float(dv @ dv) < (r + r2) ** 2:
                ok = False
                break
        if ok:
            centres.append(c)
            radii.append(r)
            vol += 4.0 / 3.0 * math.pi * r ** 3
    return np.array(centres), np.array(radii)


def spheres_phase(points_num, m, centres, radii):
    """1 inside any (periodic) sphere, else 0 (closed balls, minimum image).

    Points are binned into cells at least one diameter wide, so each sphere is
    tested only against the points of the 27 cells around its centre.
    """
    y = np.asarray(points_num, dtype=np.float64) / m
    d = y.shape[1]
    ph = np.zeros(y.shape[0], dtype=np.uint8)
    if len(radii) == 0:
        return ph
    nc = max(1, int(1.0 / (2.0 * float(np.max(radii)))))
    cell = np.floor((y + 0.5) * nc).astype(np.int64) % nc
    key = np.zeros(y.shape[0], dtype=np.int64)
    for k in range(d):
        key = key * nc + cell[:, k]
    order = np.argsort(key, kind="stable")
    skey = key[order]
    starts = np.searchsorted(skey, np.arange(nc ** d))
    ends = np.searchsorted(skey, np.arange(nc ** d), side="right")
    offs = np.array(np.meshgrid(*([[-1, 0, 1]] * d), indexing="ij")).reshape(d, -1).T
    for c, r in zip(centres, radii):
        cc = np.floor((np.asarray(c[:d]) + 0.5) * nc).astype(np.int64) % nc
        nb = (cc[None, :] + offs) % nc
        nkeys = np.unique(np.ravel_multi_index(nb.T, (nc,) * d))
        idx = np.concatenate([order[starts[k]:ends[k]] for k in nkeys])
        dv = y[idx] - np.asarray(c[:d])
        dv -= np.round(dv)
        ph[idx[np.sum(dv * dv, axis=1) <= r * r]] = 1
    return ph


# --------------------------------------------------------------------------
# 2-D batch members: non-diagonal M with 7-smooth elementary divisors
# --------------------------------------------------------------------------

@functools.lru_cache(maxsize=None)
def _seven_smooth(lo, hi):
    out = []
    for a in range(0, 40):
        for b in range(0, 26):
            for c in range(0, 18):
                for e in range(0, 15):
                    v = 2 ** a * 3 ** b * 5 ** c * 7 ** e
                    if lo <= v <= hi:
                        out.append(v)
    return tuple(sorted(set(out)))


def seven_smooth(lo, hi):
    """Sorted integers in [lo, hi] with no prime factor above 7."""
    return list(_seven_smooth(lo, hi))


def batch_2d_member(seed, lo=1024, hi=65536):
    """Pattern matrix, ellipses and contrast of one batch member."""
    rng = np.random.default_rng(seed)
    cand = np.array(seven_smooth(lo // 2, hi * 2))
    target = math.exp(rng.uniform(math.log(lo), math.log(hi)))
    det = int(cand[np.argmin(np.abs(cand - target))])
    divs = [e for e in range(1, int(math.isqrt(det)) + 1) if det % (e * e) == 0]
    e1 = int(rng.choice(divs))
    E = np.diag([e1, det // e1]).astype(np.int64)

    def shear(k):
        U = np.eye(2, dtype=np.int64)
        U[k % 2, (k + 1) % 2] = rng.integers(-3, 4)
        return U

    while True:
        Q = np.eye(2, dtype=np.int64)
        R = np.eye(2, dtype=np.int64)
        for k in range(4):
            Q = Q @ shear(k)
            R = R @ shear(k + 1)
        M = Q @ E @ R
        M = np.array(lll_reduce(M.tolist()), dtype=np.int64)
        if M[0, 1] != 0 or M[1, 0] != 0:
            break
    n_inc = int(rng.integers(2, 7))
    ell = [dict(centre=rng.uniform(-0.5, 0.5, size=2), axes=rng.uniform(0.05, 0.2, size=2),
                angle=rng.uniform(0.0, math.pi)) for _ in range(n_inc)]
    contrast = float(rng.uniform(2.0, 50.0))
    return dict(M=M, ellipses=ell, contrast=contrast, lame=(lame(1.0, 0.3), lame(contrast, 0.3)))


def ellipses_phase(points_num, m, ellipses):
    y = np.asarray(points_num, dtype=np.float64) / m
    ph = np.zeros(y.shape[0], dtype=np.uint8)
    for e in ellipses:
        dv = y - e["centre"]
        dv -= np.round(dv)
        c, s = math.cos(e["angle"]), math.sin(e["angle"])
        u = c * dv[:, 0] + s * dv[:, 1]
        v = -s * dv[:, 0] + c * dv[:, 1]
        ph[(u / e["axes"][0]) ** 2 + (v / e["axes"][1]) ** 2 <= 1.0] = 1
    return ph


def random_phase_field(m, n_phase, seed):
    return np.random.default_rng(seed).integers(0, n_phase, size=m).astype(np.uint8)


def random_rotation(rng):
    """Uniformly distributed rotation (QR of a Gaussian matrix with sign fix)."""
    A = rng.standard_normal((3, 3))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(R))[None, :]
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def ellipsoids_member(seed):
    """Learned-guess workload member: 1-20 randomly oriented ellipsoids, axis
    ratios U[1, 3], a common scale that makes the voxel volume fraction
    U[0.1, 0.4] (overlap allowed), contrast U[2, 100], nu = 0.3."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 21))
    ell = []
    for _ in range(k):
        ell.append(dict(centre=rng.uniform(-0.5, 0.5, size=3),
                        axes=np.array([1.0, rng.uniform(1.0, 3.0), rng.uniform(1.0, 3.0)]),
                        R=random_rotation(rng)))
    vf = float(rng.uniform(0.1, 0.4))
    contrast = float(rng.uniform(2.0, 100.0))
    return dict(ellipsoids=ell, vf=vf, contrast=contrast, lame=(lame(1.0, 0.3), lame(contrast, 0.3)))


def ellipsoids_phase(points_num, m, member):
    """Phase 1 where min_k (d_k^T A_k d_k) <= s^2 (minimum image d_k), s chosen
    so that the fraction of points in phase 1 is the member's vf."""
    y = np.asarray(points_num, dtype=np.float64) / m
    q = np.full(y.shape[0], np.inf)
    for e in member["ellipsoids"]:
        d = y - e["centre"]
        d -= np.round(d)
        u = d @ e["R"]                     # coordinates in the ellipsoid's axes
        q = np.minimum(q, np.sum((u / e["axes"]) ** 2, axis=1))
    s2 = np.quantile(q, member["vf"])
    return (q <= s2).astype(np.uint8)
