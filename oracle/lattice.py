"""Exact-integer lattice algebra (oracle; test infrastructure only).

Follows Sec. 2.1 (congruence mod M, lattice Lambda(M) = M^{-1} Z^d, pattern
P(M) = Lambda(M) intersected with the symmetric unit cube [-1/2, 1/2)^d,
generating set G(M) = M P(M), |P| = |G| = |det M|) and Sec. 2.2 (Smith normal
form M = Q E R with unimodular Q, R and e_j | e_{j+1}; pattern dimension
d_M = #{j : e_j > 1}).

Everything here is exact: Python integers or int64 arrays whose range is
checked.  Points y in P(M) are returned as integer numerators p = m*y with
m = |det M|, so y = p/m and -m/2 <= p_i < m/2.

Reading (unimodular Q, R): the paper asks for Q, R of determinant 1, which is
impossible when det M < 0; Q and R are taken unimodular (det +-1) and the
elementary divisors positive.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np


# --------------------------------------------------------------------------
# small exact integer linear algebra
# --------------------------------------------------------------------------

def as_int_matrix(M):
    """Return M as a list of lists of Python ints (square)."""
    A = [[int(v) for v in row] for row in np.asarray(M, dtype=object).tolist()]
    d = len(A)
    if d == 0 or any(len(r) != d for r in A):
        raise ValueError("M must be a non-empty square integer matrix")
    return A


def int_det(M) -> int:
    """Exact determinant by the Bareiss fraction-free elimination."""
    A = [row[:] for row in as_int_matrix(M)]
    d = len(A)
    sign = 1
    prev = 1
    for k in range(d - 1):
        if A[k][k] == 0:
            piv = next((i for i in range(k + 1, d) if A[i][k] != 0), None)
            if piv is None:
                return 0
            A[k], A[piv] = A[piv], A[k]
            sign = -sign
        for i in range(k + 1, d):
            for j in range(k + 1, d):
                A[i][j] = (A[i][j] * A[k][k] - A[i][k] * A[k][j]) // prev
        prev = A[k][k]
    return sign * A[d - 1][d - 1]


def minor(A, rows, cols) -> int:
    return int_det([[A[r][c] for c in cols] for r in rows])


def adjugate(M):
    """Integer adjugate adj(M), so that M adj(M) = det(M) I."""
    A = as_int_matrix(M)
    d = len(A)
    if d == 1:
        return [[1]]
    adj = [[0] * d for _ in range(d)]
    for i in range(d):
        for j in range(d):
            rows = [r for r in range(d) if r != j]
            cols = [c for c in range(d) if c != i]
            adj[i][j] = (-1) ** (i + j) * minor(A, rows, cols)
    return adj


def transpose(A):
    return [list(r) for r in zip(*A)]


def matmul(A, B):
    return [[sum(A[i][k] * B[k][j] for k in range(len(B))) for j in range(len(B[0]))]
            for i in range(len(A))]


def matvec(A, v):
    return [sum(A[i][k] * v[k] for k in range(len(v))) for i in range(len(A))]


def identity(d):
    return [[int(i == j) for j in range(d)] for i in range(d)]


def inverse_unimodular(U):
    """Exact inverse of a unimodular integer matrix."""
    D = int_det(U)
    if abs(D) != 1:
        raise ValueError("matrix is not unimodular")
    adj = adjugate(U)
    return [[D * v for v in row] for row in adj]


# --------------------------------------------------------------------------
# Smith normal form (Sec. 2.2)
# --------------------------------------------------------------------------

def determinantal_divisors(M):
    """Elementary divisors from determinantal divisors.

    The k-th determinantal divisor D_k is the gcd of all k x k minors; the
    elementary divisors are e_k = D_k / D_{k-1}.  This is an independent route
    to the diagonal of the Smith normal form.
    """
    A = as_int_matrix(M)
    d = len(A)
    Dk = [1]
    for k in range(1, d + 1):
        g = 0
        for rows in itertools.combinations(range(d), k):
            for cols in itertools.combinations(range(d), k):
                g = math.gcd(g, minor(A, rows, cols))
        Dk.append(g)
    if Dk[-1] == 0:
        raise ValueError("singular matrix")
    return [Dk[k] // Dk[k - 1] for k in range(1, d + 1)]


def smith_normal_form(M):
    """Return (Q, e, R) with M = Q diag(e) R, Q and R unimodular, e_j | e_{j+1}.

    Plain elimination: track row operations U and column operations V with
    U M V = diag(e); then Q = U^{-1} and R = V^{-1}.
    """
    A = [row[:] for row in as_int_matrix(M)]
    d = len(A)
    if int_det(A) == 0:
        raise ValueError("singular matrix")
    U = identity(d)
    V = identity(d)

    def swap_rows(X, i, j):
        X[i], X[j] = X[j], X[i]

    def swap_cols(X, i, j):
        for row in X:
            row[i], row[j] = row[j], row[i]

    def add_row(X, dst, src, f):  # row dst += f * row src
        X[dst] = [a + f * b for a, b in zip(X[dst], X[src])]

    def add_col(X, dst, src, f):  # col dst += f * col src
        for row in X:
            row[dst] += f * row[src]

    for t in range(d):
        while True:
            # pivot: smallest nonzero |entry| of the trailing block
            best = None
            for i in range(t, d):
                for j in range(t, d):
                    if A[i][j] != 0 and (best is None or abs(A[i][j]) < abs(A[best[0]][best[1]])):
                        best = (i, j)
            i, j = best
            swap_rows(A, t, i); swap_rows(U, t, i)
            swap_cols(A, t, j); swap_cols(V, t, j)
            done = True
            for i in range(t + 1, d):
                q = A[i][t] // A[t][t]
                if q:
                    add_row(A, i, t, -q); add_row(U, i, t, -q)
                if A[i][t] != 0:
                    done = False
            for j in range(t + 1, d):
                q = A[t][j] // A[t][t]
                if q:
                    add_col(A, j, t, -q); add_col(V, j, t, -q)
                if A[t][j] != 0:
                    done = False
            if not done:
                continue
            # divisibility of the trailing block by the pivot
            bad = None
            for i in range(t + 1, d):
                for j in range(t + 1, d):
                    if A[i][j] % A[t][t] != 0:
                        bad = i
                        break
                if bad is not None:
                    break
            if bad is None:
                break
            add_row(A, t, bad, 1); add_row(U, t, bad, 1)
        if A[t][t] < 0:
            A[t] = [-v for v in A[t]]
            U[t] = [-v for v in U[t]]
    e = [A[t][t] for t in range(d)]
    Q = inverse_unimodular(U)
    R = inverse_unimodular(V)
    assert matmul(matmul(Q, [[e[i] if i == j else 0 for j in range(d)] for i in range(d)]), R) == as_int_matrix(M)
    return Q, e, R


def pattern_dimension(e) -> int:
    """d_M = number of elementary divisors larger than one."""
    return sum(1 for v in e if v > 1)


# --------------------------------------------------------------------------
# patterns and generating sets (Sec. 2.1)
# --------------------------------------------------------------------------

def _centre(v, m):
    """Map integers to the symmetric residue system [-m/2, m/2) modulo m."""
    v = np.asarray(v, dtype=np.int64) % m
    return np.where(2 * v >= m, v - m, v)


def pattern_bruteforce(M):
    """P(M) by scanning every candidate numerator p in [-m/2, m/2)^d.

    y = p/m lies in Lambda(M) iff M y is integral iff M p = 0 (mod m).
    Only for tiny m (m^d candidates).  Returns sorted int64 numerators.
    """
    A = np.array(as_int_matrix(M), dtype=np.int64)
    d = A.shape[0]
    m = abs(int_det(A.tolist()))
    if m ** d > 3_000_000:
        raise ValueError("pattern_bruteforce is for tiny patterns only")
    rng = np.arange(-(m // 2), m - m // 2, dtype=np.int64)
    grids = np.meshgrid(*([rng] * d), indexing="ij")
    P = np.stack([g.ravel() for g in grids], axis=1)
    ok = np.all((P @ A.T) % m == 0, axis=1)
    return _sorted_rows(P[ok])


def _sorted_rows(P):
    P = np.asarray(P, dtype=np.int64)
    if P.shape[0] == 0:
        return P
    order = np.lexsort(P.T[::-1])
    return P[order]


def _keys(P, m):
    """uint64 key of rows of residues mod m (requires m^d < 2^64)."""
    P = np.asarray(P, dtype=np.int64) % m
    k = np.zeros(P.shape[0], dtype=np.uint64)
    for c in range(P.shape[1]):
        k = k * np.uint64(m) + P[:, c].astype(np.uint64)
    return k


def _coset_closure(generators, reduce_fn, key_fn):
    """Finite abelian group generated by `generators` under + and `reduce_fn`.

    H_0 = {0}; H_j = union over k < n_j of (H_{j-1} + k g_j), where n_j is the
    least k > 0 with k g_j in H_{j-1}.  Elements are rows of an int64 array.
    """
    d = len(generators[0])
    H = np.zeros((1, d), dtype=np.int64)
    Hk = np.sort(key_fn(H))
    for g in generators:
        g = np.asarray(g, dtype=np.int64)
        shifts = [H]
        acc = np.zeros(d, dtype=np.int64)
        while True:
            acc = reduce_fn((acc + g)[None, :])[0]
            k = key_fn(acc[None, :])[0]
            pos = np.searchsorted(Hk, k)
            if pos < Hk.size and Hk[pos] == k:
                break
            shifts.append(reduce_fn(H + acc[None, :]))
        H = np.concatenate(shifts, axis=0)
        Hk = np.sort(key_fn(H))
    return H


def pattern_points(M):
    """P(M) as sorted integer numerators, by generating the group Lambda(M)/Z^d.

    The columns of M^{-1} = adj(M)/det(M) generate Lambda(M) modulo Z^d.  No
    Smith normal form is used, so this is independent of the fast orderings.
    """
    A = as_int_matrix(M)
    d = len(A)
    D = int_det(A)
    if D == 0:
        raise ValueError("singular matrix")
    m = abs(D)
    if m ** d >= 2 ** 64:
        raise ValueError("pattern too large for exact keys")
    adj = adjugate(A)
    s = 1 if D > 0 else -1
    gens = [[s * adj[i][j] for i in range(d)] for j in range(d)]  # numerators of columns of M^{-1}

    pts = _coset_closure(gens, lambda P: _centre(P, m), lambda P: _keys(P, m))
    assert pts.shape[0] == m
    return _sorted_rows(pts)


def reduce_to_generating_set(MT, h):
    """Representative of h modulo M^T Z^d inside M^T [-1/2, 1/2)^d (exact).

    h' = h - M^T z with z = floor(M^{-T} h + 1/2), computed with integers as
    M^{-T} h = adj(M^T) h / det(M^T).
    """
    A = as_int_matrix(MT)
    D = int_det(A)
    adj = np.array(adjugate(A), dtype=object)
    H = np.atleast_2d(np.asarray(h, dtype=object))
    a = H.dot(adj.T)  # rows: adj(M^T) h
    if D < 0:
        a = -a
        D = -D
    z = (2 * a + D) // (2 * D)
    out = H - z.dot(np.array(A, dtype=object).T)
    return np.array(out, dtype=np.int64)


def in_generating_set(MT, h):
    """True where M^{-T} h lies in [-1/2, 1/2)^d, tested with integers."""
    A = as_int_matrix(MT)
    D = int_det(A)
    adj = np.array(adjugate(A), dtype=object)
    H = np.atleast_2d(np.asarray(h, dtype=object))
    a = H.dot(adj.T)
    s = 1 if D > 0 else -1
    m = abs(D)
    t = 2 * s * a
    return np.all((t >= -m) & (t < m), axis=1).astype(bool)


def generating_set_bruteforce(MT):
    """G(M^T) by scanning the bounding box of M^T [-1/2, 1/2]^d."""
    A = np.array(as_int_matrix(MT), dtype=np.int64)
    d = A.shape[0]
    half = np.abs(A).sum(axis=1)  # 2 * half-width of the bounding box
    ranges = [np.arange(-(w // 2) - 1, w // 2 + 2, dtype=np.int64) for w in half]
    total = int(np.prod([r.size for r in ranges]))
    if total > 5_000_000:
        raise ValueError("generating_set_bruteforce is for small patterns only")
    grids = np.meshgrid(*ranges, indexing="ij")
    Hc = np.stack([g.ravel() for g in grids], axis=1)
    ok = in_generating_set(A.tolist(), Hc)
    return _sorted_rows(Hc[ok])


def generating_set(MT):
    """G(M^T) by generating Z^d / M^T Z^d from unit vectors (no SNF)."""
    A = as_int_matrix(MT)
    d = len(A)
    m = abs(int_det(A))
    Aabs = np.abs(np.array(A, dtype=np.int64)).sum(axis=1)
    base = int(Aabs.max()) + 2  # representatives satisfy |h_i| <= half of row sums
    if (2 * base + 1) ** d >= 2 ** 63:
        raise ValueError("generating set too large for exact keys")

    def key_fn(H):
        H = np.asarray(H, dtype=np.int64) + base
        k = np.zeros(H.shape[0], dtype=np.uint64)
        for c in range(d):
            k = k * np.uint64(2 * base + 1) + H[:, c].astype(np.uint64)
        return k

    gens = [[int(i == j) for i in range(d)] for j in range(d)]
    G = _coset_closure(gens, lambda H: reduce_to_generating_set(A, H), key_fn)
    assert G.shape[0] == m
    return _sorted_rows(G)


# --------------------------------------------------------------------------
# Smith-normal-form addressing (Sec. 2.2, eqs. patternBasisV / genSetBasisV)
# --------------------------------------------------------------------------

class SnfIndexing:
    """Oracle's own product-of-cyclic-groups addressing of P(M) and G(M^T).

    With M = Q E R: y in Lambda(M) iff R y in E^{-1} Z^d, so
    y(lambda) = R^{-1} E^{-1} lambda (mod 1), lambda_j in Z_{e_j}; and
    h = M^T ytilde with h(kappa) = R^T kappa reduced modulo M^T.  Then
    h(kappa)^T y(lambda) = sum_j kappa_j lambda_j / e_j (mod 1), so the pattern
    DFT is the ordinary DFT over Z_{e_1} x ... x Z_{e_d}.

    Reading (basis vectors): eq. patternBasisV is garbled (index
    e_{d+d_M+j}, missing R^{-1}); taken as y_j = R^{-1} e_j / e_j (mod 1) over
    the non-trivial axes, and h_j = R^T e_j as in eq. genSetBasisV.
    Arrays are ordered lexicographically in lambda (resp. kappa) over the
    axes with e_j > 1, slowest axis first.
    """

    def __init__(self, M):
        self.M = as_int_matrix(M)
        self.d = len(self.M)
        D = int_det(self.M)
        if D == 0:
            raise ValueError("singular matrix")
        self.m = abs(D)
        self.Q, self.e, self.R = smith_normal_form(self.M)
        self.Rinv = inverse_unimodular(self.R)
        self.axes = [j for j in range(self.d) if self.e[j] > 1]
        self.shape = tuple(self.e[j] for j in self.axes) or (1,)

    def _grid(self):
        idx = np.indices(self.shape).reshape(len(self.shape), -1).T
        full = np.zeros((idx.shape[0], self.d), dtype=np.int64)
        if self.axes:
            full[:, self.axes] = idx
        return full

    def points(self):
        """Integer numerators p(lambda) = m R^{-1} E^{-1} lambda (centred mod m)."""
        lam = self._grid().astype(object)
        scaled = lam * np.array([self.m // ej for ej in self.e], dtype=object)
        p = scaled.dot(np.array(self.Rinv, dtype=object).T)
        return _centre(np.array(p % self.m, dtype=np.int64), self.m)

    def freqs(self):
        """h(kappa) = R^T kappa reduced into G(M^T)."""
        kap = self._grid().astype(object)
        h = kap.dot(np.array(self.R, dtype=object))  # rows: (R^T kappa)^T = kappa^T R
        return reduce_to_generating_set(transpose(self.M), np.array(h, dtype=object))
