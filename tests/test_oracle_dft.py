"""Pins of the oracle's pattern DFT (Sec. 2.2, Lemma 2.1)."""
import numpy as np
import pytest

from oracle import lattice as L
from oracle.dft import NaiveDFT, SnfFFT

MATS = [
    [[8, 0], [0, 8]],
    [[8, -4], [2, 7]],
    [[8, -1], [0, 8]],
    [[4, 4], [-4, 4]],
    [[6, 2], [1, 5]],
    [[4, 0, 0], [0, 3, 0], [0, 0, 2]],
    [[3, 1, 0], [0, 2, 1], [1, 0, 4]],
]


def key(rows):
    return {tuple(r): i for i, r in enumerate(np.asarray(rows).tolist())}


@pytest.mark.parametrize("n", [(8, 8), (6, 10), (5, 7), (4, 6, 3)])
def test_diagonal_pattern_is_ordinary_dft(n):
    """diag(n_1, ..., n_d) gives the usual d-dimensional DFT (Sec. 2.2).

    Reading: the symmetric cube [-1/2, 1/2) is used for points and
    frequencies (the paper's diagonal example uses [0, 1)); index i of the
    ordinary grid corresponds to y = i/n_j mod 1.
    """
    M = np.diag(n).tolist()
    T = NaiveDFT(M)
    m = T.m
    rng = np.random.default_rng(1)
    grid = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    # point p/m -> grid index (p_j * n_j / m) mod n_j
    idx = tuple(((T.points[:, j] * n[j] // m) % n[j]) for j in range(len(n)))
    a = grid[idx]
    ahat = T.forward(a)
    ref = np.fft.fftn(grid) / m
    fidx = tuple(T.freqs[:, j] % n[j] for j in range(len(n)))
    assert np.allclose(ahat, ref[fidx], atol=1e-13, rtol=0)


@pytest.mark.parametrize("M", MATS)
def test_aliasing_lemma(M):
    """Sampling exp(2 pi i k^T y) gives a unit vector at rep(k) (Lemma 2.1)."""
    T = NaiveDFT(M)
    m = T.m
    MT = L.transpose(L.as_int_matrix(M))
    pos = key(T.freqs)
    rng = np.random.default_rng(2)
    for _ in range(6):
        k = rng.integers(-3 * m, 3 * m, size=len(M))
        r = (T.points.astype(object).dot(k.astype(object))) % m
        a = np.exp(2j * np.pi * np.array(r, dtype=np.float64) / m)
        ahat = T.forward(a)
        rep = tuple(L.reduce_to_generating_set(MT, k[None, :])[0].tolist())
        expect = np.zeros(m, complex)
        expect[pos[rep]] = 1.0
        assert np.allclose(ahat, expect, atol=1e-12)


@pytest.mark.parametrize("M", MATS)
def test_parseval_and_inverse(M):
    T = NaiveDFT(M)
    rng = np.random.default_rng(3)
    a = rng.standard_normal(T.m) + 1j * rng.standard_normal(T.m)
    ahat = T.forward(a)
    assert np.isclose(np.sum(np.abs(ahat) ** 2), np.sum(np.abs(a) ** 2) / T.m, rtol=1e-12)
    assert np.allclose(T.inverse(ahat), a, atol=1e-12)


@pytest.mark.parametrize("M", MATS + [[[16, 2], [4, 16]], [[64, 32], [0, 1]]])
def test_snf_fft_matches_naive(M):
    """The d_M-dimensional FFT route equals the defining matrix (Sec. 2.2)."""
    N = NaiveDFT(M)
    F = SnfFFT(M)
    rng = np.random.default_rng(4)
    a_pts = rng.standard_normal(N.m) + 1j * rng.standard_normal(N.m)
    # same function values at the same points, in each transform's order
    pn = key(N.points)
    a_f = np.array([a_pts[pn[tuple(p)]] for p in F.points.tolist()])
    hn = key(N.freqs)
    out_n = N.forward(a_pts)
    out_f = F.forward(a_f)
    out_n_in_f = np.array([out_n[hn[tuple(h)]] for h in F.freqs.tolist()])
    assert np.allclose(out_f, out_n_in_f, atol=1e-13)
    assert np.allclose(F.inverse(out_f), a_f, atol=1e-12)
