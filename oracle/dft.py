"""Pattern DFT F(M) (oracle; test infrastructure only).

Sec. 2.2, eq. Fouriermatrix: F(M) = (1/m) (exp(-2 pi i h^T y)), rows
h in G(M^T), columns y in P(M).  The inverse is the plain sum
a_y = sum_h ahat_h exp(+2 pi i h^T y) (collocation formula of Sec. 3.2).

Two routes:
* ``NaiveDFT``: the matrix written out with exact integer phases
  r = (h . p) mod m for y = p/m, O(m^2); for small patterns.
* ``SnfFFT``: the oracle's own Smith-normal-form addressing (see
  ``lattice.SnfIndexing``) and a library d_M-dimensional FFT (scipy.fft,
  threaded over the host cores; ``AHOM_ORACLE_WORKERS`` caps the threads), as
  Sec. 2.2 states the pattern DFT reduces to one.  Cross-checked against
  NaiveDFT.
Both act on the last axes of arrays shaped (..., m) in the point order /
frequency order the object exposes as ``points`` / ``freqs``.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft

from .lattice import SnfIndexing, int_det, as_int_matrix, pattern_points, generating_set, transpose


class NaiveDFT:
    def __init__(self, M, points=None, freqs=None):
        self.M = as_int_matrix(M)
        self.m = abs(int_det(self.M))
        self.points = pattern_points(self.M) if points is None else np.asarray(points, np.int64)
        self.freqs = generating_set(transpose(self.M)) if freqs is None else np.asarray(freqs, np.int64)
        if self.m > 8192:
            raise ValueError("NaiveDFT is O(m^2); use SnfFFT for large patterns")
        r = (self.freqs.astype(object).dot(self.points.astype(object).T)) % self.m
        r = np.array(r, dtype=np.int64)
        roots = np.exp(-2j * np.pi * np.arange(self.m) / self.m)
        self.F = roots[r] / self.m          # rows h, columns y
        self.Finv = np.conj(roots[r]).T     # rows y, columns h

    def forward(self, a):
        return np.asarray(a) @ self.F.T

    def inverse(self, ahat):
        return np.asarray(ahat) @ self.Finv.T


def fft_workers():
    """Threads of the library FFT: all host cores unless AHOM_ORACLE_WORKERS is set."""
    env = os.environ.get("AHOM_ORACLE_WORKERS")
    return max(1, int(env)) if env else (os.cpu_count() or 1)


class SnfFFT:
    def __init__(self, M):
        self.idx = SnfIndexing(M)
        self.m = self.idx.m
        self.points = self.idx.points()
        self.freqs = self.idx.freqs()
        self.shape = self.idx.shape

    def forward(self, a):
        a = np.asarray(a)
        lead = a.shape[:-1]
        A = a.reshape(lead + self.shape)
        axes = tuple(range(len(lead), len(lead) + len(self.shape)))
        return (scipy.fft.fftn(A, axes=axes, workers=fft_workers()) / self.m).reshape(lead + (self.m,))

    def inverse(self, ahat):
        ahat = np.asarray(ahat)
        lead = ahat.shape[:-1]
        A = ahat.reshape(lead + self.shape)
        axes = tuple(range(len(lead), len(lead) + len(self.shape)))
        return (scipy.fft.ifftn(A, axes=axes, workers=fft_workers()) * self.m).reshape(lead + (self.m,))


def make_transform(M, naive_limit=1024):
    """NaiveDFT for small patterns, SnfFFT otherwise."""
    m = abs(int_det(as_int_matrix(M)))
    return NaiveDFT(M) if m <= naive_limit else SnfFFT(M)
