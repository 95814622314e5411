"""Helpers shared by the GPU parity tests (no arithmetic of the method)."""
import numpy as np


def perm_between(src, dst):
    """idx with src[idx] == dst, for two integer point/frequency lists (same set)."""
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    os_ = np.lexsort(src.T[::-1])
    od = np.lexsort(dst.T[::-1])
    assert np.array_equal(src[os_], dst[od]), "point sets differ"
    idx = np.empty(len(dst), np.int64)
    idx[od] = os_
    return idx


COMP3 = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
COMP2 = [(0, 0), (1, 1), (0, 1)]


def fields_to_tensors(f, d):
    """(ncomp, m) plain components -> (d, d, m) symmetric tensors."""
    comps = COMP3 if d == 3 else COMP2
    m = f.shape[-1]
    t = np.zeros((d, d, m))
    for c, (i, j) in enumerate(comps):
        t[i, j] = f[c]
        t[j, i] = f[c]
    return t


def tensors_to_fields(t):
    d = t.shape[0]
    comps = COMP3 if d == 3 else COMP2
    return np.stack([t[i, j] for i, j in comps])


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
