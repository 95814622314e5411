"""The library's flat parameter layout of the learned-guess network (test helper).

This describes how the library stores the network, not the method: the oracle
network (``oracle/learned.py``) takes plain per-layer (w (Co, Ci, 27), b (Co,))
lists, and the GPU tests convert the library's flat FP32 parameters with these
two functions.  Library layout per layer: W[cout_pad][27][cin_pad], then
b[cout_pad]; the input channels of the first layer are padded to 32, the
output channels of the last layer to 64.
"""
import numpy as np

from oracle.learned import CH, layer_shapes


def _padded(k, co, ci):
    return (64 if k == 14 else co), (32 if k == 0 else ci)


def unflatten(flat, ch=CH):
    """The library's flat parameters -> [(w (Co, Ci, 27), b (Co,))], unpadded."""
    flat = np.asarray(flat, dtype=np.float64)
    out, off = [], 0
    for k, (co, ci) in enumerate(layer_shapes(ch)):
        cop, cip = _padded(k, co, ci)
        W = flat[off: off + cop * 27 * cip].reshape(cop, 27, cip)
        off += cop * 27 * cip
        b = flat[off: off + cop]
        off += cop
        out.append((W[:co, :, :ci].transpose(0, 2, 1).copy(), b[:co].copy()))
    assert off == flat.size
    return out


def flatten(params, ch=CH):
    """Inverse of unflatten (padding entries zero)."""
    parts = []
    for k, ((co, ci), (w, b)) in enumerate(zip(layer_shapes(ch), params)):
        cop, cip = _padded(k, co, ci)
        W = np.zeros((cop, 27, cip))
        W[:co, :, :ci] = w.transpose(0, 2, 1)
        bb = np.zeros(cop)
        bb[:co] = b
        parts += [W.ravel(), bb]
    return np.concatenate(parts)
