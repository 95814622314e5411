"""The allocation-free pattern DFT (ahom_dft_noalloc) against ahom_dft, through the C ABI."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
ahom = pytest.importorskip("paper_1605_05712_amd.ahom")


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def test_dft_noalloc_equals_dft_on_two_calls_in_a_row():
    """Two patterns in a row, the second smaller: every output equals the
    allocating entry point's bit for bit (same kernels, same order), in FP64 and
    FP32, forward and inverse; a pattern beyond the scratch is refused."""
    rng = np.random.default_rng(3)
    for M in ([[64, 0, 0], [0, 32, 0], [3, 0, 64]], [[24, 0], [0, 360]]):
        P = ahom.Pattern(M)
        for prec, dt in ((ahom.FP64, np.complex128), (ahom.FP32_MIXED, np.complex64)):
            a = (rng.standard_normal(P.m) + 1j * rng.standard_normal(P.m)).astype(dt)
            d_in = ahom.DeviceArray.from_numpy(a)
            for sign in (-1, 1):
                say("dft_noalloc", M, "m", P.m, "prec", prec, "sign", sign)
                ref = P.dft(d_in, sign, prec).numpy()
                out = ahom.DeviceArray((P.m,), dt)
                P.dft_noalloc(d_in, out, sign, prec)
                assert np.array_equal(out.numpy(), ref)
    big = ahom.Pattern([[4096, 0], [0, 1024]])      # 2^22 points
    say("dft_noalloc refused", big.m)
    d = ahom.DeviceArray((16,), np.complex128)
    with pytest.raises(ahom.AhomError) as ex:
        big.dft_noalloc(d, d)
    assert ex.value.code == ahom.AHOM_E_ARG
