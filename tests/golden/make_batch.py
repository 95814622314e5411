"""Oracle values for sampled members of the 512-member 2-D batch workload.

Members: synth.batch_2d_member(seed) for the seeds below (one of them the
largest in seeds 4000..4511), ellipse phases, mean-of-extremes reference,
loads e11, e22 and the Mandel shear; FP64 Basic Scheme to r <= 1e-9.
Writes batch_c4.json next to this file.  Calls only oracle/ and synth/.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import elasticity as E  # noqa: E402
from oracle.dft import make_transform  # noqa: E402


def loads():
    out = np.zeros((3, 2, 2))
    out[0, 0, 0] = 1.0
    out[1, 1, 1] = 1.0
    out[2, 0, 1] = out[2, 1, 0] = 1.0 / np.sqrt(2.0)
    return out


def main():
    dets = {s: abs(int(round(np.linalg.det(synth.batch_2d_member(s)["M"])))) for s in range(4000, 4512)}
    largest = max(dets, key=dets.get)
    seeds = sorted({4000, 4001, 4002, 4003, largest})
    res = dict(tol=1e-9, seeds=seeds, members={})
    for s in seeds:
        mb = synth.batch_2d_member(s)
        M = mb["M"].tolist()
        T = make_transform(M)
        ph = synth.ellipses_phase(T.points, T.m, mb["ellipses"])
        lame = np.array(mb["lame"])
        lame0 = E.default_reference(lame)
        out = []
        for eb in loads():
            r = E.basic_scheme(M, ph, lame, lame0, eb, tol=1e-9, max_iter=20000, transform=T)
            assert r.status == 0, (s, r.status)
            out.append(dict(iters=r.iters, resid=r.resid, mean_stress=r.mean_stress.tolist()))
            print(s, T.m, r.iters, r.resid, flush=True)
        res["members"][str(s)] = dict(M=M, m=T.m, loads=out)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_c4.json"), "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
