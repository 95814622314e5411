"""Write spheres_c3_<n>.json: oracle C_eff of the sphere workload on diag(n,n,n).

Random sequential addition of periodic spheres (numpy PCG64 seed 3, radii
U[0.03, 0.08], volume fraction 0.3), matrix E = 1 and inclusions E = 100,
nu = 0.25 (the 3-D precision workload of 256^3, coarsened so that the CPU
FP64 oracle can converge all 6 unit loads: 32^3 to a 1e-10 residual, 64^3 to
1e-8; 256^3 would take days on the host).  Calls only the oracle and the
shared generators.

Usage: python tests/golden/make_spheres.py [n] [tol]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import elasticity as E  # noqa: E402
from oracle.dft import make_transform  # noqa: E402


def main(n=32, tol=1e-10):
    M = [[n, 0, 0], [0, n, 0], [0, 0, n]]
    T = make_transform(M)
    c, r = synth.spheres_rsa(seed=3)
    ph = synth.spheres_phase(T.points, T.m, c, r)
    lame = np.array([synth.lame(1.0, 0.25), synth.lame(100.0, 0.25)])
    t0 = time.time()
    C, runs = E.effective_stiffness(M, ph, lame, E.default_reference(lame), tol=tol, max_iter=5000, transform=T)
    json.dump(dict(_source="tests/golden/make_spheres.py (oracle Algorithm 1, FP64)", n=n, tol=tol,
                   lame=lame.tolist(), n_spheres=int(len(r)), volume_fraction=float(ph.mean()),
                   ceff=C.tolist(), iters=[int(x.iters) for x in runs], seconds=time.time() - t0),
              open(os.path.join(HERE, f"spheres_c3_{n}.json"), "w"), indent=1)


if __name__ == "__main__":
    if len(sys.argv) > 1:
        main(int(sys.argv[1]), float(sys.argv[2]))
    else:
        main()
