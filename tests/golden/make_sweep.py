"""Write sweep_example_4_1.json: closed-form data of the Sec. 5.1 shear sweep.

Calls only the oracle (closed forms of Sec. 4.2).  Structure: the coated
ellipse of Example 4.1 (c1 = 0.05, c2 = 0.35, c3 = infinity, rho_c = 0,
rho_e = 0.09, direction n at 60 degrees read as (1/2, sqrt(3)/2, 0)); core
E = 10, coating E = 0.5, nu = 0.3 (the paper gives no materials); matrix =
the neutral isotropic material; load = the assemblage's eps0.
"""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import closed_forms as CF  # noqa: E402
from oracle import elasticity as E  # noqa: E402


def main():
    c = [0.05, 0.35, math.inf]
    R = CF.rotation_e1_to([0.5, math.sqrt(3) / 2, 0.0])
    lc, le = E.lame_from_young(10.0, 0.3), E.lame_from_young(0.5, 0.3)
    h = CF.hashin(c, 0.0, 0.09, lc, le, R)
    out = dict(
        _source="tests/golden/make_sweep.py (oracle closed form, Sec. 4.2; Example 4.1 geometry)",
        c12=c[:2], c3="infinity", rho_c=0.0, rho_e=0.09, R=R.tolist(),
        lame_core=list(lc), lame_coating=list(le), lame_matrix=list(h["lame_m"]),
        eps0=h["eps0"].tolist(), ceff_eps0=h["ceff_eps0"].tolist(),
    )
    with open(os.path.join(HERE, "sweep_example_4_1.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
