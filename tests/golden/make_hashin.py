"""Write hashin_c2.json: closed-form data of the 3-D coated-ellipsoid workload.

Calls only the oracle (closed forms of Sec. 4.2) and the shared geometry
generator.  Geometry: semi-axes (0.15, 0.2, 0.3), rho_c = 0, coating 0.1 of
the cell, rotation from Euler seed 2; core E = 10, coating E = 0.5, nu = 0.3;
matrix = the neutral isotropic material (mu_m = mu_e).
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import closed_forms as CF  # noqa: E402
from oracle import elasticity as E  # noqa: E402


def main():
    g = synth.hashin_geometry(seed=2)
    lc, le = E.lame_from_young(10.0, 0.3), E.lame_from_young(0.5, 0.3)
    h = CF.hashin(g["c"], g["rho_c"], g["rho_e"], lc, le, g["R"])
    out = dict(
        _source="tests/golden/make_hashin.py (oracle closed form, Sec. 4.2)",
        c=g["c"].tolist(), rho_c=g["rho_c"], rho_e=g["rho_e"], R=g["R"].tolist(), seed=2,
        lame_core=list(lc), lame_coating=list(le), lame_matrix=list(h["lame_m"]),
        eps0=h["eps0"].tolist(), ceff_eps0=h["ceff_eps0"].tolist(), f=h["f"],
    )
    with open(os.path.join(HERE, "hashin_c2.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
