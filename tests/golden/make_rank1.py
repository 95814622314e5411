"""Write rank1_c2.json: the seeded rank-1 lattice of the 3-D Hashin workload.

Korobov generating vector z = (1, a, a^2 mod m), m = 2^21; a is the odd
candidate (4096 drawn with numpy PCG64 seed 2) whose dual lattice
{h : h . z = 0 mod m} has the longest LLL-reduced shortest vector; M^T is
that reduced dual basis (synth.rank1_generator).
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402


def main():
    m = 2 ** 21
    a, M = synth.rank1_generator(m, seed=2, candidates=4096)
    json.dump(dict(_source="tests/golden/make_rank1.py (synth.rank1_generator, seed 2, 4096 candidates)",
                   m=m, a=int(a), z=[1, int(a), int(a * a % m)], M=M.tolist()),
              open(os.path.join(HERE, "rank1_c2.json"), "w"), indent=1)


if __name__ == "__main__":
    main()
