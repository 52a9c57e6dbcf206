"""Writes the stored oracle values under tests/golden/.

Calls only the FP64 oracle and the seeded input generators; run it after a
deliberate change to the oracle's arithmetic and name, in the commit, the
passage of the paper that justifies the change.

    python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import gs  # noqa: E402
from paper_1302_0120_amd import synth  # noqa: E402


def main():
    m, phi0 = synth.spot_problem(synth.SPOTS_64)
    res = gs.gs_solve(m, phi0, synth.SPOTS_64.n_iter)
    path = os.path.join(HERE, "gs_spots64_history.txt")
    with open(path, "w") as f:
        f.write("# FP64 oracle history [E_F^0, G^0, ..., E_F^99, G^99, E_F^100] for the\n")
        f.write("# 64x64 five-spot workload (seed 1, sigma 1.5 px, unit amplitude,\n")
        f.write("# uniform initial phase), 100 iterations.  Written by make_golden.py.\n")
        for v in res["history"]:
            f.write(f"{v:.17e}\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
