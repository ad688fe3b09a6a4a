"""Write the oracle's regular/chaotic labels of the 32x32 Henon-Heiles
section grid at E = 0.125 (dt = 0.01, T = 1e4, two seeded deviation vectors
from seeded_inputs with seed 1001, K = 10, threshold 1e-8).

Calls only the oracle and the seeded-input module.  Output:
tests/golden/hh_e0125_32x32_T1e4.txt with one line per grid point:
index, label (-1 masked, 0 regular, 1 chaotic), min SALI.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import seeded_inputs as S  # noqa: E402
from oracle import oracle as O  # noqa: E402

OUT = os.path.join(HERE, "hh_e0125_32x32_T1e4.txt")


def main(threads=8):
    x0, mask = O.hh_grid(0.125, 32, 32)
    w0 = S.deviation_vectors(1001, len(x0), 2, 4)
    run = O.Run(dt=0.01, T=1e4, indicators=O.IND_SALI)
    r = O.integrate(O.henon_heiles(), x0, run, w0=w0, mask=mask, threads=threads)
    with open(OUT, "w") as f:
        f.write("# oracle labels, Henon-Heiles E=0.125 32x32 section grid, dt=0.01 T=1e4,"
                " seed 1001 (tests/golden/make_hh_labels.py)\n")
        for i in range(len(x0)):
            f.write(f"{i} {int(r['label'][i])} {r['sali_min'][i]:.17g}\n")
    print("chaotic fraction", np.mean(r["label"][mask == 1] == 1))


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 8)
