"""Writes the stored tail references the GPU tests compare with.  Calls only the oracle.

tail_reference_interim.txt -- the interim-mass case of Sec. 3.2 (m = 0.1, phi_in = phi_UV =
sqrt 42, dN = 1e-3) on bins of width 0.02 over [9.2, 15]: the bin-averaged log density of N on the
simulation's lattice from Daniels' saddle-point density with the exact cumulant generating
function (`refmath.saddlepoint_walled_reference`, no truncation of cumulants), and that
reference's own error (the size of Daniels' second-order term, squared).  It takes a few
minutes, so the GPU tests read it from here.

Run from the repository root:  python tests/golden/make_tail_references.py
"""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O                      # noqa: E402
from oracle import refmath as R         # noqa: E402


def interim_edges():
    return np.round(np.arange(9.2, 15.0 + 1e-9, 0.02), 10)


def main():
    phi = math.sqrt(42.0)
    model = O.Model(m=0.1, phi_in=phi, phi_uv=phi, dN=1e-3)
    edges = interim_edges()
    ref, err = R.saddlepoint_walled_reference(model, edges)
    path = os.path.join(HERE, "tail_reference_interim.txt")
    with open(path, "w") as f:
        f.write("# Interim-mass case of Sec. 3.2: m = 0.1, phi_in = phi_UV = sqrt 42, dN = 1e-3.\n")
        f.write("# Bin j covers N in (e_j, e_j+1], e = 9.2 + 0.02 j.  Columns: j, e_j, e_j+1,\n")
        f.write("# log P_j (natural log of the bin-averaged density on the k dN lattice, saddle-point\n")
        f.write("# density with the exact cumulant generating function), error of log P_j.\n")
        f.write("# Written by tests/golden/make_tail_references.py (oracle only).\n")
        for j in range(len(ref)):
            f.write(f"{j} {edges[j]:.2f} {edges[j + 1]:.2f} {ref[j]:.12e} {err[j]:.3e}\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
