"""Writes the stored values under tests/golden/ that come from the oracle.

Calls only oracle/ (and the seeded input module).  Run from the repo root:
    python tests/golden/make_golden.py
"""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import demag as D  # noqa: E402
from paper_2410_00966_amd import inputs as I  # noqa: E402


def c1_kittel():
    """Small-angle Kittel frequency of the uniform mode about +z for the
    32x32x1 film of 5 nm cells in 0.1 T, with the demagnetising factors
    taken as the whole-box average of the oracle's cell tensor."""
    nx, ny, nz, d = 32, 32, 1, 5e-9
    Nf = D.tensor_full(nx, ny, nz, d, d, d)
    cx = nx - np.abs(np.arange(-(nx - 1), nx))
    cy = ny - np.abs(np.arange(-(ny - 1), ny))
    cz = nz - np.abs(np.arange(-(nz - 1), nz))
    w = cz[:, None, None] * cy[None, :, None] * cx[None, None, :]
    avg = np.array([(Nf[c] * w).sum() for c in range(6)]) / (nx * ny * nz)
    mu0ms = I.MU0 * 8e5
    B = 0.1
    om = I.GAMMA * math.sqrt((B + (avg[0] - avg[2]) * mu0ms) *
                             (B + (avg[1] - avg[2]) * mu0ms))
    return om / (2 * math.pi)


if __name__ == "__main__":
    f = c1_kittel()
    with open(os.path.join(HERE, "c1_kittel_hz.txt"), "w") as fh:
        fh.write("# Kittel frequency (Hz) of the small film workload, written by\n"
                 "# tests/golden/make_golden.py from the oracle's tensor\n")
        fh.write(f"{f:.9e}\n")
    print(f)
