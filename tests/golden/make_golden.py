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


def c2_uniform_mode():
    """Uniform-mode (Kittel) frequency of the 512x32x4 nanowire of 4 nm
    cells magnetised along its axis x by its anisotropy field 2 Ku/Ms
    (Ku 5e3 J/m^3, Ms 8e5 A/m, no applied field), with the prism's
    demagnetising factors from Aharoni's closed form."""
    a, b, c = 512 * 4e-9 / 2, 32 * 4e-9 / 2, 4 * 4e-9 / 2
    nxx = D.aharoni_prism_factor(b, c, a)
    nyy = D.aharoni_prism_factor(c, a, b)
    nzz = D.aharoni_prism_factor(a, b, c)
    ms, ku = 8e5, 5e3
    mu0ms = I.MU0 * ms
    bk = 2 * ku / ms
    om = I.GAMMA * math.sqrt((bk + (nyy - nxx) * mu0ms) *
                             (bk + (nzz - nxx) * mu0ms))
    return om / (2 * math.pi)


def _write(name, what, f):
    with open(os.path.join(HERE, name), "w") as fh:
        fh.write(f"# {what} (Hz), written by\n"
                 "# tests/golden/make_golden.py from the oracle\n")
        fh.write(f"{f:.9e}\n")
    print(name, f)


if __name__ == "__main__":
    _write("c1_kittel_hz.txt", "Kittel frequency of the small film workload",
           c1_kittel())
    _write("c2_uniform_mode_hz.txt",
           "uniform-mode frequency of the nanowire workload", c2_uniform_mode())
