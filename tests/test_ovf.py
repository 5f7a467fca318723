"""OVF 2.0 files (paper_2410_00966_amd/ovf.py), CPU only.

* A hand-written text file (tests/golden/ovf_text_2x1x2.ovf, a format
  example, not data): nodes run x fastest, then y, then z, with the
  components of a node adjacent, so node (x=1, y=0, z=1) holds (10, 11, 12).
* Round trips in Binary 4, Binary 8 and text keep shape and values; a
  corrupted check value is refused.
"""
import os

import numpy as np
import pytest

from paper_2410_00966_amd.ovf import read_ovf, write_ovf

HERE = os.path.dirname(__file__)


def test_text_fixture_node_order():
    arr, head = read_ovf(os.path.join(HERE, "golden", "ovf_text_2x1x2.ovf"))
    assert arr.shape == (3, 2, 1, 2)
    assert list(arr[:, 0, 0, 0]) == [1, 2, 3]
    assert list(arr[:, 0, 0, 1]) == [4, 5, 6]
    assert list(arr[:, 1, 0, 0]) == [7, 8, 9]
    assert list(arr[:, 1, 0, 1]) == [10, 11, 12]
    assert float(head["zstepsize"]) == 3e-9


@pytest.mark.parametrize("binary", [4, 8, 0])
def test_round_trip(tmp_path, binary):
    rng = np.random.default_rng(7001 + binary)
    a = rng.normal(size=(3, 2, 5, 7)).astype(np.float32)
    path = tmp_path / f"f{binary}.ovf"
    write_ovf(path, a, (4e-9, 5e-9, 3e-9), title="B_rms", units="T",
              binary=binary)
    b, head = read_ovf(path)
    assert b.shape == a.shape
    assert np.array_equal(b.astype(np.float32), a)
    assert int(head["xnodes"]) == 7 and int(head["znodes"]) == 2
    s = read_ovf(path)[0]
    assert s.dtype == (np.float64 if binary == 8 else np.float32)


def test_scalar_map_and_bad_check(tmp_path):
    ms = np.full((1, 4, 3), 8e5, np.float32)
    path = tmp_path / "ms.ovf"
    write_ovf(path, ms, (4e-9, 4e-9, 4e-9), title="Msat", units="A/m")
    got, _ = read_ovf(path)
    assert got.shape == (1, 1, 4, 3) and np.array_equal(got[0], ms)
    raw = bytearray(path.read_bytes())
    i = raw.index(b"# Begin: Data Binary 4\n") + len(b"# Begin: Data Binary 4\n")
    raw[i] ^= 0xFF
    path.write_bytes(bytes(raw))
    with pytest.raises(ValueError):
        read_ovf(path)
