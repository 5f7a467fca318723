"""OVF 2.0 field files (the OOMMF vector-field format Mumax3 reads and
writes): per-cell maps such as a cavity's vacuum field B_rms exported from a
field solver, or Ms / Ku maps, in and out of the (valuedim, nz, ny, nx)
arrays the library takes (Problem.brms_map, ms_map, ku1_map).

Format (OVF 2.0): a text header of "# key: value" lines between
"# Begin: Header" and "# End: Header" (xnodes, ynodes, znodes, valuedim,
x/y/zstepsize, ...), then one data block, "# Begin: Data Text", "Data
Binary 4" or "Data Binary 8".  Nodes run x fastest, then y, then z, with
the valuedim components of a node adjacent.  Binary blocks are little-endian
and start with a check value (1234567.0 as float32, 123456789012345.0 as
float64).  Host-side file handling only; nothing here runs on the device.
"""
from __future__ import annotations

import numpy as np

_CHECK = {4: (np.dtype("<f4"), 1234567.0), 8: (np.dtype("<f8"),
                                                 123456789012345.0)}


def read_ovf(path):
    """Returns (array (valuedim, nz, ny, nx), header dict of strings).
    The array is float32 for text and Binary 4 data, float64 for Binary 8."""
    with open(path, "rb") as f:
        raw = f.read()
    header = {}
    pos = 0
    while True:
        end = raw.index(b"\n", pos)
        line = raw[pos:end].decode("ascii", "replace").strip()
        pos = end + 1
        if not line.startswith("#"):
            continue
        body = line[1:].strip()
        low = body.lower()
        if low.startswith("begin: data"):
            kind = low[len("begin: data"):].strip()
            break
        if ":" in body:
            k, v = body.split(":", 1)
            header[k.strip().lower()] = v.strip()
    nx, ny, nz = (int(header[k]) for k in ("xnodes", "ynodes", "znodes"))
    vd = int(header.get("valuedim", "1"))
    n = nx * ny * nz * vd
    if kind.startswith("binary"):
        width = int(kind.split()[1])
        if width not in _CHECK:
            raise ValueError(f"unsupported OVF data block: {kind}")
        dt, check = _CHECK[width]
        vals = np.frombuffer(raw, dtype=dt, count=n + 1, offset=pos)
        if vals[0] != check:
            raise ValueError("OVF binary check value mismatch")
        data = vals[1:].astype(dt.newbyteorder("="))
    elif kind.startswith("text"):
        stop = raw.index(b"# End: Data", pos)
        data = np.array(raw[pos:stop].split(), dtype=np.float32)
        if data.size != n:
            raise ValueError(f"OVF text block has {data.size} values, "
                             f"expected {n}")
    else:
        raise ValueError(f"unsupported OVF data block: {kind}")
    arr = data.reshape(nz, ny, nx, vd).transpose(3, 0, 1, 2)
    return np.ascontiguousarray(arr), header


def write_ovf(path, arr, cell, title="field", units="1", binary=4):
    """Writes `arr` (valuedim, nz, ny, nx) on cells of size `cell` = (dx, dy,
    dz) metres.  binary: 4 or 8 (Binary 4 / 8 data), 0 for text."""
    arr = np.asarray(arr)
    if arr.ndim == 3:
        arr = arr[None]
    vd, nz, ny, nx = arr.shape
    dx, dy, dz = cell
    labels = " ".join(f"{title}_{c}" for c in "xyz"[:vd]) if vd <= 3 else \
        " ".join(f"{title}_{i}" for i in range(vd))
    head = [
        "# OOMMF OVF 2.0", "# Segment count: 1", "# Begin: Segment",
        "# Begin: Header", f"# Title: {title}", "# meshtype: rectangular",
        "# meshunit: m", "# xmin: 0", "# ymin: 0", "# zmin: 0",
        f"# xmax: {nx * dx!r}", f"# ymax: {ny * dy!r}", f"# zmax: {nz * dz!r}",
        f"# valuedim: {vd}", f"# valuelabels: {labels}",
        f"# valueunits: {' '.join([units] * vd)}",
        f"# xbase: {dx / 2!r}", f"# ybase: {dy / 2!r}", f"# zbase: {dz / 2!r}",
        f"# xnodes: {nx}", f"# ynodes: {ny}", f"# znodes: {nz}",
        f"# xstepsize: {dx!r}", f"# ystepsize: {dy!r}",
        f"# zstepsize: {dz!r}", "# End: Header"]
    nodes = arr.transpose(1, 2, 3, 0).reshape(-1)
    with open(path, "wb") as f:
        f.write(("\n".join(head) + "\n").encode("ascii"))
        if binary:
            dt, check = _CHECK[binary]
            f.write(f"# Begin: Data Binary {binary}\n".encode("ascii"))
            f.write(np.asarray([check], dtype=dt).tobytes())
            f.write(nodes.astype(dt).tobytes())
            f.write(f"\n# End: Data Binary {binary}\n".encode("ascii"))
        else:
            f.write(b"# Begin: Data Text\n")
            rows = nodes.reshape(-1, vd)
            for r in rows:
                f.write((" ".join(repr(float(v)) for v in r) + "\n")
                        .encode("ascii"))
            f.write(b"# End: Data Text\n")
        f.write(b"# End: Segment\n")
