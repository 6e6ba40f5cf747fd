"""Reading and computing the per-generation output digests stored beside this file.

A digest is the first 16 hex digits of the SHA-256 of a generation's output
rows, row after row, each cut to its useful bytes (the packet length L; for a
relay's packet rows, N + L).  The stored digests are written from the oracle
by ``make_digests.py``; tests compute the same digest of the GPU's output.
This module does no field arithmetic.
"""
from __future__ import annotations

import hashlib
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def digest_rows(rows: np.ndarray) -> str:
    """Digest of a 2-D uint8 array of output rows (each row already cut to its useful bytes)."""
    return hashlib.sha256(np.ascontiguousarray(rows, dtype=np.uint8).tobytes()).hexdigest()[:16]


def path(name: str) -> str:
    return os.path.join(HERE, "digests_%s.txt" % name)


def read(name: str) -> dict:
    """{generation index: digest} of a stored workload (lines 'index digest', '#' comments)."""
    out = {}
    with open(path(name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            i, d = line.split()
            out[int(i)] = d
    return out


def write(name: str, header: list, items) -> None:
    with open(path(name), "w") as f:
        for h in header:
            f.write("# %s\n" % h)
        for i, d in items:
            f.write("%d %s\n" % (i, d))
