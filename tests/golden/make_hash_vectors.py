"""Writes hash_vectors.txt from the oracle's arbitrary-precision hash."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle.hashgrid import spatial_hash_py  # noqa: E402

PTS = [(0, 0, 0), (1, 2, 3), (16, 16, 16), (255, 0, 7), (4096, 4095, 1)]
HEADER = """# Spatial hash test vectors.
# h = (x*1 mod 2^32) xor (y*2654435761 mod 2^32) xor (z*805459861 mod 2^32), then mod T.
# Hash of the multi-resolution hash encoding the paper builds on (Sec. 3, Eq. 3;
# fine levels of Sec. 4.1).  Written by tests/golden/make_hash_vectors.py with
# Python arbitrary-precision integers (oracle.hashgrid.spatial_hash_py).
# x y z h(T=2^14) h(T=2^19)
"""
if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hash_vectors.txt")
    with open(out, "w") as f:
        f.write(HEADER)
        for p in PTS:
            f.write("%d %d %d %d %d\n" % (*p, spatial_hash_py(*p, 1 << 14), spatial_hash_py(*p, 1 << 19)))
