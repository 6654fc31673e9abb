"""Write unary_f32_digests.json: the oracle's binary32 results of exp, sqrt, abs and
neg over all 2^32 bit patterns, as one SHA-256 digest per chunk of 2^26 consecutive
patterns (pattern k * 2^26 + i, i = 0 .. 2^26 - 1).

Results are the oracle's (oracle/elementwise.py): exp correctly rounded, sqrt the
binary64 square root rounded to binary32 (exact rounding, 53 >= 2 * 24 + 2), abs and
neg the sign operations.  Every NaN result is written as the pattern 0x7FC00000 before
hashing (a NaN's payload is not part of the semantics); all other results hash their
exact bits, signed zeros included.  Calls only the oracle; run from the repository
root:  python tests/golden/make_unary_digests.py  (a few minutes on 8 cores)."""
from __future__ import annotations

import hashlib
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

CHUNK_BITS = 26
N_CHUNKS = 1 << (32 - CHUNK_BITS)
OPS = ("exp", "sqrt", "abs", "neg")
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "unary_f32_digests.json")
CANON_NAN = 0x7FC00000


def patterns(k: int) -> np.ndarray:
    """Chunk k of the binary32 bit patterns, as float32 values."""
    base = np.uint64(k) << np.uint64(CHUNK_BITS)
    return (np.arange(1 << CHUNK_BITS, dtype=np.uint64) + base).astype(np.uint32).view(np.float32)


def digest(y: np.ndarray) -> str:
    """SHA-256 of binary32 results with every NaN written as 0x7FC00000."""
    b = np.ascontiguousarray(y, dtype=np.float32).view(np.uint32).copy()
    b[np.isnan(y)] = CANON_NAN
    return hashlib.sha256(memoryview(b).cast("B")).hexdigest()


def oracle_chunk(args) -> str:
    op, k = args
    from oracle import elementwise as ew
    x = patterns(k)
    with np.errstate(all="ignore"):
        y = ew.evaluate([("load", 0), (op,)], [x.reshape(-1, 1)], [], "f32").ravel()
    return digest(y)


def main():
    jobs = [(op, k) for op in OPS for k in range(N_CHUNKS)]
    with Pool(min(8, os.cpu_count() or 1)) as p:
        res = p.map(oracle_chunk, jobs, chunksize=1)
    out = {"what": "SHA-256 per chunk of 2^26 binary32 patterns of the oracle's results, NaN as 0x7FC00000",
           "chunk_bits": CHUNK_BITS, "digests": {}}
    for (op, k), d in zip(jobs, res):
        out["digests"].setdefault(op, []).append(d)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
