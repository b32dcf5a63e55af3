"""Writes dkss_digests.txt: SHA-256 digests of products computed once by the CPU oracle's DKSS.

The products at 2^28 and 2^30 bits per operand take the oracle minutes each, too long for a
test run; their digests are stored instead, and the GPU tests compare the SHA-256 of their
own limbs (little-endian uint32 bytes) with them.  Only ``oracle/`` and ``seeded_inputs`` are
used here: operands from the seeded splitmix64 stream, products from ``coracle.dkss_mul``
(Steps 4-8 of Sec. 3.2 with the thesis's parameter rule, Sec. 4.1).

    python tests/golden/make_dkss_digests.py [--jobs J] [name ...]

Each case runs in its own process (the oracle is single-threaded).
"""
import argparse
import hashlib
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import seeded_inputs as SI  # noqa: E402

OUT = os.path.join(HERE, "dkss_digests.txt")

# name -> (seed of the operand pair or of the squared operand, alen, blen, squaring)
N28 = 1 << 23          # limbs of a 2^28-bit operand
N30 = 1 << 25          # limbs of a 2^30-bit operand
CASES = {
    "2p28_random": (SI.SEED_BASE + 2, N28, N28, False),
    "2p28_square": (SI.SEED_BASE + 3, N28, N28, True),
    "2p28_unbalanced": (SI.SEED_BASE + 4, N28, N28 // 8, False),
    "2p30_heldout": (SI.SEED_BASE + 30, N30, N30, False),
}


def operands(name):
    seed, alen, blen, square = CASES[name]
    if square:
        a = SI.limbs(seed, alen)
        return a, a
    return SI.operand_pair(seed, alen, blen)


def digest(c):
    return hashlib.sha256(c.astype("<u4").tobytes()).hexdigest()


def run_case(name):
    from oracle import coracle
    a, b = operands(name)
    t0 = time.time()
    c = coracle.dkss_mul(a, b)
    return name, digest(c), time.time() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("names", nargs="*")
    args = ap.parse_args()
    names = args.names or list(CASES)
    from oracle import coracle
    coracle.lib()                       # build once before the workers start
    rows = {}
    if os.path.exists(OUT):
        for line in open(OUT):
            if line.strip() and not line.startswith("#"):
                f = line.split()
                rows[f[0]] = line.rstrip("\n")
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        for name, dg, secs in ex.map(run_case, names):
            seed, alen, blen, square = CASES[name]
            rows[name] = "%s %d %d %d %d %s" % (name, seed, alen, blen, int(square), dg)
            print("%s: %.0f s %s" % (name, secs, dg), flush=True)
    with open(OUT, "w") as f:
        f.write("# SHA-256 of the little-endian uint32 limbs of products computed by the CPU oracle's\n")
        f.write("# DKSS (thesis rule, Sec. 4.1; Steps 4-8 of Sec. 3.2), written by make_dkss_digests.py.\n")
        f.write("# Operands: seeded_inputs (splitmix64); squaring: the operand drawn by limbs(seed, alen).\n")
        f.write("# columns: name seed alen blen squaring sha256\n")
        for name in CASES:
            if name in rows:
                f.write(rows[name] + "\n")


if __name__ == "__main__":
    main()
