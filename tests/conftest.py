import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU oracle checks")


def golden_rows(name):
    """Rows of a whitespace-separated fixture under tests/golden/ ('#' starts a comment)."""
    path = os.path.join(ROOT, "tests", "golden", name)
    rows = []
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


# ----- product checks shared by the GPU tests (host side: the oracle's residues) --------------

def primes61(seed, count):
    """`count` random 61-bit primes from a seeded generator (Miller-Rabin with the first twelve
    prime bases, deterministic below 3.3e24)."""
    import random
    rng = random.Random(seed)
    out = []
    while len(out) < count:
        q = rng.getrandbits(61) | (1 << 60) | 1
        if _isprime(q):
            out.append(q)
    return out


def _isprime(n):
    if n % 2 == 0:
        return False
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def host_residues(arrays, primes, threads=16):
    """[[x mod q for q in primes] for x in arrays], computed by the oracle on the host (ctypes
    releases the interpreter lock, so the calls run on several cores)."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import coracle
    coracle.lib()
    jobs = [(i, j) for i in range(len(arrays)) for j in range(len(primes))]
    out = [[0] * len(primes) for _ in arrays]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for (i, j), r in zip(jobs, ex.map(lambda ij: coracle.residue(arrays[ij[0]], primes[ij[1]]), jobs)):
            out[i][j] = r
    return out


def residues_agree(ra, rb, rc, primes):
    """c = a*b modulo every prime, from residue lists."""
    return all(z == x * y % q for x, y, z, q in zip(ra, rb, rc, primes))


def sha256_limbs(c):
    """SHA-256 of uint32 limbs as little-endian bytes (the digests of tests/golden)."""
    import hashlib
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(c, dtype=np.uint32).astype("<u4").tobytes()).hexdigest()
