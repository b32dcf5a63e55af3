"""ctypes binding of the C oracle (dkss_oracle.c) -- test infrastructure, not product code.

Only the test suite, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg may use
this module.  Arrays are numpy uint32 limb arrays, little-endian (thesis Sec. 2.1);
polynomials are element-major (element, inner coefficient, limb).
"""
import ctypes
import os
import subprocess

import numpy as np

from . import params as P

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dkss_oracle.c")
_LIB = os.path.join(_HERE, "libdkss_oracle.so")
_lib = None


def build():
    """Compile the C oracle with gcc (plain -O2, no machine-specific tuning)."""
    subprocess.check_call(["gcc", "-O2", "-Wall", "-shared", "-fPIC", "-o", _LIB, _SRC])


_native = {}


def lib_native(dirpath):
    """The same C source built with -O3 -march=native into dirpath (for timing the oracle on the
    machine that runs it; the arithmetic is the source's, only the compiler flags differ)."""
    path = os.path.join(dirpath, "libdkss_oracle_native.so")
    if path not in _native:
        os.makedirs(dirpath, exist_ok=True)
        subprocess.check_call(["gcc", "-O3", "-march=native", "-Wall", "-shared", "-fPIC", "-o", path, _SRC])
        _native[path] = _load(path)
    return _native[path]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _load(_LIB)
    return _lib


def _load(path):
    L = ctypes.CDLL(path)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    sz, lg, i32 = ctypes.c_size_t, ctypes.c_long, ctypes.c_int
    L.or_schoolbook.argtypes = [u32p, u32p, sz, u32p, sz]
    L.or_residue.argtypes = [u32p, sz, ctypes.c_uint64]
    L.or_residue.restype = ctypes.c_uint64
    L.or_mod_reduce.argtypes = [u64p, u64p, i32, u64p, i32]
    L.or_ring_mul.argtypes = [u32p, u32p, u32p, i32, i32, u32p]
    L.or_ring_rotate.argtypes = [u32p, u32p, lg, i32, i32, u32p]
    L.or_encode.argtypes = [u32p, u32p, sz, lg, i32, i32, i32]
    L.or_fft.argtypes = [u32p, lg, i32, i32, u32p, u32p]
    L.or_rho_powers.argtypes = [u32p, lg, i32, i32, u32p, u32p]
    L.or_pointwise.argtypes = [u32p, u32p, u32p, lg, i32, i32, u32p]
    L.or_decode.argtypes = [u32p, sz, u32p, lg, i32, i32, i32, u32p, u32p]
    L.or_decode.restype = i32
    L.or_dkss_mul.argtypes = [u32p, u32p, sz, u32p, sz, lg, i32, i32, i32, u32p, u32p, u32p]
    L.or_dkss_mul.restype = i32
    return L


def _p32(a):
    assert a.dtype == np.uint32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _p64(a):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


# ---- conversions between Python ints and limb arrays ---------------------------------------

def to_limbs(x, n):
    """Python int -> n little-endian uint32 limbs."""
    assert 0 <= x < (1 << (32 * n))
    return np.frombuffer(x.to_bytes(4 * n, "little"), dtype=np.uint32).copy()


def from_limbs(a):
    return int.from_bytes(np.ascontiguousarray(a, dtype=np.uint32).tobytes(), "little")


def coeffs_to_limbs(coeffs, L):
    """list of residues -> flat uint32 array of len(coeffs)*L limbs"""
    return np.concatenate([to_limbs(int(c), L) for c in coeffs]) if coeffs else \
        np.zeros(0, np.uint32)


def limbs_to_coeffs(arr, L):
    arr = np.ascontiguousarray(arr, dtype=np.uint32).reshape(-1, L)
    return [from_limbs(r) for r in arr]


# ---- wrappers ---------------------------------------------------------------------------

def schoolbook(a, b):
    """c = a*b, alen + blen limbs (Sec. 2.3 OMUL)."""
    a = np.ascontiguousarray(a, np.uint32)
    b = np.ascontiguousarray(b, np.uint32)
    c = np.zeros(len(a) + len(b), np.uint32)
    if len(c):
        lib().or_schoolbook(_p32(c), _p32(a), len(a), _p32(b), len(b))
    return c


def residue(a, q):
    a = np.ascontiguousarray(a, np.uint32)
    return int(lib().or_residue(_p32(a), len(a), q))


def mod_reduce(x, q):
    """x mod q with the oracle's long division (for pinning that routine)."""
    W = max(1, -(-q.bit_length() // 64))
    n = max(1, -(-x.bit_length() // 64))
    xa = np.frombuffer(x.to_bytes(8 * n, "little"), np.uint64).copy()
    qa = np.frombuffer(q.to_bytes(8 * W, "little"), np.uint64).copy()
    r = np.zeros(W, np.uint64)
    lib().or_mod_reduce(_p64(r), _p64(xa), n, _p64(qa), W)
    return int.from_bytes(r.tobytes(), "little")


def ring_mul(x, y, m, L, q):
    """product in R = (Z/qZ)[alpha]/(alpha^m+1); x, y lists of m residues"""
    xa, ya = coeffs_to_limbs(x, L), coeffs_to_limbs(y, L)
    r = np.zeros(m * L, np.uint32)
    lib().or_ring_mul(_p32(r), _p32(xa), _p32(ya), m, L, _p32(to_limbs(q, L)))
    return limbs_to_coeffs(r, L)


def ring_rotate(x, e, m, L, q):
    """alpha^e * x in R"""
    xa = coeffs_to_limbs(x, L)
    r = np.zeros(m * L, np.uint32)
    lib().or_ring_rotate(_p32(r), _p32(xa), e, m, L, _p32(to_limbs(q, L)))
    return limbs_to_coeffs(r, L)


def encode(a, M, m, L, u):
    a = np.ascontiguousarray(a, np.uint32)
    poly = np.zeros(2 * M * m * L, np.uint32)
    lib().or_encode(_p32(poly), _p32(a), len(a), M, m, L, u)
    return poly


def fft(poly, M2, m, L, q, rho):
    out = np.ascontiguousarray(poly, np.uint32).copy()
    lib().or_fft(_p32(out), M2, m, L, _p32(to_limbs(q, L)), _p32(coeffs_to_limbs(rho, L)))
    return out


def rho_powers(count, m, L, q, rho):
    out = np.zeros(count * m * L, np.uint32)
    lib().or_rho_powers(_p32(out), count, m, L, _p32(to_limbs(q, L)),
                        _p32(coeffs_to_limbs(rho, L)))
    return out


def pointwise(a, b, count, m, L, q):
    a = np.ascontiguousarray(a, np.uint32)
    b = np.ascontiguousarray(b, np.uint32)
    c = np.zeros_like(a)
    lib().or_pointwise(_p32(c), _p32(a), _p32(b), count, m, L, _p32(to_limbs(q, L)))
    return c


def decode(cc, outlen, M2, m, L, u, q):
    out = np.zeros(outlen, np.uint32)
    inv = pow(M2, -1, q)
    rc = lib().or_decode(_p32(out), outlen, _p32(np.ascontiguousarray(cc, np.uint32)), M2, m, L,
                         u, _p32(to_limbs(q, L)), _p32(to_limbs(inv, L)))
    if rc:
        raise ValueError("decoded bits beyond %d limbs" % outlen)
    return out


def dkss_mul(a, b, setup=None, library=None):
    """c = a*b through Steps 4-8 of Sec. 3.2 in the C oracle.  ``setup`` is an
    ``oracle.params.Setup``; by default the thesis rule for N = 32*max(alen, blen).  ``library``:
    a build of the oracle from lib_native (default: lib())."""
    a = np.ascontiguousarray(a, np.uint32)
    b = np.ascontiguousarray(b, np.uint32)
    n = len(a) + len(b)
    if len(a) == 0 or len(b) == 0:
        return np.zeros(n, np.uint32)
    if setup is None:
        setup = P.setup(P.thesis_rule(32 * max(len(a), len(b))))
    S = setup
    L = S.L
    M2 = 2 * S.params.M
    c = np.zeros(n, np.uint32)
    rc = (library or lib()).or_dkss_mul(_p32(c), _p32(a), len(a), _p32(b), len(b), M2, S.params.m, L,
                           S.params.u, _p32(to_limbs(S.q, L)), _p32(coeffs_to_limbs(S.rho, L)),
                           _p32(to_limbs(pow(M2, -1, S.q), L)))
    if rc:
        raise ValueError("parameters too small for the operands")
    return c
