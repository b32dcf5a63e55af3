"""DKSS parameters and ring constants, in Python integers (oracle; test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline
leg may use this module.  Every function cites the thesis passage it follows
(C. Lueders, arXiv 1503.04955).

Contents
  thesis_rule       Sec. 4.1 (Parameter Selection) with Sec. 3.2 Steps 1-2
  proth_prime       Sec. 3.2.2 and Sec. 4.6 (table of primes h*2^n+1, smallest odd h)
  generator         Sec. 3.2.3 (generator zeta of F_p^*)
  hensel_lift       Sec. 3.2.3, Hensel lifting theorem
  principal_root    Sec. 3.2.3 (omega = zeta_z^h)
  rho_lagrange      Sec. 3.2.3, Lagrange interpolation, Eq. (dkss:lagrange)
  setup             all of the above for one multiplication
"""
import math
from dataclasses import dataclass, field


# ----------------------------------------------------------------------------------------------
# Sec. 4.1 Parameter Selection (with Steps 1 and 2 of Sec. 3.2)
# ----------------------------------------------------------------------------------------------

def modulus_bits_rule(N, word=64):
    """Bits of p^z chosen first (Sec. 4.1, Eq. (tightpzbound)): p^z >= N^5 / (2 log N),
    the bit count rounded up to a multiple of the machine word (64 bits in the thesis)."""
    lg = math.log2(N)
    need = math.ceil(5.0 * lg - 1.0 - math.log2(lg))
    return word * max(1, -(-need // word))


def split_rule(N, log2_Mm):
    """M/m = 2^k with k of the parity of log2(Mm), nearest to log2(sqrt(2) * N / log^3 N)
    (Sec. 4.1, last paragraph).  The factor sqrt(2) is this repository's reading: read literally
    (factor 1) the rule contradicts the m that the thesis's memory table implies at 5 of its 16
    lengths, while any factor with log2 in (0.399, 0.516) fits all 16.
    Ties go to the smaller k; m >= 2 and M >= m (Sec. 3.2 Step 1)."""
    lg = math.log2(N)
    target = 0.5 + lg - 3.0 * math.log2(lg)
    best = None
    for k in range(log2_Mm % 2, log2_Mm - 1, 2):   # k <= log2_Mm - 2 keeps m >= 2
        key = (abs(k - target), k)
        if best is None or key < best[0]:
            best = (key, k)
    k = best[1]
    log2_m = (log2_Mm - k) // 2
    return log2_Mm - log2_m, log2_m                   # (log2 M, log2 m)


@dataclass
class Params:
    N: int            # bits per operand (the longer one)
    log2_M: int
    log2_m: int
    u: int            # input bits per inner coefficient
    p_bits: int       # bit length of the prime p
    z: int            # exponent of p in the modulus p^z

    @property
    def M(self):
        return 1 << self.log2_M

    @property
    def m(self):
        return 1 << self.log2_m

    @property
    def mu(self):
        """mu = 2M / 2m (Sec. 3.2 Step 1)."""
        return self.M // self.m


def thesis_rule(N, p_bits=None, z=1):
    """Thesis parameter rule (Sec. 4.1): pick the size of p^z first, then the largest u
    (equivalently the smallest power of two Mm) with p^z >= Mm 2^(2u) (Sec. 3.2 Step 2),
    then split Mm into M and m.  With z = 1 the prime has exactly the chosen number of bits
    and p >= 2^(bits-1), so the bound reads log2(Mm) + 2u <= bits - 1.  For z > 1 the same
    bound uses z * (p_bits - 1), a lower bound of log2(p^z)."""
    if N < 1:
        raise ValueError("N must be positive")
    if p_bits is None:
        p_bits = modulus_bits_rule(N)
    budget = z * (p_bits - 1)
    log2_Mm = 2
    while log2_Mm + 2 * (-(-2 * N // (1 << log2_Mm))) > budget:
        log2_Mm += 1
        if log2_Mm > budget:
            raise ValueError("no feasible Mm for N=%d with %d-bit p, z=%d" % (N, p_bits, z))
    u = -(-2 * N // (1 << log2_Mm))
    log2_M, log2_m = split_rule(N, log2_Mm)
    return Params(N=N, log2_M=log2_M, log2_m=log2_m, u=u, p_bits=p_bits, z=z)


# ----------------------------------------------------------------------------------------------
# Sec. 3.2.2 Finding the prime p; Sec. 4.6 (table of primes h*2^n + 1 with the smallest odd h)
# ----------------------------------------------------------------------------------------------

def _small_factors(h):
    """Prime factors of a small positive integer by trial division."""
    f, d = [], 2
    while d * d <= h:
        if h % d == 0:
            f.append(d)
            while h % d == 0:
                h //= d
        d += 1
    if h > 1:
        f.append(h)
    return f


def is_prime_proth(h, n):
    """Primality of p = h*2^n + 1 (h odd).  If h < 2^n, Proth's theorem: p is prime iff some a
    has a^((p-1)/2) = -1 (mod p); a value other than +-1 proves p composite.  Small p with
    h >= 2^n are decided by trial division."""
    p = h * (1 << n) + 1
    if p < 4:
        return p in (2, 3)
    if h >= (1 << n):
        if p > 1 << 44:
            raise ValueError("trial division range exceeded")
        return all(p % d for d in range(2, math.isqrt(p) + 1))
    for a in range(2, 200):
        if a % p == 0:
            continue
        x = pow(a, (p - 1) // 2, p)
        if x == p - 1:
            return True
        if x != 1:
            return False
    return False   # every tried a a quadratic residue: treat as composite (never seen for primes)


def proth_prime(bits, min_two_power=1):
    """Prime p = h*2^n + 1 with exactly ``bits`` bits, the smallest odd h, n = bits - bitlen(h)
    (Sec. 4.6: one prime per bit length with the smallest odd h), and 2^min_two_power | p - 1
    (Sec. 3.2.2: 2M | p - 1).  Returns (p, h, n)."""
    h = 1
    while True:
        n = bits - h.bit_length()
        if n < min_two_power:
            raise ValueError("no %d-bit prime with 2^%d | p-1" % (bits, min_two_power))
        if is_prime_proth(h, n):
            return h * (1 << n) + 1, h, n
        h += 2


def generator(p, h, n):
    """Smallest generator zeta >= 2 of F_p^* (Sec. 3.2.3), p - 1 = h * 2^n: zeta^((p-1)/r) != 1
    for every prime r dividing p - 1."""
    primes = sorted(set([2] + _small_factors(h)))
    g = 2
    while True:
        if all(pow(g, (p - 1) // r, p) != 1 for r in primes):
            return g
        g += 1


# ----------------------------------------------------------------------------------------------
# Sec. 3.2.3 Computing the root of unity rho
# ----------------------------------------------------------------------------------------------

def hensel_lift(zeta, p, z):
    """Lift a root zeta of f(x) = x^(p-1) - 1 mod p to a root mod p^z (Hensel lifting theorem,
    Sec. 3.2.3): zeta_(s+1) = zeta_s - f(zeta_s) / f'(zeta_s) mod p^(s+1), f'(x) = (p-1) x^(p-2)."""
    zs = zeta % p
    for s in range(1, z):
        mod = p ** (s + 1)
        f = (pow(zs, p - 1, mod) - 1) % mod
        fp = ((p - 1) * pow(zs, p - 2, mod)) % mod
        zs = (zs - f * pow(fp, -1, mod)) % mod
    return zs


def principal_root(zeta_z, p, z, log2_M):
    """omega = zeta_z^h with h = (p-1)/2M, a principal 2M-th root of unity in Z/p^zZ
    (Sec. 3.2.3)."""
    two_M = 1 << (log2_M + 1)
    if (p - 1) % two_M:
        raise ValueError("2M does not divide p-1")
    return pow(zeta_z, (p - 1) // two_M, p ** z)


def _polymul_linear(poly, c, q):
    """poly(alpha) * (alpha - c) over Z/qZ, coefficients lowest first (no reduction)."""
    out = [0] * (len(poly) + 1)
    for i, a in enumerate(poly):
        out[i + 1] = (out[i + 1] + a) % q
        out[i] = (out[i] - a * c) % q
    return out


def rho_lagrange(omega, m, mu, q):
    """rho(alpha) by Lagrange interpolation through (gamma^i, omega^i), i odd < 2m, with
    gamma = omega^mu (Sec. 3.2.3, Eq. (dkss:lagrange)).  Returns m coefficients mod q."""
    gamma = pow(omega, mu, q)
    odd = list(range(1, 2 * m, 2))
    rho = [0] * m
    for i in odd:
        num = [1]
        den = 1
        for j in odd:
            if j == i:
                continue
            gj = pow(gamma, j, q)
            num = _polymul_linear(num, gj, q)
            den = den * (pow(gamma, i, q) - gj) % q
        scale = pow(omega, i, q) * pow(den, -1, q) % q
        assert len(num) == m
        for k in range(m):
            rho[k] = (rho[k] + scale * num[k]) % q
    return rho


@dataclass
class Setup:
    params: Params
    p: int
    h: int            # p = h * 2^n + 1
    n: int
    q: int            # modulus p^z
    zeta: int
    zeta_z: int
    omega: int
    rho: list = field(repr=False)

    @property
    def d(self):
        return self.q.bit_length()

    @property
    def L(self):
        """uint32 limbs per inner coefficient."""
        return -(-self.d // 32)


def setup(params):
    """Steps 2 and 3 of Sec. 3.2 for given parameters: prime, generator, Hensel lift, omega,
    rho.  Checks p^z >= Mm 2^(2u) (Sec. 3.2.2)."""
    P = params
    p, h, n = proth_prime(P.p_bits, P.log2_M + 1)
    q = p ** P.z
    if q < (1 << (P.log2_M + P.log2_m + 2 * P.u)):
        raise ValueError("p^z below Mm 2^(2u)")
    zeta = generator(p, h, n)
    zeta_z = hensel_lift(zeta, p, P.z)
    omega = principal_root(zeta_z, p, P.z, P.log2_M)
    rho = rho_lagrange(omega, P.m, P.mu, q)
    return Setup(params=P, p=p, h=h, n=n, q=q, zeta=zeta, zeta_z=zeta_z, omega=omega, rho=rho)
