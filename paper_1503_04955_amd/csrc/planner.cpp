// Host-side planning for DKSS multiplication (thesis Sec. 3.2 Steps 1-3 and Sec. 4.1).
#include "planner.hpp"

#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>

namespace dkss {

// ---------------------------------------------------------------------------------------------
// Big
// ---------------------------------------------------------------------------------------------

bool Big::is_zero() const {
    for (int i = 0; i < kWords; ++i)
        if (w[i]) return false;
    return true;
}

int Big::bitlen() const {
    for (int i = kWords - 1; i >= 0; --i)
        if (w[i]) return 64 * i + 64 - __builtin_clzll(w[i]);
    return 0;
}

int Big::cmp(const Big& o) const {
    for (int i = kWords - 1; i >= 0; --i)
        if (w[i] != o.w[i]) return w[i] < o.w[i] ? -1 : 1;
    return 0;
}

Big Big::shl(int s) const {
    Big r;
    int ws = s / 64, bs = s % 64;
    for (int i = kWords - 1; i >= ws; --i) {
        uint64_t v = w[i - ws] << bs;
        if (bs && i - ws - 1 >= 0) v |= w[i - ws - 1] >> (64 - bs);
        r.w[i] = v;
    }
    return r;
}

Big Big::shr(int s) const {
    Big r;
    int ws = s / 64, bs = s % 64;
    for (int i = 0; i + ws < kWords; ++i) {
        uint64_t v = w[i + ws] >> bs;
        if (bs && i + ws + 1 < kWords) v |= w[i + ws + 1] << (64 - bs);
        r.w[i] = v;
    }
    return r;
}

Big Big::add(const Big& o) const {
    Big r;
    unsigned __int128 c = 0;
    for (int i = 0; i < kWords; ++i) {
        c += (unsigned __int128)w[i] + o.w[i];
        r.w[i] = (uint64_t)c;
        c >>= 64;
    }
    return r;
}

Big Big::sub(const Big& o) const {
    Big r;
    uint64_t borrow = 0;
    for (int i = 0; i < kWords; ++i) {
        uint64_t a = w[i], b = o.w[i];
        uint64_t d = a - b - borrow;
        borrow = (a < b) || (a - b < borrow) ? 1 : 0;
        r.w[i] = d;
    }
    return r;
}

Big Big::mul(const Big& o) const {
    Big r;
    for (int i = 0; i < kWords; ++i) {
        if (!w[i]) continue;
        unsigned __int128 c = 0;
        for (int j = 0; i + j < kWords; ++j) {
            c += (unsigned __int128)w[i] * o.w[j] + r.w[i + j];
            r.w[i + j] = (uint64_t)c;
            c >>= 64;
        }
    }
    return r;
}

// ---------------------------------------------------------------------------------------------
// ModQ
// ---------------------------------------------------------------------------------------------

Big ModQ::reduce(const Big& x) const {
    Big r;
    for (int i = x.bitlen() - 1; i >= 0; --i) {
        r = r.shl(1);
        if (x.bit(i)) r.w[0] |= 1;
        if (r.cmp(q) >= 0) r = r.sub(q);
    }
    return r;
}

Big ModQ::add(const Big& x, const Big& y) const {
    Big s = x.add(y);
    if (s.cmp(q) >= 0) s = s.sub(q);
    return s;
}

Big ModQ::sub(const Big& x, const Big& y) const {
    if (x.cmp(y) >= 0) return x.sub(y);
    return x.add(q).sub(y);
}

Big ModQ::mul(const Big& x, const Big& y) const {
    Big r;
    for (int i = y.bitlen() - 1; i >= 0; --i) {
        r = add(r, r);
        if (y.bit(i)) r = add(r, x);
    }
    return r;
}

Big ModQ::pow(const Big& x, const Big& e) const {
    Big r = reduce(Big::of(1));
    Big b = reduce(x);
    for (int i = e.bitlen() - 1; i >= 0; --i) {
        r = mul(r, r);
        if (e.bit(i)) r = mul(r, b);
    }
    return r;
}

Big ModQ::half(const Big& x) const {
    if (!(x.w[0] & 1)) return x.shr(1);
    return x.add(q).shr(1);
}

// ---------------------------------------------------------------------------------------------
// Parameter rule (Sec. 4.1 with Sec. 3.2 Steps 1-2)
// ---------------------------------------------------------------------------------------------

bool thesis_params(uint64_t N, int* log2_M, int* log2_m, int* u, int* p_bits) {
    if (N == 0 || N > (1ULL << 40)) return false;
    // bits of p^z first: p^z >= N^5 / (2 log N), rounded up to a multiple of 64 bits
    double lg = std::log2((double)N);
    if (lg < 1.0) lg = 1.0;
    long need = (long)std::ceil(5.0 * lg - 1.0 - std::log2(lg));
    int d = 64 * (int)((need + 63) / 64);
    if (d < 64) d = 64;
    // smallest power of two Mm = 2^t (t >= 2) with t + 2 ceil(2N / 2^t) <= d - 1
    int t = 2;
    for (;; ++t) {
        if (t > 62) return false;
        uint64_t uu = ((2 * N) + (1ULL << t) - 1) >> t;
        if ((uint64_t)t + 2 * uu <= (uint64_t)(d - 1)) break;
    }
    uint64_t uu = ((2 * N) + (1ULL << t) - 1) >> t;
    // M/m = 2^k, k of the parity of t, nearest to log2(sqrt(2) N / log^3 N), ties to the
    // smaller k; m >= 2 and M >= m
    double target = 0.5 + lg - 3.0 * std::log2(lg);
    int best_k = -1;
    double best = 1e300;
    for (int k = t % 2; k <= t - 2; k += 2) {
        double dist = std::fabs(k - target);
        if (dist < best) {
            best = dist;
            best_k = k;
        }
    }
    if (best_k < 0) return false;
    *log2_m = (t - best_k) / 2;
    *log2_M = t - *log2_m;
    *u = (int)uu;
    *p_bits = d;
    return true;
}

bool candidate_params(uint64_t N, int c, int* log2_M, int* log2_m, int* u, int* p_bits, int* z) {
    if (N == 0 || N > (1ULL << 40) || c < 0 || c >= kNumCandidates) return false;
    auto need_bits = [&](int t) -> uint64_t {       // bits of p: p - 1 >= Mm 2^(2u)
        const uint64_t uu = ((2 * N) + (1ULL << t) - 1) >> t;
        return (uint64_t)t + 2 * uu + 1;
    };
    int t = 2;
    while (t <= 62 && need_bits(t) > 256) ++t;
    if (t > 62) return false;
    const bool squared = c >= kNumCandidatesZ1;
    if (!squared) t += c / 6;
    const int lm = (squared ? c - kNumCandidatesZ1 : c) % 6 + 1;
    if (lm > t - lm) return false;                   // M >= m
    const uint64_t uu = ((2 * N) + (1ULL << t) - 1) >> t;
    uint64_t pb;
    if (!squared) {
        // the fewest whole limbs, or where the modulus can be one 28-bit digit shorter than those
        // limbs need (2p < 2^(28 D)), the largest prime of that many digits
        const uint64_t nb = need_bits(t), limbs = (nb + 31) / 32;
        const uint64_t digits = (nb + 1 + 27) / 28;
        pb = (limbs >= 2 && digits < (32 * limbs + 28) / 28) ? 28 * digits - 1 : 32 * limbs;
    } else {
        // q = p^2 with p of b bits: p^2 >= 2^(2b - 2), so 2b - 2 >= t + 2u gives q > Mm 2^(2u)
        pb = ((uint64_t)t + 2 * uu + 3) / 2;
        if (2 * pb > 256) return false;
    }
    if (pb > 256) return false;
    *log2_m = lm;
    *log2_M = t - lm;
    *u = (int)uu;
    *p_bits = (int)pb;
    *z = squared ? 2 : 1;
    return true;
}

// ---------------------------------------------------------------------------------------------
// Prime p (Sec. 3.2.2, Sec. 4.6) and generator (Sec. 3.2.3)
// ---------------------------------------------------------------------------------------------

// Proth's theorem for p = h 2^n + 1, h < 2^n: p is prime iff a^((p-1)/2) = -1 for some a; a
// value other than +-1 proves p composite.  Small p with h >= 2^n: trial division.
static bool is_prime_hn(uint64_t h, int n, const Big& p) {
    if (n < 64 && (h >> n) != 0) {
        if (p.bitlen() > 44) return false;
        uint64_t v = p.w[0];
        if (v < 2) return false;
        for (uint64_t d = 2; d * d <= v; ++d)
            if (v % d == 0) return false;
        return true;
    }
    ModQ mq(p);
    Big pm1 = p.sub(Big::of(1));
    Big e = pm1.shr(1);
    for (uint64_t a = 2; a < 200; ++a) {
        Big x = mq.pow(Big::of(a), e);
        if (x == pm1) return true;
        if (x != Big::of(1)) return false;
    }
    return false;
}

bool proth_prime(int bits, int min_n, Big* p, uint64_t* h, int* n) {
    static std::mutex mu;
    static std::map<std::pair<int, int>, std::pair<uint64_t, int>> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find({bits, min_n});
    if (it != cache.end()) {
        *h = it->second.first;
        *n = it->second.second;
        *p = Big::of(*h).shl(*n).add(Big::of(1));
        return true;
    }
    for (uint64_t hh = 1; hh < (1ULL << 40); hh += 2) {
        int hb = 64 - __builtin_clzll(hh);
        int nn = bits - hb;
        if (nn < min_n || nn < 1) return false;
        Big cand = Big::of(hh).shl(nn).add(Big::of(1));
        if (is_prime_hn(hh, nn, cand)) {
            cache[{bits, min_n}] = {hh, nn};
            *p = cand;
            *h = hh;
            *n = nn;
            return true;
        }
    }
    return false;
}

static uint64_t smallest_generator(const Big& p, uint64_t h) {
    std::vector<uint64_t> primes = {2};
    uint64_t x = h;
    for (uint64_t d = 3; d * d <= x; d += 2) {
        if (x % d == 0) {
            primes.push_back(d);
            while (x % d == 0) x /= d;
        }
    }
    if (x > 1) primes.push_back(x);
    ModQ mq(p);
    Big pm1 = p.sub(Big::of(1));
    for (uint64_t g = 2;; ++g) {
        bool ok = true;
        for (uint64_t r : primes) {
            // (p-1)/r: p-1 = h 2^n; divide by r exactly
            Big e;
            if (r == 2) {
                e = pm1.shr(1);
            } else {
                // long division of pm1 by the small r
                unsigned __int128 rem = 0;
                for (int i = Big::kWords - 1; i >= 0; --i) {
                    unsigned __int128 cur = (rem << 64) | pm1.w[i];
                    e.w[i] = (uint64_t)(cur / r);
                    rem = cur % r;
                }
            }
            if (mq.pow(Big::of(g), e) == Big::of(1)) {
                ok = false;
                break;
            }
        }
        if (ok) return g;
    }
}

// ---------------------------------------------------------------------------------------------
// Constants (Sec. 3.2.3): zeta_z, omega, rho
// ---------------------------------------------------------------------------------------------

bool compute_constants(Plan* P) {
    int two_M_log = P->log2_M + 1;
    if (P->log2_m < 1 || P->log2_M < P->log2_m || P->u < 1 || P->z < 1) return false;
    if (!proth_prime(P->p_bits, two_M_log, &P->p, &P->h, &P->n)) return false;
    // q = p^z
    Big q = Big::of(1);
    for (int i = 0; i < P->z; ++i) {
        q = q.mul(P->p);
        if (q.bitlen() > 512) return false;
    }
    P->q = q;
    P->q_bits = q.bitlen();
    P->L = (P->q_bits + 31) / 32;
    // p^z >= Mm 2^(2u) (Sec. 3.2 Step 2)
    int need = P->log2_M + P->log2_m + 2 * P->u;
    if (need >= 1000) return false;
    if (q.bitlen() <= need) return false;   // q < 2^need (q is odd, never a power of two)
    ModQ mq(q);
    P->zeta = smallest_generator(P->p, P->h);
    // the (p-1)-th root of unity mod p^z above zeta: zeta^(p^(z-1)) (unique lift of zeta)
    Big pz1 = Big::of(1);
    for (int i = 0; i + 1 < P->z; ++i) pz1 = pz1.mul(P->p);
    Big zeta_z = mq.pow(Big::of(P->zeta), pz1);
    // omega = zeta_z^((p-1)/2M)
    Big hh = P->p.sub(Big::of(1)).shr(two_M_log);
    P->omega = mq.pow(zeta_z, hh);
    // gamma = omega^mu, a principal 2m-th root; rho_k = m^-1 sum_t omega^(2t+1) gamma^(-(2t+1)k),
    // the polynomial whose values at gamma^(2t+1) are omega^(2t+1)
    int m = P->m();
    Big gamma = mq.pow(P->omega, Big::of((uint64_t)P->mu_top()));
    Big ginv = mq.pow(gamma, Big::of((uint64_t)(2 * m - 1)));
    Big minv = mq.reduce(Big::of(1));
    for (int i = 0; i < P->log2_m; ++i) minv = mq.half(minv);
    std::vector<Big> cur(m), step(m);
    Big om_odd = P->omega;                        // omega^(2t+1)
    Big om2 = mq.mul(P->omega, P->omega);
    Big g_odd = ginv;                             // gamma^-(2t+1)
    Big ginv2 = mq.mul(ginv, ginv);
    for (int t = 0; t < m; ++t) {
        cur[t] = om_odd;
        step[t] = g_odd;
        om_odd = mq.mul(om_odd, om2);
        g_odd = mq.mul(g_odd, ginv2);
    }
    P->rho.assign(m, Big());
    for (int k = 0; k < m; ++k) {
        Big s;
        for (int t = 0; t < m; ++t) {
            s = mq.add(s, cur[t]);
            cur[t] = mq.mul(cur[t], step[t]);
        }
        P->rho[k] = mq.mul(s, minv);
    }
    return true;
}

std::string Plan::key() const {
    char buf[96];
    snprintf(buf, sizeof buf, "M%d_m%d_p%d_z%d", log2_M, log2_m, p_bits, z);
    return buf;
}

int max_radix_log2(int log2_m, int L) {
    // one column of 2^t elements of m residues of L limbs, staged twice in LDS (ping-pong
    // buffers within kLdsBytes), and at most 1024 butterfly tasks (2^(t-1) pairs x m
    // coefficients) per radix-2 pass
    int t = log2_m + 1;
    while (t > 1 && ((2 * (4LL * L) << (t + log2_m)) > kLdsBytes || ((1LL << (t - 1 + log2_m)) > 1024)))
        --t;
    return t;
}

std::vector<int> default_radices(int log2_M, int log2_m, int L) {
    std::vector<int> r;
    int rem = log2_M + 1;
    int cap = max_radix_log2(log2_m, L);
    while (rem > cap) {
        r.push_back(cap);
        rem -= cap;
    }
    if (rem > 0) r.push_back(rem);
    return r;
}

}  // namespace dkss
