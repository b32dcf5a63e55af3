// Host build of the library's device arithmetic (kernels.hpp is __host__ __device__), so that
// CPU tests can compare it with Python integers.  Not part of the library.
#include <cstdint>
#include <cstring>

#include "../../paper_1503_04955_amd/csrc/kernels.hpp"

using namespace dkss;

namespace {

// e >= 1 when q = 1 + qd[e] 2^(28e) + qd[e+1] 2^(28(e+1)) (the library's rule for its sparse
// Montgomery steps), else 0
int sparse_e(int D, const uint32_t* qd) {
    if (qd[0] != 1) return 0;
    int e = 1;
    while (e < D && qd[e] == 0) ++e;
    if (e >= D) return 0;
    for (int k = e + 2; k < D; ++k)
        if (qd[k] != 0) return 0;
    return e;
}

template <int L>
void run(int op, const uint32_t* qd, uint32_t qinv, const uint32_t* a, const uint32_t* b, int log2m,
         int j, int r, uint32_t* out) {
    QConst Q;
    memset(&Q, 0, sizeof Q);
    memcpy(Q.qd, qd, sizeof(uint32_t) * Dig<L>::D);
    digits_to_limbs<L>(qd, Q.ql);
    Q.qinv28 = qinv;
    Q.se = sparse_e(Dig<L>::D, qd);
    switch (op) {
        case 0: dmod_add<L>(out, a, b, Q); break;
        case 1: dmod_sub<L>(out, a, b, Q); break;
        case 2: dneg_q<L>(out, a, Q); break;
        case 3: case 9: {
            // a: T_0..T_(2m-1) at DS words; staged for t alpha^r as the kernels stage it
            constexpr int DS = Dig<L>::DS;
            const int m2 = 2 << log2m;
            uint32_t tp[2 * 64 * DS];
            for (int i = 0; i < m2; ++i)
                memcpy(tp + stage_pos(i, r, log2m) * DS, a + i * DS, sizeof(uint32_t) * DS);
            if (op == 3) rprod_coeff<L>(tp, b, log2m, j, Q, out);
            else rprod_coeff<L, true>(tp, b, log2m, j, Q, out);      // out in limbs
            break;
        }
        case 4: mont_scalar<L>(a, b, Q, out); break;
        case 5: digits_to_limbs<L>(a, out); break;
        case 6: lmod_add<L>(out, a, b, Q.ql); break;   // a, b, out in limbs
        case 7: lmod_sub<L>(out, a, b, Q.ql); break;
        case 8: limbs_to_digits<L>(a, out); break;
        default: break;
    }
}

}  // namespace

extern "C" {

int da_D(int L) {
    switch (L) {
        case 1: return Dig<1>::D; case 2: return Dig<2>::D; case 3: return Dig<3>::D; case 4: return Dig<4>::D;
        case 5: return Dig<5>::D; case 6: return Dig<6>::D; case 7: return Dig<7>::D; case 8: return Dig<8>::D;
    }
    return -1;
}

int da_DS(int L) {
    switch (L) {
        case 1: return Dig<1>::DS; case 2: return Dig<2>::DS; case 3: return Dig<3>::DS; case 4: return Dig<4>::DS;
        case 5: return Dig<5>::DS; case 6: return Dig<6>::DS; case 7: return Dig<7>::DS; case 8: return Dig<8>::DS;
    }
    return -1;
}

// the LDS layout of the products in R (words per staged operand and per element in digits,
// staging position of operand entry i for a product by t alpha^r)
int da_stage_words(int m, int L) { return stage_words(m, (32 * L + 28) / 28 | 1); }
int da_elem_words(int m, int L) { return elem_words(m, (32 * L + 28) / 28); }
int da_stage_pos(int i, int r, int log2m) { return stage_pos(i, r, log2m); }

// 1 when the Montgomery reduction for modulus digits qd takes its sparse steps
int da_sparse(int L, const uint32_t* qd) {
    switch (L) {
        case 1: return sparse_e(Dig<1>::D, qd) == (32 * 1 - 1) / 28;
        case 2: return sparse_e(Dig<2>::D, qd) == (32 * 2 - 1) / 28;
        case 3: return sparse_e(Dig<3>::D, qd) == (32 * 3 - 1) / 28;
        case 4: return sparse_e(Dig<4>::D, qd) == (32 * 4 - 1) / 28;
        case 5: return sparse_e(Dig<5>::D, qd) == (32 * 5 - 1) / 28;
        case 6: return sparse_e(Dig<6>::D, qd) == (32 * 6 - 1) / 28;
        case 7: return sparse_e(Dig<7>::D, qd) == (32 * 7 - 1) / 28;
        case 8: return sparse_e(Dig<8>::D, qd) == (32 * 8 - 1) / 28;
    }
    return 0;
}

int da_K(int L) {
    switch (L) {
        case 1: return Dig<1>::K; case 2: return Dig<2>::K; case 3: return Dig<3>::K; case 4: return Dig<4>::K;
        case 5: return Dig<5>::K; case 6: return Dig<6>::K; case 7: return Dig<7>::K; case 8: return Dig<8>::K;
    }
    return -1;
}

void da_run(int L, int op, const uint32_t* qd, uint32_t qinv, const uint32_t* a, const uint32_t* b,
            int log2m, int j, int r, uint32_t* out) {
    switch (L) {
        case 1: run<1>(op, qd, qinv, a, b, log2m, j, r, out); break;
        case 2: run<2>(op, qd, qinv, a, b, log2m, j, r, out); break;
        case 3: run<3>(op, qd, qinv, a, b, log2m, j, r, out); break;
        case 4: run<4>(op, qd, qinv, a, b, log2m, j, r, out); break;
        case 5: run<5>(op, qd, qinv, a, b, log2m, j, r, out); break;
        case 6: run<6>(op, qd, qinv, a, b, log2m, j, r, out); break;
        case 7: run<7>(op, qd, qinv, a, b, log2m, j, r, out); break;
        case 8: run<8>(op, qd, qinv, a, b, log2m, j, r, out); break;
    }
}

}  // extern "C"
