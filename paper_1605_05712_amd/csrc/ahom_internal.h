// Internal definitions shared by the host library and the HIP kernels.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#define AHOM_MAX_AXES 8
#define AHOM_MAX_STAGES 16
#define AHOM_WG 256

// One kernel axis of the Smith-form array after long axes have been split.
// A split Smith axis of length N = L_0 L_1 ... (slowest sub-axis first) is the
// four-step factorization: index n = n_last + L_last (... ), the forward
// transform runs the sub-axes slowest first, multiplying after each sub-axis
// by W_N'^{q k} with N' the product of this and the later sub-axis lengths
// and q the position along the later sub-axes.  The frequency along the Smith
// axis is kappa = sum_a mult_a k_a with mult_a the product of the earlier
// sub-axis lengths.
struct AxisDesc {
    int len;                        // transform length L
    int slen;                       // stored length (axis 0 of the half spectrum: L/2 + 1)
    int snf;                        // Smith axis this sub-axis belongs to
    int nstage;
    int radix[AHOM_MAX_STAGES];
    int tw_off;                     // offset of the table W_L^k (k < L) in the twiddle buffers
    int split;                      // 1: apply the four-step twiddle in this axis' pass
    int64_t mult;                   // kappa multiplier
    int64_t tailN;                  // N' for the four-step twiddle
    int64_t qdiv;                   // q = inner_index / qdiv
    int64_t spB;                    // two-level table split: W^j = T1[j % B] * T2[j / B]
    int sp_off1, sp_off2;           // offsets of T1, T2 in the FP64 twiddle buffer
};

// Integer data that maps a frequency position to h(kappa) (Sec. 2.2):
// N = centred(A kappa mod emax), h = M^T N / emax.
struct FreqMap {
    int d;
    int64_t emax;
    int64_t A[3][3];                // A[i][s] = (Q^{-T})_{is} (emax / e_s) mod emax
    int64_t MT[3][3];               // M^T
    int64_t e[3];                   // elementary divisors
    // Direction map of Gamma0 and of the residual: xi is parallel to G N.
    // G = M^T (exact integers) on P(M); G = L^{-T} M^T on the transformed
    // pattern P_L(M) of Def. 3.3, whose frequencies are L^{-T} h.
    double G[3][3];
};

struct Plan {
    int d;                          // 2 or 3
    int D;                          // number of kernel axes (>= 2)
    int64_t m;                      // |det M|
    int64_t S;                      // stored complex elements per field (half spectrum)
    AxisDesc ax[AHOM_MAX_AXES];
    FreqMap fm;
    int64_t canon_stride[3];        // canonical kappa-lex stride of Smith axis s (0 if e_s = 1)
};

// Exact frequency of a Smith-form index kappa (host and device).
// Writes the centred numerators N[0..d-1] with N/emax = rep(Q^{-T} E^{-1} kappa)
// and returns 1 if some coordinate equals -1/2 (possible boundary class).
#if defined(__HIPCC__)
#define AHOM_HD __host__ __device__
#else
#define AHOM_HD
#endif

AHOM_HD inline int ahom_centred_numerators(const FreqMap& f, const int64_t* kappa, int64_t* N) {
    int half = 0;
    for (int i = 0; i < f.d; ++i) {
        int64_t acc = 0;
        for (int s = 0; s < f.d; ++s) {
            acc += f.A[i][s] * kappa[s];
            acc %= f.emax;
        }
        if (2 * acc >= f.emax) acc -= f.emax;
        if (2 * acc == -f.emax) half = 1;
        N[i] = acc;
    }
    return half;
}

AHOM_HD inline int ahom_self_conjugate(const FreqMap& f, const int64_t* kappa) {
    for (int s = 0; s < f.d; ++s)
        if ((2 * kappa[s]) % f.e[s] != 0) return 0;
    return 1;
}

// ---------------------------------------------------------------- host side
struct SmithForm {
    int d;
    int64_t M[3][3], Q[3][3], R[3][3], Rinv[3][3], Qinv[3][3];
    int64_t e[3];
    int64_t m;
    int dM;
};

int ahom_smith_form(int d, const int64_t* M, SmithForm* out, std::string* err);
int ahom_build_plan(const SmithForm& sf, int lmax, Plan* plan, std::string* err);
// max_radix 8: radix-8 stages first; 4: radix 4 and 2 only for the powers of two
int ahom_build_plan_ex(const SmithForm& sf, int lmax, int max_radix, Plan* plan, std::string* err);
// Transformed pattern P_L(M) (Def. 3.3): sets the plan's direction map
// G = L^{-T} M^T for the real regular cell matrix L (d*d, row-major).
// AHOM_E_ARG for a non-finite entry, AHOM_E_SINGULAR for |det L| <= 1e-12 max|L_ij|^d.
int ahom_plan_set_cell(Plan* plan, int d, const double* L, std::string* err);
// Twiddle tables for a plan: FP64 values (and their FP32 rounding).
void ahom_build_twiddles(Plan* plan, std::vector<double>* tw64);
void ahom_canonical_points(const SmithForm& sf, int64_t* num);
void ahom_canonical_freqs(const SmithForm& sf, const FreqMap& fm, int64_t* h);
void ahom_set_error(const std::string& msg);
