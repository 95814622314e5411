// Exact-integer layer: Smith normal form, canonical orders, transform plans.
//
// Sec. 2.2: M = Q E R with unimodular Q, R (determinant +-1 when det M < 0)
// and e_j | e_{j+1}.  Points y(lambda) = R^{-1} E^{-1} lambda (mod 1) and
// frequencies h(kappa) = M^T rep(Q^{-T} E^{-1} kappa) make the pattern DFT the
// ordinary DFT over Z_{e_1} x ... x Z_{e_d}: h(kappa)^T y(lambda) =
// sum_j kappa_j lambda_j / e_j (mod 1).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "ahom_internal.h"
#include "../../include/ahom.h"

namespace {

struct Overflow {};

inline int64_t ck_add(int64_t a, int64_t b) {
    int64_t r;
    if (__builtin_add_overflow(a, b, &r)) throw Overflow();
    return r;
}
inline int64_t ck_mul(int64_t a, int64_t b) {
    int64_t r;
    if (__builtin_mul_overflow(a, b, &r)) throw Overflow();
    return r;
}

int64_t det_exact(int d, const int64_t a[3][3]) {
    if (d == 2) return ck_add(ck_mul(a[0][0], a[1][1]), -ck_mul(a[0][1], a[1][0]));
    int64_t t0 = ck_add(ck_mul(a[1][1], a[2][2]), -ck_mul(a[1][2], a[2][1]));
    int64_t t1 = ck_add(ck_mul(a[1][0], a[2][2]), -ck_mul(a[1][2], a[2][0]));
    int64_t t2 = ck_add(ck_mul(a[1][0], a[2][1]), -ck_mul(a[1][1], a[2][0]));
    return ck_add(ck_add(ck_mul(a[0][0], t0), -ck_mul(a[0][1], t1)), ck_mul(a[0][2], t2));
}

// inverse of a unimodular matrix: adj(U) * det(U)
void unimodular_inverse(int d, const int64_t U[3][3], int64_t out[3][3]) {
    int64_t D = det_exact(d, U);
    if (D != 1 && D != -1) throw Overflow();
    if (d == 2) {
        out[0][0] = D * U[1][1];  out[0][1] = -D * U[0][1];
        out[1][0] = -D * U[1][0]; out[1][1] = D * U[0][0];
        return;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            // cofactor C_ji
            int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
            int64_t cof = ck_add(ck_mul(U[r0][c0], U[r1][c1]), -ck_mul(U[r0][c1], U[r1][c0]));
            out[i][j] = ck_mul(D, cof);
        }
}

void matmul3(int d, const int64_t A[3][3], const int64_t B[3][3], int64_t C[3][3]) {
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            int64_t s = 0;
            for (int k = 0; k < d; ++k) s = ck_add(s, ck_mul(A[i][k], B[k][j]));
            C[i][j] = s;
        }
}

bool seven_smooth(int64_t v) {
    for (int p : {2, 3, 5, 7})
        while (v % p == 0) v /= p;
    return v == 1;
}

inline int64_t floordiv(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

inline int64_t pmod(int64_t a, int64_t m) {
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

}  // namespace

// Smith normal form by elimination: row operations U and column operations V
// with U M V = diag(e); Q = U^{-1}, R = V^{-1}.
int ahom_smith_form(int d, const int64_t* Min, SmithForm* out, std::string* err) {
    if (d != 2 && d != 3) { *err = "d must be 2 or 3"; return AHOM_E_ARG; }
    try {
        SmithForm sf{};
        sf.d = d;
        int64_t A[3][3] = {}, U[3][3] = {}, V[3][3] = {};
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) { A[i][j] = Min[i * d + j]; sf.M[i][j] = A[i][j]; }
        for (int i = 0; i < d; ++i) { U[i][i] = 1; V[i][i] = 1; }
        int64_t D = det_exact(d, A);
        if (D == 0) { *err = "singular pattern matrix (det M = 0)"; return AHOM_E_SINGULAR; }
        int64_t m = D < 0 ? -D : D;
        if (m > (int64_t(1) << 31)) { *err = "|det M| exceeds 2^31"; return AHOM_E_OVERFLOW; }

        auto swap_rows = [&](int a, int b) { for (int j = 0; j < d; ++j) { std::swap(A[a][j], A[b][j]); std::swap(U[a][j], U[b][j]); } };
        auto swap_cols = [&](int a, int b) { for (int i = 0; i < d; ++i) { std::swap(A[i][a], A[i][b]); std::swap(V[i][a], V[i][b]); } };
        for (int t = 0; t < d; ++t) {
            for (int guard = 0;; ++guard) {
                if (guard > 10000) throw Overflow();
                int bi = -1, bj = -1;
                for (int i = t; i < d; ++i)
                    for (int j = t; j < d; ++j)
                        if (A[i][j] != 0 && (bi < 0 || std::llabs(A[i][j]) < std::llabs(A[bi][bj]))) { bi = i; bj = j; }
                if (bi != t) swap_rows(t, bi);
                if (bj != t) swap_cols(t, bj);
                bool clean = true;
                for (int i = t + 1; i < d; ++i) {
                    int64_t q = floordiv(A[i][t], A[t][t]);
                    if (q) for (int j = 0; j < d; ++j) {
                        A[i][j] = ck_add(A[i][j], -ck_mul(q, A[t][j]));
                        U[i][j] = ck_add(U[i][j], -ck_mul(q, U[t][j]));
                    }
                    if (A[i][t] != 0) clean = false;
                }
                for (int j = t + 1; j < d; ++j) {
                    int64_t q = floordiv(A[t][j], A[t][t]);
                    if (q) for (int i = 0; i < d; ++i) {
                        A[i][j] = ck_add(A[i][j], -ck_mul(q, A[i][t]));
                        V[i][j] = ck_add(V[i][j], -ck_mul(q, V[i][t]));
                    }
                    if (A[t][j] != 0) clean = false;
                }
                if (!clean) continue;
                int bad = -1;
                for (int i = t + 1; i < d && bad < 0; ++i)
                    for (int j = t + 1; j < d; ++j)
                        if (A[i][j] % A[t][t] != 0) { bad = i; break; }
                if (bad < 0) break;
                for (int j = 0; j < d; ++j) {
                    A[t][j] = ck_add(A[t][j], A[bad][j]);
                    U[t][j] = ck_add(U[t][j], U[bad][j]);
                }
            }
            if (A[t][t] < 0)
                for (int j = 0; j < d; ++j) { A[t][j] = -A[t][j]; U[t][j] = -U[t][j]; }
        }
        for (int t = 0; t < d; ++t) sf.e[t] = A[t][t];
        unimodular_inverse(d, U, sf.Q);
        unimodular_inverse(d, V, sf.R);
        std::memcpy(sf.Rinv, V, sizeof(V));
        std::memcpy(sf.Qinv, U, sizeof(U));
        // verify Q E R = M exactly
        int64_t QE[3][3] = {}, QER[3][3] = {};
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) QE[i][j] = ck_mul(sf.Q[i][j], sf.e[j]);
        matmul3(d, QE, sf.R, QER);
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j)
                if (QER[i][j] != sf.M[i][j]) { *err = "internal: Smith form check failed"; return AHOM_E_OVERFLOW; }
        sf.m = m;
        sf.dM = 0;
        for (int t = 0; t < d; ++t) {
            if (sf.e[t] > 1) ++sf.dM;
            if (!seven_smooth(sf.e[t])) {
                *err = "elementary divisor " + std::to_string(sf.e[t]) + " has a prime factor above 7";
                return AHOM_E_UNSUPPORTED_SIZE;
            }
        }
        *out = sf;
        return AHOM_OK;
    } catch (Overflow&) {
        *err = "int64 overflow in the Smith normal form";
        return AHOM_E_OVERFLOW;
    }
}

// Canonical point order: lambda lexicographic over the axes with e_s > 1;
// numerators p = m R^{-1} E^{-1} lambda centred modulo m.
void ahom_canonical_points(const SmithForm& sf, int64_t* num) {
    const int d = sf.d;
    int64_t lam[3] = {0, 0, 0};
    const int64_t m = sf.m;
    for (int64_t idx = 0; idx < m; ++idx) {
        int64_t r = idx;
        for (int s = d - 1; s >= 0; --s) { lam[s] = r % sf.e[s]; r /= sf.e[s]; }
        for (int i = 0; i < d; ++i) {
            __int128 acc = 0;
            for (int s = 0; s < d; ++s) acc += (__int128)sf.Rinv[i][s] * (__int128)((m / sf.e[s]) * lam[s]);
            int64_t v = (int64_t)(acc % m);
            if (v < 0) v += m;
            if (2 * v >= m) v -= m;
            num[idx * d + i] = v;
        }
    }
}

int ahom_plan_set_cell(Plan* plan, int d, const double* L, std::string* err) {
    double a[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    double scale = 0.0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            a[i][j] = L[i * d + j];
            if (!std::isfinite(a[i][j])) {
                *err = "L has a non-finite entry";
                return AHOM_E_ARG;
            }
            scale = std::max(scale, std::fabs(a[i][j]));
        }
    // L^{-1} by cofactors; a determinant that vanishes next to the entries'
    // size is a singular cell
    const double det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                       a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
    if (!(std::fabs(det) > 1e-12 * std::pow(scale, d))) {
        *err = "L is singular";
        return AHOM_E_SINGULAR;
    }
    double inv[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int j1 = (j + 1) % 3, j2 = (j + 2) % 3, i1 = (i + 1) % 3, i2 = (i + 2) % 3;
            inv[i][j] = (a[j1][i1] * a[j2][i2] - a[j1][i2] * a[j2][i1]) / det;
        }
    // G = L^{-T} M^T: (L^{-T})_{ij} = (L^{-1})_{ji}
    FreqMap& fm = plan->fm;
    for (int i = 0; i < d; ++i)
        for (int s = 0; s < d; ++s) {
            double g = 0.0;
            for (int j = 0; j < d; ++j) g += inv[j][i] * (double)fm.MT[j][s];
            fm.G[i][s] = g;
        }
    return AHOM_OK;
}

// Canonical frequency order: kappa lexicographic; h = M^T N / emax.
void ahom_canonical_freqs(const SmithForm& sf, const FreqMap& fm, int64_t* h) {
    const int d = sf.d;
    int64_t kap[3] = {0, 0, 0}, N[3];
    for (int64_t idx = 0; idx < sf.m; ++idx) {
        int64_t r = idx;
        for (int s = d - 1; s >= 0; --s) { kap[s] = r % sf.e[s]; r /= sf.e[s]; }
        ahom_centred_numerators(fm, kap, N);
        for (int i = 0; i < d; ++i) {
            __int128 acc = 0;
            for (int j = 0; j < d; ++j) acc += (__int128)fm.MT[i][j] * N[j];
            h[idx * d + i] = (int64_t)(acc / fm.emax);
        }
    }
}

namespace {

std::vector<int> radix_plan(int L, int max_radix) {
    std::vector<int> r;
    int v = L;
    if (max_radix >= 8)
        while (v % 8 == 0) { r.push_back(8); v /= 8; }
    while (v % 4 == 0) { r.push_back(4); v /= 4; }
    if (v % 2 == 0) { r.push_back(2); v /= 2; }
    for (int p : {3, 5, 7})
        while (v % p == 0) { r.push_back(p); v /= p; }
    return r;  // v == 1 for 7-smooth L
}

// balanced factorization of L into k factors, each <= lmax (slowest first)
bool factorize(int64_t L, int k, int64_t lmax, std::vector<int64_t>* out) {
    if (k == 1) {
        if (L <= lmax) { out->push_back(L); return true; }
        return false;
    }
    std::vector<int64_t> divs;
    for (int64_t f = 1; f * f <= L; ++f)
        if (L % f == 0) { divs.push_back(f); divs.push_back(L / f); }
    double target = std::pow((double)L, 1.0 / k);
    std::sort(divs.begin(), divs.end(), [&](int64_t a, int64_t b) {
        double da = std::fabs(std::log((double)a) - std::log(target));
        double db = std::fabs(std::log((double)b) - std::log(target));
        return da < db || (da == db && a < b);
    });
    for (int64_t f : divs) {
        if (f > lmax) continue;
        std::vector<int64_t> rest;
        if (factorize(L / f, k - 1, lmax, &rest)) {
            out->push_back(f);
            out->insert(out->end(), rest.begin(), rest.end());
            return true;
        }
    }
    return false;
}

}  // namespace

int ahom_build_plan(const SmithForm& sf, int lmax, Plan* plan, std::string* err) {
    return ahom_build_plan_ex(sf, lmax, 8, plan, err);
}

int ahom_build_plan_ex(const SmithForm& sf, int lmax, int max_radix, Plan* plan, std::string* err) {
    Plan p{};
    p.d = sf.d;
    p.m = sf.m;
    // frequency map
    FreqMap& fm = p.fm;
    fm.d = sf.d;
    fm.emax = 1;
    for (int s = 0; s < sf.d; ++s) { fm.e[s] = sf.e[s]; fm.emax = std::max(fm.emax, sf.e[s]); }
    for (int s = sf.d; s < 3; ++s) fm.e[s] = 1;
    for (int i = 0; i < sf.d; ++i)
        for (int s = 0; s < sf.d; ++s) {
            // (Q^{-T})_{is} = (Q^{-1})_{si}
            __int128 v = (__int128)sf.Qinv[s][i] * (fm.emax / sf.e[s]);
            int64_t r = (int64_t)(v % fm.emax);
            if (r < 0) r += fm.emax;
            fm.A[i][s] = r;
            fm.MT[i][s] = sf.M[s][i];
            fm.G[i][s] = (double)sf.M[s][i];
        }
    // canonical strides
    int64_t stride = 1;
    for (int s = sf.d - 1; s >= 0; --s) {
        p.canon_stride[s] = sf.e[s] > 1 ? stride : 0;
        stride *= sf.e[s];
    }
    // kernel axes
    std::vector<int> smith_axes;
    for (int s = 0; s < sf.d; ++s)
        if (sf.e[s] > 1) smith_axes.push_back(s);
    int D = 0;
    if (smith_axes.empty()) {
        *err = "trivial pattern (m = 1)";
        return AHOM_E_ARG;
    }
    for (int s : smith_axes) {
        int64_t L = sf.e[s];
        int k = 1;
        while (true) {
            int64_t cap = 1;
            for (int t = 0; t < k; ++t) cap = std::min<int64_t>(cap * lmax, int64_t(1) << 40);
            if (cap >= L) break;
            ++k;
        }
        if (smith_axes.size() == 1) k = std::max(k, 2);
        std::vector<int64_t> f;
        while (!factorize(L, k, lmax, &f)) { f.clear(); ++k; if (k > 6) { *err = "cannot factor axis"; return AHOM_E_UNSUPPORTED_SIZE; } }
        int64_t mult = 1;
        for (size_t t = 0; t < f.size(); ++t) {
            if (D >= AHOM_MAX_AXES) { *err = "too many kernel axes"; return AHOM_E_UNSUPPORTED_SIZE; }
            AxisDesc& a = p.ax[D++];
            a.len = (int)f[t];
            a.snf = s;
            a.mult = mult;
            mult *= f[t];
            int64_t tail = 1;
            for (size_t u = t; u < f.size(); ++u) tail *= f[u];
            a.tailN = tail;
            a.split = (t + 1 < f.size()) ? 1 : 0;
            std::vector<int> r = radix_plan(a.len, max_radix);
            a.nstage = (int)r.size();
            for (size_t u = 0; u < r.size(); ++u) a.radix[u] = r[u];
        }
    }
    p.D = D;
    // stored lengths (half spectrum along axis 0)
    for (int a = 0; a < D; ++a) p.ax[a].slen = p.ax[a].len;
    p.ax[0].slen = p.ax[0].len / 2 + 1;
    p.S = 1;
    for (int a = 0; a < D; ++a) p.S *= p.ax[a].slen;
    // q divisor for split twiddles: product of stored lengths after the group
    for (int a = 0; a < D; ++a) {
        int64_t after = 1;
        int b = a + 1;
        while (b < D && p.ax[b].snf == p.ax[a].snf) ++b;
        for (int c = b; c < D; ++c) after *= p.ax[c].slen;
        p.ax[a].qdiv = after;
    }
    *plan = p;
    return AHOM_OK;
}

// W_L^k = exp(-2 pi i k / L), computed in long double and rounded.
static void push_roots(std::vector<double>* tw, int64_t N, int64_t count, int64_t step) {
    const long double twopi = 6.283185307179586476925286766559005768L;
    for (int64_t k = 0; k < count; ++k) {
        int64_t j = (k * step) % N;
        long double ang = -twopi * (long double)j / (long double)N;
        tw->push_back((double)cosl(ang));
        tw->push_back((double)sinl(ang));
    }
}

void ahom_build_twiddles(Plan* plan, std::vector<double>* tw) {
    tw->clear();
    for (int a = 0; a < plan->D; ++a) {
        AxisDesc& ax = plan->ax[a];
        int found = -1;
        for (int b = 0; b < a; ++b)
            if (plan->ax[b].len == ax.len) found = b;
        if (found >= 0) {
            ax.tw_off = plan->ax[found].tw_off;
        } else {
            ax.tw_off = (int)(tw->size() / 2);
            push_roots(tw, ax.len, ax.len, 1);
        }
        if (ax.split) {
            int64_t N = ax.tailN;
            int64_t B = (int64_t)std::ceil(std::sqrt((double)N));
            ax.spB = B;
            ax.sp_off1 = (int)(tw->size() / 2);
            push_roots(tw, N, B, 1);
            ax.sp_off2 = (int)(tw->size() / 2);
            push_roots(tw, N, (N + B - 1) / B, B);
        }
    }
}
