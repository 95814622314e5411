// HIP kernels (gfx950) for one iteration of the generalized Basic Scheme.
//
// Field storage (per load case, per strain component): the half spectrum
// along kernel axis 0 (stored length L0/2 + 1), full length along the other
// kernel axes, row-major, interleaved complex.  One iteration (Algorithm 1,
// Sec. 3.2) is a chain of passes over HBM:
//   k_real   axis 0 : inverse C2R, local law tau = (C - C0) : eps, forward R2C
//   k_axis   axes 1..D-2 forward, then later inverse (plain complex FFTs)
//   k_spec   axis D-1 : forward FFT, Gamma0 at h(kappa) + residual terms,
//                       inverse FFT
//   k_reduce          : FP64 residual and mean stress, loop control
// Each 1-D transform is a mixed-radix Stockham FFT held in LDS.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "ahom_internal.h"
#include "ahom_kernels.h"

#define AHOM_CHECK_LAUNCH() (hipGetLastError() == hipSuccess ? 0 : -1)

namespace {

template <typename T> struct CT;
template <> struct CT<double> { using t = double2; };
template <> struct CT<float> { using t = float2; };

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) { return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) { return C{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }
// multiply by -i (forward, DIR = -1) or +i (inverse, DIR = +1)
template <int DIR, typename C> __device__ __forceinline__ C mul_i(C a) {
    return DIR < 0 ? C{a.y, -a.x} : C{-a.y, a.x};
}

// ---------------------------------------------------------------- butterflies
// y_k = sum_r v_r W_R^{r k}, W_R = exp(DIR 2 pi i / R)
template <int DIR, typename C> __device__ __forceinline__ void bfly2(C* v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <int DIR, typename C> __device__ __forceinline__ void bfly4(C* v) {
    C a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    C c = cadd(v[1], v[3]), d = mul_i<DIR>(csub(v[1], v[3]));
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
}

template <int DIR, typename C> __device__ __forceinline__ void bfly8(C* v) {
    using T = decltype(v[0].x);
    C e[4] = {v[0], v[2], v[4], v[6]};
    C o[4] = {v[1], v[3], v[5], v[7]};
    bfly4<DIR>(e);
    bfly4<DIR>(o);
    const T r = (T)0.70710678118654752440;
    // W8^1 o1, W8^2 o2, W8^3 o3
    C o1 = DIR < 0 ? C{r * (o[1].x + o[1].y), r * (o[1].y - o[1].x)} : C{r * (o[1].x - o[1].y), r * (o[1].y + o[1].x)};
    C o2 = mul_i<DIR>(o[2]);
    C o3 = DIR < 0 ? C{r * (o[3].y - o[3].x), -r * (o[3].x + o[3].y)} : C{-r * (o[3].x + o[3].y), r * (o[3].x - o[3].y)};
    v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);   v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);   v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);   v[7] = csub(e[3], o3);
}

// small odd radices: direct sum with cos/sin of 2 pi j / R
template <int R, int DIR, typename C> __device__ __forceinline__ void bfly_odd(C* v) {
    using T = decltype(v[0].x);
    constexpr double c3[3] = {1.0, -0.5, -0.5};
    constexpr double s3[3] = {0.0, 0.86602540378443864676, -0.86602540378443864676};
    constexpr double c5[5] = {1.0, 0.30901699437494742410, -0.80901699437494742410, -0.80901699437494742410, 0.30901699437494742410};
    constexpr double s5[5] = {0.0, 0.95105651629515357212, 0.58778525229247312917, -0.58778525229247312917, -0.95105651629515357212};
    constexpr double c7[7] = {1.0, 0.62348980185873353053, -0.22252093395631440429, -0.90096886790241912624,
                              -0.90096886790241912624, -0.22252093395631440429, 0.62348980185873353053};
    constexpr double s7[7] = {0.0, 0.78183148246802980871, 0.97492791218182360702, 0.43388373911755812048,
                              -0.43388373911755812048, -0.97492791218182360702, -0.78183148246802980871};
    const double* cs = R == 3 ? c3 : (R == 5 ? c5 : c7);
    const double* sn = R == 3 ? s3 : (R == 5 ? s5 : s7);
    C out[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        C acc = v[0];
#pragma unroll
        for (int r = 1; r < R; ++r) {
            const int j = (r * k) % R;
            const T c = (T)cs[j], s = (T)(DIR < 0 ? -sn[j] : sn[j]);
            acc.x += v[r].x * c - v[r].y * s;
            acc.y += v[r].x * s + v[r].y * c;
        }
        out[k] = acc;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = out[k];
}

// Division by a divisor that is fixed for a whole tile: floor(n / d) as one
// high-half product with m = floor((2^32 - 1) / d) + 1 = 2^32 / d + e,
// 0 <= e < 1.  Then n m / 2^32 = n / d + n e / 2^32, and the floor is exact
// when n d < 2^32 (the fraction of n / d is at most 1 - 1/d).  Used only for
// positions inside an LDS tile and divisors that are tile extents (both below
// 2^16, as a tile holds fewer than 2^16 elements); d = 1 wraps m to 0.
struct UDiv {
    uint32_t d, m;
    __device__ __forceinline__ explicit UDiv(int dd) : d((uint32_t)dd), m(0xFFFFFFFFu / (uint32_t)dd + 1u) {}
    __device__ __forceinline__ int div(int n) const { return m ? (int)__umulhi((uint32_t)n, m) : n; }
    __device__ __forceinline__ void divmod(int n, int& q, int& r) const {
        q = div(n);
        r = n - q * (int)d;
    }
};

// One radix-R Stockham stage over `total` butterflies of all columns.
template <int R, int DIR, typename C>
__device__ __forceinline__ void stage(const C* __restrict__ src, C* __restrict__ dst, int ncol, int L, int CS, int Ns,
                                      const C* __restrict__ tw) {
    const int nb = L / R;
    const int total = ncol * nb;
    const int tstep = L / (Ns * R);
    const UDiv by_nb(nb), by_ns(Ns);
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        int j, b, bq, k;
        by_nb.divmod(t, j, b);
        by_ns.divmod(b, bq, k);
        C v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = src[j * CS + b + r * nb];
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const C w = tw[k * r * tstep];
                v[r] = DIR < 0 ? cmul(v[r], w) : cmulc(v[r], w);
            }
        }
        if constexpr (R == 2) bfly2<DIR>(v);
        else if constexpr (R == 4) bfly4<DIR>(v);
        else if constexpr (R == 8) bfly8<DIR>(v);
        else bfly_odd<R, DIR>(v);
        const int o = bq * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[j * CS + o + r * Ns] = v[r];
    }
}

// In-LDS FFT of `ncol` columns of length L (column stride CS); result in buf.
template <int DIR, typename C>
__device__ void lds_fft(C* buf, C* tmp, int ncol, int CS, const AxisDesc& ax, const C* __restrict__ tw) {
    const int L = ax.len;
    C* src = buf;
    C* dst = tmp;
    int Ns = 1;
    for (int s = 0; s < ax.nstage; ++s) {
        const int R = ax.radix[s];
        switch (R) {
            case 8: stage<8, DIR>(src, dst, ncol, L, CS, Ns, tw); break;
            case 4: stage<4, DIR>(src, dst, ncol, L, CS, Ns, tw); break;
            case 2: stage<2, DIR>(src, dst, ncol, L, CS, Ns, tw); break;
            case 3: stage<3, DIR>(src, dst, ncol, L, CS, Ns, tw); break;
            case 5: stage<5, DIR>(src, dst, ncol, L, CS, Ns, tw); break;
            default: stage<7, DIR>(src, dst, ncol, L, CS, Ns, tw); break;
        }
        __syncthreads();
        C* t = src; src = dst; dst = t;
        Ns *= R;
    }
    if (src != buf) {
        const UDiv by_l(L);
        for (int e = threadIdx.x; e < ncol * L; e += blockDim.x) {
            int j, l;
            by_l.divmod(e, j, l);
            buf[j * CS + l] = src[j * CS + l];
        }
        __syncthreads();
    }
}

// Four-step twiddle W_N^{j} from the two-level FP64 table, rounded to C.
// x / d and x % d for x >= 0, d > 0: 32-bit unsigned division while both
// fit (a 64-bit division is a long instruction sequence on this GPU)
__device__ __forceinline__ void divmod_fast(int64_t x, int64_t d, int64_t& q, int64_t& r) {
    if (((uint64_t)x | (uint64_t)d) < (uint64_t(1) << 32)) {
        const uint32_t qq = (uint32_t)x / (uint32_t)d;
        q = qq;
        r = (int64_t)((uint32_t)x - qq * (uint32_t)d);
    } else {
        q = x / d;
        r = x % d;
    }
}
__device__ __forceinline__ int64_t div_fast(int64_t x, int64_t d) {
    int64_t q, r;
    divmod_fast(x, d, q, r);
    return q;
}
__device__ __forceinline__ int64_t mod_fast(int64_t x, int64_t d) {
    int64_t q, r;
    divmod_fast(x, d, q, r);
    return r;
}

template <typename C>
__device__ __forceinline__ C split_twiddle(const AxisDesc& ax, const double2* __restrict__ tw64, int64_t j) {
    int64_t hi, lo;
    divmod_fast(j, ax.spB, hi, lo);
    const double2 a = tw64[ax.sp_off1 + lo];
    const double2 b = tw64[ax.sp_off2 + hi];
    const double2 w = cmul(a, b);
    using T = decltype(C{}.x);
    return C{(T)w.x, (T)w.y};
}

template <typename T> __device__ __forceinline__ T* lds_base() {
    extern __shared__ __align__(16) unsigned char ahom_smem[];
    return reinterpret_cast<T*>(ahom_smem);
}

// Copy of an axis's twiddle table (L entries) in LDS after the tile buffers;
// the Stockham stages read it there instead of from global memory in every
// butterfly.  Visible to the first transform through the barrier that follows
// the tile's gather.  (The block reductions after a tile may reuse the space.)
template <typename C>
__device__ __forceinline__ C* stage_twiddles(C* twl, const C* __restrict__ tw, int L) {
    for (int i = threadIdx.x; i < L; i += blockDim.x) twl[i] = tw[i];
    return twl;
}

// block-wide sum of NV doubles per thread (fixed order) over NT threads (the
// workgroup size, a power of two); result valid in thread 0
template <int NV, int NT = AHOM_WG>
__device__ void block_sum(double* vals, double* scratch) {
    const int tid = threadIdx.x;
    for (int c = 0; c < NV; ++c) scratch[c * NT + tid] = vals[c];
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
        if (tid < off)
            for (int c = 0; c < NV; ++c) scratch[c * NT + tid] += scratch[c * NT + tid + off];
        __syncthreads();
    }
    if (tid == 0)
        for (int c = 0; c < NV; ++c) vals[c] = scratch[c * NT];
}

template <int DIM, int PH = PHYS_ELASTIC> using Comp = Fields<DIM, PH>;

}  // namespace

// =============================================================================
// axis 0: real-space turnaround
// =============================================================================
// One tile (a.NC columns) of the axis-0 pass for load case `load`; the
// stress sums of REAL_TURN are added to sig[0..ncomp) (per thread), and with
// a.en_part set the sum of eps : tau to sig[ncomp].  All threads of the
// workgroup take part (LDS barriers inside).
template <typename T, int DIM, int MODE, int PH = PHYS_ELASTIC>
__device__ void real_tile(const RealArgs& a, const LoadState& st, int load, int64_t tile, double* sig) {
    using C = typename CT<T>::t;
    constexpr int NC_ = Comp<DIM, PH>::N, NP = Comp<DIM, PH>::NP;
    const Plan& P = *a.plan;
    const AxisDesc& ax = P.ax[0];
    const int L = ax.len, H = ax.slen;
    const int64_t I = P.S / H;
    const int64_t c0 = tile * a.NC;
    const int ncol = (int)((I - c0) < a.NC ? (I - c0) : a.NC);
    const int CS = a.CS;
    const int tid = threadIdx.x;
    const UDiv by_nc(a.NC);

    // LDS: the NP packed fields (a.NC columns each, field p's column j at
    // (p a.NC + j) CS), the Stockham ping-pong buffer of the same size (all
    // fields are transformed in one call: one barrier per stage for all of
    // them), the twiddle table
    C* Z = lds_base<C>();
    C* tmp = Z + NP * a.NC * CS;
    C* twl = stage_twiddles(tmp + NP * a.NC * CS, reinterpret_cast<const C*>(a.tw) + ax.tw_off, L);
    const int ncol_all = (NP - 1) * a.NC + ncol;   // through the last valid column of the last field

    int src_buf = 0;
    if (MODE == REAL_TURN) src_buf = st.iter & 1;
    if (MODE == REAL_TO_REAL) src_buf = st.final_buf;
    const C* src = reinterpret_cast<const C*>(src_buf ? a.buf1 : a.buf0) + (int64_t)load * NC_ * P.S;
    C* dst = reinterpret_cast<C*>((MODE == REAL_TURN ? (src_buf ^ 1) : 0) ? a.buf1 : a.buf0) + (int64_t)load * NC_ * P.S;
    const C* tw = reinterpret_cast<const C*>(a.tw) + ax.tw_off;

    // Lame pairs of the law points e = tid + q blockDim (q < GEPL): phase ids
    // and table entries are loaded up front, all independent, so the law does
    // not wait for two dependent global loads per point.  Tiles with more law
    // points than GEPL per thread use the per-point loads below.
    constexpr int GEPL = 8;
    const bool pre_law = MODE == REAL_TURN && L * a.NC <= GEPL * (int)blockDim.x;
    T lamq[GEPL], muq[GEPL];
    if (pre_law) {
        int phq[GEPL];
#pragma unroll
        for (int q = 0; q < GEPL; ++q) {
            const int e = tid + q * (int)blockDim.x;
            int n, j;
            by_nc.divmod(e, n, j);
            const bool ok = e < L * a.NC && j < ncol;
            const int64_t pt = ok ? (int64_t)n * I + c0 + j : c0;
            if (a.lame_pts) {
                lamq[q] = (T)a.lame_pts[2 * pt];
                muq[q] = (T)a.lame_pts[2 * pt + 1];
            } else {
                phq[q] = a.phase[pt];
            }
        }
        if (!a.lame_pts) {
#pragma unroll
            for (int q = 0; q < GEPL; ++q) {
                lamq[q] = (T)a.lame_tab[2 * phq[q]];
                muq[q] = (T)a.lame_tab[2 * phq[q] + 1];
            }
        }
    }

    if (MODE != REAL_FROM_REAL) {
        // ---- gather the half spectra and form packed full spectra Z_p = A + i B
        for (int e = tid; e < H * a.NC; e += blockDim.x) {
            int k, j;
            by_nc.divmod(e, k, j);
            if (j >= ncol) continue;
            const int64_t col = c0 + j;
            C w = C{(T)1, (T)0};
            if (ax.split) w = split_twiddle<C>(ax, a.tw64, div_fast(col, ax.qdiv) * (int64_t)k);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int fa = 2 * p, fb = 2 * p + 1;
                C A = src[(int64_t)fa * P.S + (int64_t)k * I + col];
                C B = fb < NC_ ? src[(int64_t)fb * P.S + (int64_t)k * I + col] : C{(T)0, (T)0};
                if (ax.split) { A = cmulc(A, w); B = cmulc(B, w); }
                if (k == 0 || 2 * k == L) { A.y = 0; B.y = 0; }
                C* Zp = Z + p * a.NC * CS + j * CS;
                Zp[k] = C{A.x - B.y, A.y + B.x};
                if (k > 0 && 2 * k != L) Zp[L - k] = C{A.x + B.y, B.x - A.y};
            }
        }
        __syncthreads();
        lds_fft<+1>(Z, tmp, ncol_all, CS, ax, twl);
    }

    if (MODE == REAL_TO_REAL) {
        double* out = a.real_io + (int64_t)load * NC_ * P.m;
        for (int e = tid; e < L * a.NC; e += blockDim.x) {
            int n, j;
            by_nc.divmod(e, n, j);
            if (j >= ncol) continue;
            const int64_t pt = (int64_t)n * I + c0 + j;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const C z = Z[p * a.NC * CS + j * CS + n];
                double* oa = out + (int64_t)(2 * p) * P.m + pt;
                double* ob = out + (int64_t)(2 * p + 1) * P.m + pt;
                *oa = (double)z.x + (a.accumulate ? *oa : 0.0);
                if (2 * p + 1 < NC_) *ob = (double)z.y + (a.accumulate ? *ob : 0.0);
            }
        }
        return;
    }

    if (MODE == REAL_TURN) {
        const T lam0 = (T)a.lam0, mu0 = (T)a.mu0;
        auto point = [&](int n, int j, T lam, T mu) __attribute__((always_inline)) {
            T eps[NC_];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const C z = Z[p * a.NC * CS + j * CS + n];
                eps[2 * p] = z.x;
                if (2 * p + 1 < NC_) eps[2 * p + 1] = z.y;
            }
            T tau[NC_];
            if constexpr (PH == PHYS_THERMAL) {
                // flux q = k e, polarization (k - k0) e; k in the lambda slot
#pragma unroll
                for (int c = 0; c < NC_; ++c) {
                    sig[c] += (double)(lam * eps[c]);
                    tau[c] = (lam - lam0) * eps[c];
                }
            } else {
                const T tr = DIM == 3 ? eps[0] + eps[1] + eps[2] : eps[0] + eps[1];
                const T dl = lam - lam0, dm = (T)2 * (mu - mu0);
#pragma unroll
                for (int c = 0; c < NC_; ++c) {
                    const bool diag = DIM == 3 ? c < 3 : c < 2;
                    const T s = (T)2 * mu * eps[c] + (diag ? lam * tr : (T)0);
                    sig[c] += (double)s;
                    tau[c] = dm * eps[c] + (diag ? dl * tr : (T)0);
                }
            }
            if (a.en_part) {
                double en = 0.0;
#pragma unroll
                for (int c = 0; c < NC_; ++c) en += field_weight(PH, DIM, c) * (double)eps[c] * (double)tau[c];
                sig[NC_] += en;
            }
#pragma unroll
            for (int p = 0; p < NP; ++p)
                Z[p * a.NC * CS + j * CS + n] = C{tau[2 * p], 2 * p + 1 < NC_ ? tau[2 * p + 1] : (T)0};
        };
        if (pre_law) {
#pragma unroll
            for (int q = 0; q < GEPL; ++q) {
                const int e = tid + q * (int)blockDim.x;
                int n, j;
                by_nc.divmod(e, n, j);
                if (e < L * a.NC && j < ncol) point(n, j, lamq[q], muq[q]);
            }
        } else {
            for (int e = tid; e < L * a.NC; e += blockDim.x) {
                int n, j;
                by_nc.divmod(e, n, j);
                if (j >= ncol) continue;
                const int64_t pt = (int64_t)n * I + c0 + j;
                if (a.lame_pts) {
                    point(n, j, (T)a.lame_pts[2 * pt], (T)a.lame_pts[2 * pt + 1]);
                } else {
                    const int ph = a.phase[pt];
                    point(n, j, (T)a.lame_tab[2 * ph], (T)a.lame_tab[2 * ph + 1]);
                }
            }
        }
    } else {  // REAL_FROM_REAL: eps = eps_bar + init
        const double* in = a.real_io + (int64_t)load * NC_ * P.m;
        const double* eb = a.eps_bar + (int64_t)load * NC_;
        for (int e = tid; e < L * a.NC; e += blockDim.x) {
            int n, j;
            by_nc.divmod(e, n, j);
            if (j >= ncol) continue;
            const int64_t pt = (int64_t)n * I + c0 + j;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int fa = 2 * p, fb = 2 * p + 1;
                const T va = (T)(eb[fa] + in[(int64_t)fa * P.m + pt]);
                const T vb = fb < NC_ ? (T)(eb[fb] + in[(int64_t)fb * P.m + pt]) : (T)0;
                Z[p * a.NC * CS + j * CS + n] = C{va, vb};
            }
        }
    }
    __syncthreads();
    lds_fft<-1>(Z, tmp, ncol_all, CS, ax, twl);

    // ---- split the packed spectra and store the half spectra
    const T scale = MODE == REAL_FROM_REAL ? (T)(1.0 / L) : (T)1;
    for (int e = tid; e < H * a.NC; e += blockDim.x) {
        int k, j;
        by_nc.divmod(e, k, j);
        if (j >= ncol) continue;
        const int64_t col = c0 + j;
        C w = C{(T)1, (T)0};
        if (ax.split) w = split_twiddle<C>(ax, a.tw64, div_fast(col, ax.qdiv) * (int64_t)k);
        const int km = k == 0 ? 0 : L - k;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const C* Zp = Z + p * a.NC * CS + j * CS;
            const C zk = Zp[k], zm = Zp[km];
            // A = (Z_k + conj Z_{-k})/2,  B = (Z_k - conj Z_{-k})/(2i)
            C A = C{(T)0.5 * (zk.x + zm.x) * scale, (T)0.5 * (zk.y - zm.y) * scale};
            C B = C{(T)0.5 * (zk.y + zm.y) * scale, (T)0.5 * (zm.x - zk.x) * scale};
            if (ax.split) { A = cmul(A, w); B = cmul(B, w); }
            dst[(int64_t)(2 * p) * P.S + (int64_t)k * I + col] = A;
            if (2 * p + 1 < NC_) dst[(int64_t)(2 * p + 1) * P.S + (int64_t)k * I + col] = B;
        }
    }
}

template <typename T, int DIM, int MODE, int PH>
__global__ void __launch_bounds__(AHOM_WG) k_real(RealArgs a) {
    using C = typename CT<T>::t;
    constexpr int NC_ = Comp<DIM, PH>::N, NP = Comp<DIM, PH>::NP;
    const int load = blockIdx.y;
    if (MODE == REAL_TURN && a.st[load].done) return;
    double sig[NC_ + 1];
#pragma unroll
    for (int c = 0; c <= NC_; ++c) sig[c] = 0.0;
    real_tile<T, DIM, MODE, PH>(a, a.st[load], load, blockIdx.x, sig);
    if (MODE == REAL_TURN) {
        __syncthreads();
        double* red = reinterpret_cast<double*>(lds_base<C>() + 2 * NP * a.NC * a.CS);
        block_sum<NC_ + 1>(sig, red);
        if (threadIdx.x == 0) {
            for (int c = 0; c < NC_; ++c) a.sig_part[((int64_t)load * gridDim.x + blockIdx.x) * NC_ + c] = sig[c];
            if (a.en_part) a.en_part[(int64_t)load * gridDim.x + blockIdx.x] = sig[NC_];
        }
    }
}

// =============================================================================
// middle axes: plain complex FFT passes (also the bare pattern DFT)
// =============================================================================
// One tile of a middle-axis pass (field `field` of load case `load`).
template <typename T, int DIR>
__device__ void axis_tile(const AxisArgs& a, int par, int load, int field, int64_t tile) {
    using C = typename CT<T>::t;
    const Plan& P = *a.plan;
    const AxisDesc& ax = P.ax[a.axis];
    const int L = ax.len;
    int64_t O = 1, I = 1;
    for (int b = 0; b < a.axis; ++b) O *= a.slen0_full && b == 0 ? P.ax[0].len : P.ax[b].slen;
    for (int b = a.axis + 1; b < P.D; ++b) I *= P.ax[b].slen;
    const int64_t ncols = O * I;
    const int64_t c0 = tile * a.NC;
    const int ncol = (int)((ncols - c0) < a.NC ? (ncols - c0) : a.NC);
    const int CS = a.CS;
    C* base = reinterpret_cast<C*>(par ? a.buf1 : a.buf0) + (int64_t)load * a.load_stride + (int64_t)field * a.field_stride;
    const C* tw = reinterpret_cast<const C*>(a.tw) + ax.tw_off;
    C* X = lds_base<C>();
    C* tmp = X + a.NC * CS;
    C* twl = stage_twiddles(tmp + a.NC * CS, tw, L);
    const bool rowmajor = I >= a.NC;
    const int tid = threadIdx.x;
    const UDiv by_nc(a.NC), by_l(L);

    for (int e = tid; e < L * a.NC; e += blockDim.x) {
        int j, l;
        if (rowmajor) by_nc.divmod(e, l, j); else by_l.divmod(e, j, l);
        if (j >= ncol) continue;
        const int64_t col = c0 + j;
        int64_t cq, cr;
        divmod_fast(col, I, cq, cr);
        const int64_t addr = cq * (int64_t)L * I + cr + (int64_t)l * I;
        C v = base[addr];
        if (DIR > 0 && ax.split) v = cmulc(v, split_twiddle<C>(ax, a.tw64, div_fast(cr, ax.qdiv) * (int64_t)l));
        X[j * CS + l] = v;
    }
    __syncthreads();
    lds_fft<DIR>(X, tmp, ncol, CS, ax, twl);
    for (int e = tid; e < L * a.NC; e += blockDim.x) {
        int j, l;
        if (rowmajor) by_nc.divmod(e, l, j); else by_l.divmod(e, j, l);
        if (j >= ncol) continue;
        const int64_t col = c0 + j;
        int64_t cq, cr;
        divmod_fast(col, I, cq, cr);
        const int64_t addr = cq * (int64_t)L * I + cr + (int64_t)l * I;
        C v = X[j * CS + l];
        if (DIR < 0 && ax.split) v = cmul(v, split_twiddle<C>(ax, a.tw64, div_fast(cr, ax.qdiv) * (int64_t)l));
        base[addr] = v;
    }
}

template <typename T, int DIR>
__global__ void __launch_bounds__(AHOM_WG) k_axis(AxisArgs a) {
    const int load = blockIdx.z;
    if (a.st && a.st[load].done) return;
    axis_tile<T, DIR>(a, a.st ? (a.st[load].iter + 1) & 1 : 0, load, blockIdx.y, blockIdx.x);
}

// =============================================================================
// last axis: spectral turnaround with Gamma0 and the residual terms
// =============================================================================
// One tile of the last-axis pass; the residual terms are added to res.
template <typename T, int DIM, int MODE, int PH = PHYS_ELASTIC>
__device__ void spec_tile(const SpecArgs& a, const LoadState& st, int load, int64_t tile, double& res, double& cau) {
    using C = typename CT<T>::t;
    constexpr int NC_ = Comp<DIM, PH>::N, NT = Comp<DIM, PH>::NT;
    const Plan& P = *a.plan;
    const int par = MODE == SPEC_INIT ? 0 : (st.iter + 1) & 1;
    const int D = P.D;
    const AxisDesc& ax = P.ax[D - 1];
    const int L = ax.len;
    const int64_t ncols = P.S / L;
    const int64_t c0 = tile * a.NC;
    const int ncol = (int)((ncols - c0) < a.NC ? (ncols - c0) : a.NC);
    const int CS = a.CS;
    const int tid = threadIdx.x;
    C* base = reinterpret_cast<C*>(par ? a.buf1 : a.buf0) + (int64_t)load * NC_ * P.S;
    C* tb = reinterpret_cast<C*>(a.tbuf) + (int64_t)load * NT * P.S;
    const C* tw = reinterpret_cast<const C*>(a.tw) + ax.tw_off;
    // LDS: the NC_ fields (field f's column j at (f a.NC + j) CS), the
    // Stockham ping-pong buffer of the same size (all fields in one
    // transform call), the twiddle table
    C* F = lds_base<C>();
    C* tmp = F + NC_ * a.NC * CS;
    C* twl = stage_twiddles(tmp + NC_ * a.NC * CS, tw, L);
    const int ncol_all = (NC_ - 1) * a.NC + ncol;
    const UDiv by_l(L);

    for (int e = tid; e < L * a.NC; e += blockDim.x) {
        int j, l;
        by_l.divmod(e, j, l);
        if (j >= ncol) continue;
        const int64_t addr = (c0 + j) * L + l;
#pragma unroll
        for (int f = 0; f < NC_; ++f) F[f * a.NC * CS + j * CS + l] = base[(int64_t)f * P.S + addr];
    }
    __syncthreads();
    lds_fft<-1>(F, tmp, ncol_all, CS, ax, twl);

    const double* eb = a.eps_bar + (int64_t)load * NC_;
    const T inv_m = (T)(1.0 / (double)P.m);
    const T mu0 = (T)a.mu0, beta = (T)a.beta;
    // |eps_hat(n+1) - eps_hat(n)|^2 from the traction step: (|dt|^2 + c1 |xi . dt|^2) / (2 mu0^2)
    // in elasticity, |dt|^2 / k0^2 for conductivity
    const double cau_c1 = PH == PHYS_THERMAL ? 0.0 : 1.0 - 4.0 * a.beta + 2.0 * a.beta * a.beta;
    const int L0 = P.ax[0].len;
    // Centred numerators in exact doubles while emax <= 2^24 (A in [0, emax),
    // 0 <= kappa_s < e_s <= emax: products < 2^48, sums of three < 2^53), the
    // same integers as the 64-bit formula without a 64-bit division per point.
    const int64_t emax = P.fm.emax;
    const bool nfast = emax <= (int64_t(1) << 24);
    const double emax_d = (double)emax, inv_e = 1.0 / emax_d;
    double Ad[3][3];
    for (int i2 = 0; i2 < 3; ++i2)
        for (int s2 = 0; s2 < 3; ++s2) Ad[i2][s2] = (i2 < DIM && s2 < DIM) ? (double)P.fm.A[i2][s2] : 0.0;
    const bool small_cols = ncols < (int64_t(1) << 31);
    for (int e = tid; e < L * a.NC; e += blockDim.x) {
        int j, l;
        by_l.divmod(e, j, l);
        if (j >= ncol) continue;
        // position -> kappa (32-bit division while the column count fits)
        int64_t kpos[AHOM_MAX_AXES];
        if (small_cols) {
            uint32_t o = (uint32_t)(c0 + j);
            for (int b = D - 2; b >= 0; --b) {
                const uint32_t sl = (uint32_t)P.ax[b].slen;
                kpos[b] = o % sl;
                o /= sl;
            }
        } else {
            int64_t o = c0 + j;
            for (int b = D - 2; b >= 0; --b) {
                const int64_t sl = P.ax[b].slen;
                kpos[b] = o % sl;
                o /= sl;
            }
        }
        kpos[D - 1] = l;
        int64_t kap[3] = {0, 0, 0};
        for (int b = 0; b < D; ++b) kap[P.ax[b].snf] += P.ax[b].mult * kpos[b];
        const bool is_zero = kap[0] == 0 && kap[1] == 0 && kap[2] == 0;
        int64_t N[3];
        int half = 0;
        if (nfast) {
            for (int i2 = 0; i2 < DIM; ++i2) {
                double x = 0.0;
                for (int s2 = 0; s2 < DIM; ++s2) x += Ad[i2][s2] * (double)kap[s2];
                double r = x - floor(x * inv_e) * emax_d;
                if (r < 0) r += emax_d;
                if (r >= emax_d) r -= emax_d;
                if (2 * r >= emax_d) r -= emax_d;
                if (2 * r == -emax_d) half = 1;
                N[i2] = (int64_t)r;
            }
        } else {
            half = ahom_centred_numerators(P.fm, kap, N);
        }
        // self-conjugate test 2 kappa = 0 (mod e): for 0 <= kappa_s < e_s a comparison
        bool sc = true;
        if (half)
            for (int s2 = 0; s2 < DIM; ++s2) {
                const int64_t k2 = 2 * kap[s2], es = P.fm.e[s2];
                sc = sc && ((kap[s2] >= 0 && kap[s2] < es) ? (k2 == 0 || k2 == es) : (k2 % es == 0));
            }
        const bool active = !half || sc;
        const int64_t spos = (c0 + j) * L + l;
        C* fp[NC_];
#pragma unroll
        for (int f = 0; f < NC_; ++f) fp[f] = F + f * a.NC * CS + j * CS + l;
        if (is_zero) {
#pragma unroll
            for (int f = 0; f < NC_; ++f) *fp[f] = C{(T)eb[f], (T)0};
            continue;
        }
        if (!active) {
#pragma unroll
            for (int f = 0; f < NC_; ++f) *fp[f] = C{(T)0, (T)0};
            continue;
        }
        double hd[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < DIM; ++i)
            for (int q = 0; q < DIM; ++q) hd[i] += P.fm.G[i][q] * (double)N[q];
        double hn = 0.0;
        for (int i = 0; i < DIM; ++i) hn += hd[i] * hd[i];
        hn = 1.0 / sqrt(hn);
        T xi[3];
        for (int i = 0; i < DIM; ++i) xi[i] = (T)(hd[i] * hn);
        if constexpr (MODE == SPEC_INIT && PH == PHYS_THERMAL) {
            // e_hat(0) = value * L0 / m; t(0) = -k0 e_hat(0) . xi
            const T sc = (T)((double)L0 / (double)P.m), k0 = (T)a.mu0;
            C acc = C{(T)0, (T)0};
#pragma unroll
            for (int f = 0; f < NC_; ++f) { const C v = *fp[f]; acc.x += v.x * sc * xi[f]; acc.y += v.y * sc * xi[f]; }
            tb[spos] = C{-k0 * acc.x, -k0 * acc.y};
            continue;
        }
        if constexpr (MODE == SPEC_INIT && PH == PHYS_ELASTIC) {
            // eps_hat(0) = value * L0 / m; t(0) = -(C0 : eps_hat(0)) xi
            const T sc = (T)((double)L0 / (double)P.m);
            C ev[NC_];
#pragma unroll
            for (int f = 0; f < NC_; ++f) { C v = *fp[f]; ev[f] = C{v.x * sc, v.y * sc}; }
            const T lam0 = (T)a.lam0_init, two_mu0 = (T)2 * (T)a.mu0;
            C trc = DIM == 3 ? cadd(cadd(ev[0], ev[1]), ev[2]) : cadd(ev[0], ev[1]);
            C E[3][3];
            if constexpr (DIM == 3) {
                E[0][0] = ev[0]; E[1][1] = ev[1]; E[2][2] = ev[2];
                E[1][2] = E[2][1] = ev[3]; E[0][2] = E[2][0] = ev[4]; E[0][1] = E[1][0] = ev[5];
            } else {
                E[0][0] = ev[0]; E[1][1] = ev[1]; E[0][1] = E[1][0] = ev[2];
            }
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                C acc = C{lam0 * trc.x * xi[i], lam0 * trc.y * xi[i]};
#pragma unroll
                for (int q = 0; q < DIM; ++q) { acc.x += two_mu0 * E[i][q].x * xi[q]; acc.y += two_mu0 * E[i][q].y * xi[q]; }
                tb[(int64_t)i * P.S + spos] = C{-acc.x, -acc.y};
            }
            continue;
        }
        // tau_hat tensor entries (normalized by 1/m)
        C tv[NC_];
#pragma unroll
        for (int f = 0; f < NC_; ++f) { C v = *fp[f]; tv[f] = C{v.x * inv_m, v.y * inv_m}; }
        C t[NT];
        if constexpr (PH == PHYS_THERMAL) {
            // normal flux tau_hat . xi
            t[0] = C{(T)0, (T)0};
#pragma unroll
            for (int i = 0; i < DIM; ++i) { t[0].x += tv[i].x * xi[i]; t[0].y += tv[i].y * xi[i]; }
        } else if constexpr (DIM == 3) {
            // components (11,22,33,23,13,12)
            const C T00 = tv[0], T11 = tv[1], T22 = tv[2], T12 = tv[3], T02 = tv[4], T01 = tv[5];
            t[0] = C{T00.x * xi[0] + T01.x * xi[1] + T02.x * xi[2], T00.y * xi[0] + T01.y * xi[1] + T02.y * xi[2]};
            t[1] = C{T01.x * xi[0] + T11.x * xi[1] + T12.x * xi[2], T01.y * xi[0] + T11.y * xi[1] + T12.y * xi[2]};
            t[NT - 1] = C{T02.x * xi[0] + T12.x * xi[1] + T22.x * xi[2], T02.y * xi[0] + T12.y * xi[1] + T22.y * xi[2]};
        } else {
            // components (11,22,12)
            const C T00 = tv[0], T11 = tv[1], T01 = tv[2];
            t[0] = C{T00.x * xi[0] + T01.x * xi[1], T00.y * xi[0] + T01.y * xi[1]};
            t[1] = C{T01.x * xi[0] + T11.x * xi[1], T01.y * xi[0] + T11.y * xi[1]};
        }
        // residual: sigma_hat(n) xi = t(n+1) - t(n) on active frequencies;
        // conjugate gradients: the traction of the updated iterate, t + alpha t_p
        const double wgt = (kpos[0] == 0 || 2 * kpos[0] == L0) ? 1.0 : 2.0;
        const bool chk = ahom_check_iter(st.iter, a.resid_period, a.max_iter);
        const bool wrt = ahom_write_traction(st.iter, a.resid_period, a.max_iter);
        const T cg_a = a.cg_alpha ? (T)a.cg_alpha[load] : (T)0;
        double r2 = 0.0, xdx = 0.0, xdy = 0.0;
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            if (a.cg_alpha) {
                const C old = tb[(int64_t)c * P.S + spos];
                const C nt = C{old.x + cg_a * t[c].x, old.y + cg_a * t[c].y};
                r2 += (double)nt.x * (double)nt.x + (double)nt.y * (double)nt.y;
                tb[(int64_t)c * P.S + spos] = nt;
                continue;
            }
            if (chk) {
                const C old = tb[(int64_t)c * P.S + spos];
                const double dx = (double)t[c].x - (double)old.x, dy = (double)t[c].y - (double)old.y;
                r2 += dx * dx + dy * dy;
                xdx += (double)xi[c] * dx;
                xdy += (double)xi[c] * dy;
                if (a.dout) {
                    const int64_t o = ((int64_t)load * NT + c) * P.S + spos;
                    reinterpret_cast<float2*>(a.dout)[o] = float2{(float)dx, (float)dy};
                    reinterpret_cast<float2*>(a.dneg)[o] = float2{(float)-dx, (float)-dy};
                }
            }
            if (wrt) tb[(int64_t)c * P.S + spos] = t[c];
        }
        res += wgt * r2;
        // Cauchy term: eps_hat(n+1) - eps_hat(n) = -sym(xi (x) K^{-1} dt) has squared
        // norm (|dt|^2 + (1 - 4 beta + 2 beta^2) |xi . dt|^2) / (2 mu0^2)
        cau += wgt * (r2 + cau_c1 * (xdx * xdx + xdy * xdy));
        if (a.toff) {
            const C* to = reinterpret_cast<const C*>(a.toff) + (int64_t)load * NT * P.S;
#pragma unroll
            for (int c = 0; c < NT; ++c) t[c] = cadd(t[c], to[(int64_t)c * P.S + spos]);
        }
        if constexpr (PH == PHYS_THERMAL) {
            // e_hat = -xi (tau_hat . xi) / k0
            const T ik0 = (T)1 / mu0;
#pragma unroll
            for (int i = 0; i < DIM; ++i) *fp[i] = C{-xi[i] * t[0].x * ik0, -xi[i] * t[0].y * ik0};
        } else {
        // v = (t - beta (xi . t) xi) / mu0 ; eps_hat = -sym(xi (x) v)
        C xt = C{(T)0, (T)0};
#pragma unroll
        for (int i = 0; i < DIM; ++i) { xt.x += xi[i] * t[i].x; xt.y += xi[i] * t[i].y; }
        C v[3];
        const T im0 = (T)1 / mu0;
#pragma unroll
        for (int i = 0; i < DIM; ++i) v[i] = C{(t[i].x - beta * xt.x * xi[i]) * im0, (t[i].y - beta * xt.y * xi[i]) * im0};
        if constexpr (DIM == 3) {
            *fp[0] = C{-xi[0] * v[0].x, -xi[0] * v[0].y};
            *fp[1] = C{-xi[1] * v[1].x, -xi[1] * v[1].y};
            *fp[2] = C{-xi[2] * v[2].x, -xi[2] * v[2].y};
            *fp[3] = C{(T)-0.5 * (xi[1] * v[2].x + xi[2] * v[1].x), (T)-0.5 * (xi[1] * v[2].y + xi[2] * v[1].y)};
            *fp[4] = C{(T)-0.5 * (xi[0] * v[2].x + xi[2] * v[0].x), (T)-0.5 * (xi[0] * v[2].y + xi[2] * v[0].y)};
            *fp[5] = C{(T)-0.5 * (xi[0] * v[1].x + xi[1] * v[0].x), (T)-0.5 * (xi[0] * v[1].y + xi[1] * v[0].y)};
        } else {
            *fp[0] = C{-xi[0] * v[0].x, -xi[0] * v[0].y};
            *fp[1] = C{-xi[1] * v[1].x, -xi[1] * v[1].y};
            *fp[NC_ - 1] = C{(T)-0.5 * (xi[0] * v[1].x + xi[1] * v[0].x), (T)-0.5 * (xi[0] * v[1].y + xi[1] * v[0].y)};
        }
        }
    }
    if (MODE == SPEC_INIT) return;
    __syncthreads();
    lds_fft<+1>(F, tmp, ncol_all, CS, ax, twl);
    for (int e = tid; e < L * a.NC; e += blockDim.x) {
        int j, l;
        by_l.divmod(e, j, l);
        if (j >= ncol) continue;
        const int64_t addr = (c0 + j) * L + l;
#pragma unroll
        for (int f = 0; f < NC_; ++f) base[(int64_t)f * P.S + addr] = F[f * a.NC * CS + j * CS + l];
    }
}

template <typename T, int DIM, int MODE, int PH>
__global__ void __launch_bounds__(AHOM_WG) k_spec(SpecArgs a) {
    using C = typename CT<T>::t;
    constexpr int NC_ = Comp<DIM, PH>::N;
    const int load = blockIdx.y;
    if (a.st[load].done) return;
    double res = 0.0, cau = 0.0;
    spec_tile<T, DIM, MODE, PH>(a, a.st[load], load, blockIdx.x, res, cau);
    if (MODE == SPEC_INIT) return;
    double rv[2] = {res, cau};
    block_sum<2>(rv, reinterpret_cast<double*>(lds_base<C>() + 2 * NC_ * a.NC * a.CS));
    if (threadIdx.x == 0) {
        a.res_part[(int64_t)load * gridDim.x + blockIdx.x] = rv[0];
        if (a.cau_part) a.cau_part[(int64_t)load * gridDim.x + blockIdx.x] = rv[1];
    }
}

// =============================================================================
// residual / mean stress reduction and loop control (one block per load)
// =============================================================================
template <int DIM, int PH>
__global__ void __launch_bounds__(AHOM_WG) k_reduce(ReduceArgs a) {
    constexpr int NC_ = Comp<DIM, PH>::N;
    __shared__ double scratch[(NC_ + 1) * AHOM_WG];
    const int load = blockIdx.x;
    LoadState& st = a.st[load];
    if (st.done) return;
    const int tid = threadIdx.x;
    double v[NC_ + 1];
    for (int c = 0; c <= NC_; ++c) v[c] = 0.0;
    for (int w = tid; w < a.n_real; w += AHOM_WG)
        for (int c = 0; c < NC_; ++c) v[c] += a.sig_part[((int64_t)load * a.n_real + w) * NC_ + c];
    for (int w = tid; w < a.n_spec; w += AHOM_WG) v[NC_] += a.res_part[(int64_t)load * a.n_spec + w];
    block_sum<NC_ + 1>(v, scratch);
    double cs[1] = {0.0};
    if (a.chist) {
        __syncthreads();
        for (int w = tid; w < a.n_spec; w += AHOM_WG) cs[0] += a.cau_part[(int64_t)load * a.n_spec + w];
        block_sum<1>(cs, scratch);
    }
    if (tid != 0) return;
    const double inv_m = 1.0 / (double)a.m;
    double mean[NC_];
    double fro = 0.0;
    for (int c = 0; c < NC_; ++c) {
        mean[c] = v[c] * inv_m + (a.sig_base ? a.sig_base[(int64_t)load * NC_ + c] : 0.0);
        fro += field_weight(PH, DIM, c) * mean[c] * mean[c];
    }
    const int n = st.iter;
    for (int c = 0; c < NC_; ++c) st.mean[c] = mean[c];
    if (!ahom_check_iter(n, a.resid_period, a.max_iter)) {
        // residual not evaluated on this iteration (recorded as -1)
        if (n < a.hist_cap) a.hist[(int64_t)load * a.hist_cap + n] = -1.0;
        if (a.chist && n < a.hist_cap) a.chist[(int64_t)load * a.hist_cap + n] = -1.0;
        st.iter = n + 1;
        return;
    }
    const double r = sqrt(v[NC_]) / sqrt(fro);
    if (n < a.hist_cap) a.hist[(int64_t)load * a.hist_cap + n] = r;
    // Cauchy measure |eps(n+1) - eps(n)| / |eps(0)| (Parseval, 1/m-normalised transform)
    double c = r;
    if (a.chist) {
        c = sqrt(a.cau_scale * cs[0]) / a.norm0[load];
        if (n < a.hist_cap) a.chist[(int64_t)load * a.hist_cap + n] = c;
    }
    if (n == 0) st.r0 = r;
    st.resid = r;
    const bool bad = !(r == r) || isinf(r) || (st.r0 > 0.0 && r > 1e3 * st.r0);
    if (bad) { st.done = 1; st.status = 2; st.final_buf = n & 1; return; }
    if ((a.stop_cauchy ? c : r) <= a.tol) { st.done = 1; st.status = 0; st.final_buf = n & 1; return; }
    if (n >= a.max_iter) { st.done = 1; st.status = 1; st.final_buf = n & 1; return; }
    st.iter = n + 1;
}

// =============================================================================
// batched solves: persistent workgroups, one (pattern, load) item at a time
// =============================================================================
namespace {

// Global-memory writes of this workgroup made visible to its later reads.
// An item's buffers are written and read by the one workgroup that owns the
// item, so workgroup scope suffices; agent scope would write back and
// invalidate the whole L2 of the XCD at every pass.
__device__ __forceinline__ void wg_mem_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Pass boundary of an item: workgroup-level for k = 1; for a group of k
// workgroups (any CUs and XCDs) an agent-scope release, an arrival on the
// item's counter and a wait for the k arrivals of this phase, then an
// agent-scope acquire.  Every workgroup of the group calls it the same number
// of times (phase counts them).  The wait is bounded (wait ticks of the
// 100 MHz clock, 4 s by default): without the group's arrivals by then it
// marks the counter (bit 30) and this and all later barriers of the item stop
// waiting, so a lost workgroup cannot hang the launch (the item's result is
// then wrong and its status says so).
constexpr int kGroupAbort = 1 << 30;
__device__ __forceinline__ void group_sync(const BatchItem& it, int& phase, long long wait) {
    if (it.k == 1) {
        wg_mem_sync();
        return;
    }
    ++phase;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(it.gcount, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int target = it.k * phase;
        const long long t0 = wall_clock64();
        for (;;) {
            const int c = __hip_atomic_load(it.gcount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((c & kGroupAbort) || c >= target) break;
            if (wall_clock64() - t0 > wait) {
                __hip_atomic_fetch_or(it.gcount, kGroupAbort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// element loops below: the group's k workgroups share them (slot = this
// workgroup's position in the group)
template <typename T>
__device__ void wg_fill_state(void* buf, const double* eps_bar, int64_t S, int64_t row, int nfield, int slot, int k) {
    using C = typename CT<T>::t;
    C* b = reinterpret_cast<C*>(buf);
    const int64_t n = (int64_t)nfield * S;
    for (int64_t i = (int64_t)slot * blockDim.x + threadIdx.x; i < n; i += (int64_t)k * blockDim.x) {
        const int f = (int)(i / S);
        const int64_t k = i - (int64_t)f * S;
        b[i] = k < row ? C{(T)eps_bar[f], (T)0} : C{(T)0, (T)0};
    }
}

template <typename T>
__device__ void wg_zero(void* p, int64_t n_complex, int slot, int k) {
    using C = typename CT<T>::t;
    C* q = reinterpret_cast<C*>(p);
    for (int64_t i = (int64_t)slot * blockDim.x + threadIdx.x; i < n_complex; i += (int64_t)k * blockDim.x) q[i] = C{(T)0, (T)0};
}

// Iterate one item (all passes, then the FP64 reduction and loop control of
// k_reduce) until it stops at tol, max_iter or divergence.  st is the item's
// state in LDS; sig_base (nullable) is added to the mean stress.
template <typename T, int DIM, int WGS>
__device__ void batch_stage(const BatchItem& it, const RealArgs& ra, const AxisArgs* ax, const SpecArgs& sa,
                            int64_t t_real, int64_t t_spec, const int64_t* t_axis, LoadState& st,
                            const double* sig_base, double tol, int max_iter, int resid_period, bool record,
                            double* red, int slot, int& phase, int& rround, long long wait, double norm0) {
    constexpr int NC_ = Comp<DIM>::N;
    const int tid = threadIdx.x;
    const int k = it.k;
    for (;;) {
        double v[NC_ + 2];   // stress sums, residual sum, Cauchy sum
#pragma unroll
        for (int c = 0; c <= NC_ + 1; ++c) v[c] = 0.0;
        // the tiles of every pass are dealt round-robin to the group's workgroups
        for (int64_t t = slot; t < t_real; t += k) {
            real_tile<T, DIM, REAL_TURN>(ra, st, 0, t, v);
            __syncthreads();
        }
        group_sync(it, phase, wait);
        const int par = (st.iter + 1) & 1;
        for (int a = 1; a <= it.D - 2; ++a) {
            const int64_t nt = (int64_t)NC_ * t_axis[a];
            for (int64_t u = slot; u < nt; u += k) {
                axis_tile<T, -1>(ax[a], par, 0, (int)(u / t_axis[a]), u % t_axis[a]);
                __syncthreads();
            }
            group_sync(it, phase, wait);
        }
        for (int64_t t = slot; t < t_spec; t += k) {
            spec_tile<T, DIM, SPEC_TURN>(sa, st, 0, t, v[NC_], v[NC_ + 1]);
            __syncthreads();
        }
        group_sync(it, phase, wait);
        for (int a = it.D - 2; a >= 1; --a) {
            const int64_t nt = (int64_t)NC_ * t_axis[a];
            for (int64_t u = slot; u < nt; u += k) {
                axis_tile<T, +1>(ax[a], par, 0, (int)(u / t_axis[a]), u % t_axis[a]);
                __syncthreads();
            }
            group_sync(it, phase, wait);
        }
        block_sum<NC_ + 2, WGS>(v, red);
        if (k > 1) {
            // the group's partial sums, combined in slot order by every member
            double* gp = it.gpart + (rround & 1) * (k * 8);
            if (tid == 0)
                for (int c = 0; c <= NC_ + 1; ++c) gp[slot * 8 + c] = v[c];
            group_sync(it, phase, wait);
            if (tid == 0)
                for (int c = 0; c <= NC_ + 1; ++c) {
                    double acc = 0.0;
                    for (int s2 = 0; s2 < k; ++s2) acc += gp[s2 * 8 + c];
                    v[c] = acc;
                }
            ++rround;
        }
        if (tid == 0) {
            const double inv_m = 1.0 / (double)it.m;
            double fro = 0.0;
            for (int c = 0; c < NC_; ++c) {
                const double mc = v[c] * inv_m + (sig_base ? sig_base[c] : 0.0);
                st.mean[c] = mc;
                const bool diag = DIM == 3 ? c < 3 : c < 2;
                fro += (diag ? 1.0 : 2.0) * mc * mc;
            }
            const int n = st.iter;
            const bool rec = record && slot == 0;
            if (!ahom_check_iter(n, resid_period, max_iter)) {
                if (rec && n < it.hist_cap) {
                    it.hist[n] = -1.0;
                    it.chist[n] = -1.0;
                }
                st.iter = n + 1;
            } else {
                const double r = sqrt(v[NC_]) / sqrt(fro);
                if (rec && n < it.hist_cap) {
                    it.hist[n] = r;
                    // Cauchy measure |eps(n+1) - eps(n)| / |eps(0)|
                    it.chist[n] = sqrt((double)it.m * v[NC_ + 1] / (2.0 * sa.mu0 * sa.mu0)) / norm0;
                }
                if (n == 0) st.r0 = r;
                st.resid = r;
                const bool bad = !(r == r) || isinf(r) || (st.r0 > 0.0 && r > 1e3 * st.r0);
                if (bad) { st.done = 1; st.status = 2; st.final_buf = n & 1; }
                else if (r <= tol) { st.done = 1; st.status = 0; st.final_buf = n & 1; }
                else if (n >= max_iter) { st.done = 1; st.status = 1; st.final_buf = n & 1; }
                else st.iter = n + 1;
            }
            if (k > 1 && (__hip_atomic_load(it.gcount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kGroupAbort)) {
                st.done = 1;
                st.status = 3;   // group barrier timed out: result invalid
            }
        }
        __syncthreads();
        if (st.done) return;
    }
}

// |eps(0)| = sqrt(m) |eps_bar|_F of an item's load (the Cauchy denominator)
template <int DIM>
__device__ double item_norm0(const BatchItem& it) {
    constexpr int NC_ = Comp<DIM>::N;
    double nb = 0.0;
    for (int c = 0; c < NC_; ++c) {
        const bool diag = DIM == 3 ? c < 3 : c < 2;
        nb += (diag ? 1.0 : 2.0) * it.ra.eps_bar[c] * it.ra.eps_bar[c];
    }
    return sqrt((double)it.m * nb);
}

// Algorithm 1 on one item, one stage: from eps(0) = eps_bar to the item's
// stop (FP64 items; FP32 items without restarts) or to the first stage
// tolerance max(tol, refine) of an FP32 item with restarts; or (corr) the
// FP32 correction stage after a restart's FP64 step: e from 0 with the
// traction offset, mean stress = sbase + mean of the correction, to
// max(tol, refine x the restart's residual).  Then publish the state.  One
// call site of batch_stage serves both, so the kernel holds one copy of it.
template <typename T, int DIM, int WGS>
__device__ void batch_item(const BatchArgs& b, const BatchItem& it, int slot, LoadState& st, double* red, bool corr) {
    constexpr int NC_ = Comp<DIM>::N, NT = Comp<DIM>::NT;
    const int tid = threadIdx.x;
    const int k = it.k;
    int phase = 0, rround = 0;
    if (corr) {
        if (tid == 0) st = *it.st;
        __syncthreads();
        if (st.done) return;   // the same decision in every workgroup of the group
    } else {
        wg_fill_state<T>(it.ra.buf0, it.ra.eps_bar, it.S, it.row, NC_, slot, k);
        wg_zero<T>(it.sa.tbuf, (int64_t)NT * it.S, slot, k);
        if (tid == 0) st = LoadState{};
        group_sync(it, phase, b.group_wait);
    }
    const double norm0 = item_norm0<DIM>(it);
    const double stage_tol = corr ? fmax(b.tol, b.refine * st.resid) : b.refine_on ? fmax(b.tol, b.refine) : b.tol;
    batch_stage<T, DIM, WGS>(it, it.ra, it.ax, corr ? it.sa_corr : it.sa, it.t_real, it.t_spec, it.t_axis, st,
                        corr ? it.sbase : nullptr, stage_tol, b.max_iter, b.resid_period, true, red, slot, phase,
                        rround, b.group_wait, norm0);
    if (tid == 0 && slot == 0) {
        *it.st = st;
        if (!corr) *it.restarts = 0;
    }
}

// An FP32 item whose stage stopped at its stage tolerance above tol needs a
// defect-correction restart (the single-pattern solver's scheme).
__device__ __forceinline__ bool needs_restart(const BatchArgs& b, const LoadState& st) {
    return b.refine_on && st.done && st.status == 0 && st.resid > b.tol;
}

// The FP64 step of a restart: eps_h = (FP64 base, from the second restart on)
// + FP32 state, one FP64 update eps_b = F(eps_h) (its buffer is the next
// base) whose traction step d becomes the offset of the correction stage
// (written by the FP64 spectral pass), the FP32 state cleared for the
// correction e = eps - eps_b, and the loop control of the correction stage.
template <int DIM, int WGS>
__device__ void batch_restart64(const BatchArgs& b, const BatchItem& it, int slot, LoadState& st, LoadState& st64,
                                double* red) {
    constexpr int NC_ = Comp<DIM>::N, NT = Comp<DIM>::NT;
    const int tid = threadIdx.x;
    const int k = it.k;
    __shared__ int nres_s;
    if (tid == 0) {
        st = *it.st;
        nres_s = *it.restarts;
    }
    __syncthreads();
    if (!needs_restart(b, st)) return;   // the same decision in every workgroup of the group
    const int nres = nres_s;
    int phase = 0, rround = 0;
    {
        const float2* in = reinterpret_cast<const float2*>(st.final_buf ? it.ra.buf1 : it.ra.buf0);
        double2* out = reinterpret_cast<double2*>(it.ra64.buf0);
        const double2* base = nres ? reinterpret_cast<const double2*>(it.ra64.buf1) : nullptr;
        const int64_t n = (int64_t)NC_ * it.S;
        for (int64_t i = (int64_t)slot * blockDim.x + tid; i < n; i += (int64_t)k * blockDim.x) {
            const float2 x = in[i];
            double2 r = double2{(double)x.x, (double)x.y};
            if (base) { r.x += base[i].x; r.y += base[i].y; }
            out[i] = r;
        }
    }
    wg_zero<double>(it.sa64.tbuf, (int64_t)NT * it.S, slot, k);
    if (tid == 0) st64 = LoadState{};
    const double norm0 = item_norm0<DIM>(it);
    group_sync(it, phase, b.group_wait);
    batch_stage<double, DIM, WGS>(it, it.ra64, it.ax64, it.sa64, it.t_real64, it.t_spec64, it.t_axis64, st64, nullptr,
                             -1.0, 1, 1, false, red, slot, phase, rround, b.group_wait, norm0);
    // correction stage: e(0) = 0, t(e(-1)) = -d
    if (tid == 0) {
        LoadState ns{};
        ns.iter = st.iter + 1 < b.max_iter ? st.iter + 1 : b.max_iter;
        ns.r0 = st.r0;
        ns.resid = st64.resid;
        for (int c = 0; c < NC_; ++c) ns.mean[c] = st64.mean[c];
        ns.final_buf = ns.iter & 1;
        const double r = st64.resid;
        if (!(r == r) || isinf(r)) { ns.done = 1; ns.status = 2; }
        else if (r <= b.tol) { ns.done = 1; ns.status = 0; }
        else if (ns.iter >= b.max_iter) { ns.done = 1; ns.status = 1; }
        if (st64.status == 3) { ns.done = 1; ns.status = 3; }
        if (slot == 0 && ns.done && ns.iter < it.hist_cap) {
            it.hist[ns.iter] = r;
            it.chist[ns.iter] = -1.0;   // a restart's FP64 step: Cauchy measure not recorded
        }
        st = ns;
    }
    wg_zero<float>(it.ra.buf0, (int64_t)NC_ * it.S, slot, k);
    wg_zero<float>(it.ra.buf1, (int64_t)NC_ * it.S, slot, k);
    // every workgroup of the group has read the state above before slot 0 publishes the new one
    group_sync(it, phase, b.group_wait);
    if (tid == 0 && slot == 0) {
        for (int c = 0; c < NC_; ++c) it.sbase[c] = st.mean[c];
        *it.st = st;
        *it.restarts = nres + 1;
    }
}

// Persistent workgroups over the item queue.  KIND selects the work per item:
// BATCH_SOLVE (FP64 items, the whole solve), BATCH_FP32 (b.phase 0: the first
// FP32 stage, 1: a correction stage) or BATCH_RESTART64 (a restart's FP64
// step).  The FP32 solve is split over launches so that the FP32 kernel holds
// no FP64 tile code: its registers then allow 8 waves per CU, run as one
// workgroup of WGS = 512 threads whose tiles get the whole LDS budget.
template <int DIM, int KIND, int WGS>
__global__ void __launch_bounds__(WGS) k_batch(BatchArgs b) {
    constexpr int NC_ = Comp<DIM>::N;
    __shared__ double red[(NC_ + 2) * WGS];
    __shared__ LoadState st, st64;
    __shared__ int qi;
    for (;;) {
        if (threadIdx.x == 0) qi = atomicAdd(b.counter, 1);
        __syncthreads();
        const int q = qi;
        __syncthreads();
        if (q >= b.n_queue) return;
        const BatchItem& it = b.items[b.order[q]];
        const int slot = b.qslot[q];
        if constexpr (KIND == BATCH_SOLVE) {
            batch_item<double, DIM, WGS>(b, it, slot, st, red, false);
        } else if constexpr (KIND == BATCH_FP32) {
            batch_item<float, DIM, WGS>(b, it, slot, st, red, b.phase != 0);
        } else {
            batch_restart64<DIM, WGS>(b, it, slot, st, st64, red);
        }
        __syncthreads();
    }
}

__global__ void k_batch_reset(int* counter, int* gcount, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *counter = 0;
    if (i < n) gcount[i] = 0;
}

}  // namespace

int ahom_launch_batch_reset(int* counter, int* gcount, int n_items, hipStream_t s) {
    const int nb = n_items > 0 ? (n_items + 255) / 256 : 1;
    hipLaunchKernelGGL(k_batch_reset, dim3(nb), dim3(256), 0, s, counter, gcount, n_items);
    return AHOM_CHECK_LAUNCH();
}

size_t ahom_batch_static_lds(int dim, int wgs) {
    const int nc = dim == 3 ? 6 : 3;
    return (size_t)(nc + 2) * wgs * 8 + 2 * sizeof(LoadState) + 16;
}

namespace {
template <int DIM>
const void* batch_fn(int kind) {
    switch (kind) {
    case BATCH_SOLVE: return (const void*)k_batch<DIM, BATCH_SOLVE, AHOM_WG>;
    case BATCH_FP32: return (const void*)k_batch<DIM, BATCH_FP32, kBatchWg32>;
    default: return (const void*)k_batch<DIM, BATCH_RESTART64, AHOM_WG>;
    }
}
}  // namespace

int ahom_batch_wg_size(int kind) { return kind == BATCH_FP32 ? kBatchWg32 : AHOM_WG; }

int ahom_batch_occupancy(int kind, int dim, size_t lds) {
    int n = 0;
    const void* f = dim == 3 ? batch_fn<3>(kind) : batch_fn<2>(kind);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, ahom_batch_wg_size(kind), lds) == hipSuccess ? n : 0;
}

int ahom_launch_batch(int kind, int dim, const BatchArgs& a, int nwg, size_t lds, hipStream_t s) {
    const int wgs = ahom_batch_wg_size(kind);
    const void* f = dim == 3 ? batch_fn<3>(kind) : batch_fn<2>(kind);
    BatchArgs arg = a;
    void* params[] = {&arg};
    if (hipLaunchKernel(f, dim3(nwg), dim3(wgs), params, lds, s) != hipSuccess) return -1;
    return AHOM_CHECK_LAUNCH();
}

// =============================================================================
// helpers: state initialisation and DFT reordering
// =============================================================================
template <typename T>
__global__ void k_fill_state(FillArgs a) {
    using C = typename CT<T>::t;
    const int load = blockIdx.y;
    const int f = blockIdx.z;
    C* buf = reinterpret_cast<C*>(a.buf) + ((int64_t)load * a.nfield + f) * a.S;
    const double v = a.eps_bar[(int64_t)load * a.nfield + f];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.S; i += (int64_t)gridDim.x * blockDim.x)
        buf[i] = i < a.row ? C{(T)v, (T)0} : C{(T)0, (T)0};
}

__global__ void k_reset_states(LoadState* st, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        LoadState s{};
        st[i] = s;
    }
}

template <typename T>
__global__ void k_zero(T* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = (T)0;
}

// defect-correction restart: FP64 state = FP64 base + FP32 correction
__global__ void k_refine_gather(GatherArgs a) {
    const int load = blockIdx.y;
    const float2* in = (a.st[load].final_buf ? a.in1 : a.in0) + (int64_t)load * a.per_load;
    double2* out = a.out + (int64_t)load * a.per_load;
    const double2* base = a.base ? a.base + (int64_t)load * a.per_load : nullptr;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.per_load; i += (int64_t)gridDim.x * blockDim.x) {
        const float2 v = in[i];
        double2 r = double2{(double)v.x, (double)v.y};
        if (base) { const double2 b = base[i]; r.x += b.x; r.y += b.y; }
        out[i] = r;
    }
}

// kernel order position <-> canonical kappa order; dir = 0 gather to canonical
// (out[canon] = in[pos] * scale), dir = 1 scatter from canonical.
template <typename T>
__global__ void k_reorder(ReorderArgs a) {
    using C = typename CT<T>::t;
    const Plan& P = *a.plan;
    const C* in = reinterpret_cast<const C*>(a.in);
    C* out = reinterpret_cast<C*>(a.out);
    for (int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pos < P.m; pos += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = pos, kap[3] = {0, 0, 0};
        for (int b = P.D - 1; b >= 0; --b) {
            const int64_t k = r % P.ax[b].len;
            r /= P.ax[b].len;
            kap[P.ax[b].snf] += P.ax[b].mult * k;
        }
        int64_t canon = 0;
        for (int s = 0; s < P.d; ++s) canon += kap[s] * P.canon_stride[s];
        if (a.dir == 0) {
            C v = in[pos];
            out[canon] = C{v.x * (decltype(v.x))a.scale, v.y * (decltype(v.x))a.scale};
        } else {
            out[pos] = in[canon];
        }
    }
}

// ----------------------------------------------------------------- launchers

template <typename T>
static int set_lds(const void* fn, size_t bytes) {
    if (bytes > 64 * 1024)
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
    return 0;
}

int ahom_launch_real(int prec, int dim, int mode, const RealArgs& a, int nwg, int nload, size_t lds, hipStream_t s) {
    dim3 grid(nwg, nload), block(AHOM_WG);
#define AHOM_REAL(T, D, M)                                                             \
    do {                                                                               \
        auto fn = a.phys == PHYS_THERMAL ? k_real<T, D, M, PHYS_THERMAL> : k_real<T, D, M, PHYS_ELASTIC>; \
        if (set_lds<T>((const void*)fn, lds)) return -1;                               \
        hipLaunchKernelGGL(fn, grid, block, lds, s, a);                                \
    } while (0)
#define AHOM_REAL_M(T, D)                                                              \
    do {                                                                               \
        if (mode == REAL_TURN) AHOM_REAL(T, D, REAL_TURN);                             \
        else if (mode == REAL_TO_REAL) AHOM_REAL(T, D, REAL_TO_REAL);                  \
        else AHOM_REAL(T, D, REAL_FROM_REAL);                                          \
    } while (0)
    if (prec == 0) { if (dim == 3) AHOM_REAL_M(double, 3); else AHOM_REAL_M(double, 2); }
    else { if (dim == 3) AHOM_REAL_M(float, 3); else AHOM_REAL_M(float, 2); }
    return AHOM_CHECK_LAUNCH();
}

int ahom_launch_axis(int prec, int dir, const AxisArgs& a, int nwg, int nfield, int nload, size_t lds, hipStream_t s) {
    dim3 grid(nwg, nfield, nload), block(AHOM_WG);
#define AHOM_AXIS(T, DIR)                                                              \
    do {                                                                               \
        auto fn = k_axis<T, DIR>;                                                      \
        if (set_lds<T>((const void*)fn, lds)) return -1;                               \
        hipLaunchKernelGGL(fn, grid, block, lds, s, a);                                \
    } while (0)
    if (prec == 0) { if (dir < 0) AHOM_AXIS(double, -1); else AHOM_AXIS(double, 1); }
    else { if (dir < 0) AHOM_AXIS(float, -1); else AHOM_AXIS(float, 1); }
    return AHOM_CHECK_LAUNCH();
}

#define AHOM_SPEC(T, D, M)                                                             \
    do {                                                                               \
        auto fn = a.phys == PHYS_THERMAL ? k_spec<T, D, M, PHYS_THERMAL> : k_spec<T, D, M, PHYS_ELASTIC>; \
        if (set_lds<T>((const void*)fn, lds)) return -1;                               \
        hipLaunchKernelGGL(fn, grid, block, lds, s, a);                                \
    } while (0)
int ahom_launch_spec(int prec, int dim, const SpecArgs& a, int nwg, int nload, size_t lds, hipStream_t s) {
    dim3 grid(nwg, nload), block(AHOM_WG);
    if (prec == 0) { if (dim == 3) AHOM_SPEC(double, 3, SPEC_TURN); else AHOM_SPEC(double, 2, SPEC_TURN); }
    else { if (dim == 3) AHOM_SPEC(float, 3, SPEC_TURN); else AHOM_SPEC(float, 2, SPEC_TURN); }
    return AHOM_CHECK_LAUNCH();
}

int ahom_launch_spec_init(int prec, int dim, const SpecArgs& a, int nwg, int nload, size_t lds, hipStream_t s) {
    dim3 grid(nwg, nload), block(AHOM_WG);
    if (prec == 0) { if (dim == 3) AHOM_SPEC(double, 3, SPEC_INIT); else AHOM_SPEC(double, 2, SPEC_INIT); }
    else { if (dim == 3) AHOM_SPEC(float, 3, SPEC_INIT); else AHOM_SPEC(float, 2, SPEC_INIT); }
    return AHOM_CHECK_LAUNCH();
}

int ahom_launch_reduce(int dim, const ReduceArgs& a, int nload, hipStream_t s) {
    auto fn = a.phys == PHYS_THERMAL ? (dim == 3 ? k_reduce<3, PHYS_THERMAL> : k_reduce<2, PHYS_THERMAL>)
                                     : (dim == 3 ? k_reduce<3, PHYS_ELASTIC> : k_reduce<2, PHYS_ELASTIC>);
    hipLaunchKernelGGL(fn, dim3(nload), dim3(AHOM_WG), 0, s, a);
    return AHOM_CHECK_LAUNCH();
}

int ahom_launch_fill(int prec, const FillArgs& a, int nload, hipStream_t s) {
    int64_t blocks = (a.S + AHOM_WG - 1) / AHOM_WG;
    if (blocks > 4096) blocks = 4096;
    dim3 grid((unsigned)blocks, nload, a.nfield);
    if (prec == 0) hipLaunchKernelGGL(k_fill_state<double>, grid, dim3(AHOM_WG), 0, s, a);
    else hipLaunchKernelGGL(k_fill_state<float>, grid, dim3(AHOM_WG), 0, s, a);
    return AHOM_CHECK_LAUNCH();
}

int ahom_launch_reset(LoadState* st, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_states, dim3((n + 63) / 64), dim3(64), 0, s, st, n);
    return AHOM_CHECK_LAUNCH();
}

int ahom_launch_zero(int prec, void* p, int64_t n_complex, hipStream_t s) {
    int64_t n = 2 * n_complex;
    int64_t blocks = (n + AHOM_WG - 1) / AHOM_WG;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    if (prec == 0) hipLaunchKernelGGL(k_zero<double>, dim3((unsigned)blocks), dim3(AHOM_WG), 0, s, (double*)p, n);
    else hipLaunchKernelGGL(k_zero<float>, dim3((unsigned)blocks), dim3(AHOM_WG), 0, s, (float*)p, n);
    return AHOM_CHECK_LAUNCH();
}

int ahom_launch_refine_gather(const GatherArgs& a, int nload, hipStream_t s) {
    int64_t blocks = (a.per_load + AHOM_WG - 1) / AHOM_WG;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_refine_gather, dim3((unsigned)blocks, nload), dim3(AHOM_WG), 0, s, a);
    return AHOM_CHECK_LAUNCH();
}

int ahom_launch_reorder(int prec, const ReorderArgs& a, int64_t m, hipStream_t s) {
    int64_t blocks = (m + AHOM_WG - 1) / AHOM_WG;
    if (blocks > 4096) blocks = 4096;
    if (prec == 0) hipLaunchKernelGGL(k_reorder<double>, dim3((unsigned)blocks), dim3(AHOM_WG), 0, s, a);
    else hipLaunchKernelGGL(k_reorder<float>, dim3((unsigned)blocks), dim3(AHOM_WG), 0, s, a);
    return AHOM_CHECK_LAUNCH();
}

template <typename E>
__global__ void k_transpose(const E* __restrict__ src, E* __restrict__ dst, int64_t L0, int64_t I) {
    const int64_t n_all = L0 * I;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_all; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i / L0, n = i - c * L0;
        dst[i] = src[n * I + c];
    }
}

int ahom_launch_transpose(const void* src, void* dst, int64_t L0, int64_t I, int bytes, hipStream_t s) {
    int64_t blocks = (L0 * I + AHOM_WG - 1) / AHOM_WG;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    if (bytes == 1)
        hipLaunchKernelGGL(k_transpose<uint8_t>, dim3((unsigned)blocks), dim3(AHOM_WG), 0, s, (const uint8_t*)src, (uint8_t*)dst, L0, I);
    else
        hipLaunchKernelGGL(k_transpose<double2>, dim3((unsigned)blocks), dim3(AHOM_WG), 0, s, (const double2*)src, (double2*)dst, L0, I);
    return AHOM_CHECK_LAUNCH();
}
