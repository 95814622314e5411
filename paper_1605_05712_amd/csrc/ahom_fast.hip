// Pass kernels specialised on a power-of-two transform length L <= 256.
//
// Same passes and data layout as the generic kernels (ahom_kernels.hip); the
// 1-D FFT of each column is a two-level factorisation L = N1 * N2 held in
// registers: thread tau < N1 of a column takes the N2 samples
// x[tau + N1 q], does a radix-N2 DFT, multiplies by W_L^{tau k_a}, exchanges
// through LDS once and finishes with N2/N1 radix-N1 DFTs, giving
// X[k_a + N2 k_b].  All index arithmetic is compile-time.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>

#include "ahom_internal.h"
#include "ahom_kernels.h"

namespace {

// plain aggregates (not HIP vector types) so that register arrays of them are
// promoted out of scratch; same layout as double2 / float2
struct alignas(16) cplx64 { double x, y; };
struct alignas(8) cplx32 { float x, y; };
template <typename T> struct CT;
template <> struct CT<double> { using t = cplx64; };
template <> struct CT<float> { using t = cplx32; };

// global-memory element access through native 2-vectors (one 16 B / 8 B
// access, and no aggregate copy that would pin register arrays to scratch)
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cplx64 ldg(const cplx64* p) {
    const v2d v = *reinterpret_cast<const v2d*>(p);
    return cplx64{v.x, v.y};
}
__device__ __forceinline__ cplx32 ldg(const cplx32* p) {
    const v2f v = *reinterpret_cast<const v2f*>(p);
    return cplx32{v.x, v.y};
}
__device__ __forceinline__ void stg(cplx64* p, cplx64 c) {
    v2d v;
    v.x = c.x;
    v.y = c.y;
    *reinterpret_cast<v2d*>(p) = v;
}
__device__ __forceinline__ void stg(cplx32* p, cplx32 c) {
    v2f v;
    v.x = c.x;
    v.y = c.y;
    *reinterpret_cast<v2f*>(p) = v;
}

// compile-time loop: f(std::integral_constant<int, i>) for i in [B, E).  Array
// indices in the body are constants from the start, so register arrays are
// split into scalars before any alloca promotion decision.
template <int B, int E, typename F> __device__ __forceinline__ void sfor(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) { return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) { return C{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }

// cos / sin of 2 pi j / 16
constexpr double kC16[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                             0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                             -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                             0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
constexpr double kS16[16] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                             1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                             0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                             -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

// v * W_16^j with W_16 = exp(DIR 2 pi i / 16)
template <int DIR, int J, typename C> __device__ __forceinline__ C tw16(C v) {
    using T = decltype(C{}.x);
    constexpr int j = J % 16;
    if constexpr (j == 0) return v;
    else if constexpr (j == 4) return DIR < 0 ? C{v.y, -v.x} : C{-v.y, v.x};
    else if constexpr (j == 8) return C{-v.x, -v.y};
    else if constexpr (j == 12) return DIR < 0 ? C{-v.y, v.x} : C{v.y, -v.x};
    else {
        const T c = (T)kC16[j], s = (T)(DIR < 0 ? -kS16[j] : kS16[j]);
        return C{v.x * c - v.y * s, v.x * s + v.y * c};
    }
}

// in-place DFT of N = 1, 2, 4, 8, 16 points, natural order in and out
template <int N, int DIR, typename C> __device__ __forceinline__ void dft(C* v) {
    if constexpr (N == 2) {
        C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (N == 4) {
        C a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
        C c = cadd(v[1], v[3]), d = tw16<DIR, 4>(csub(v[1], v[3]));
        v[0] = cadd(a, c);
        v[2] = csub(a, c);
        v[1] = cadd(b, d);
        v[3] = csub(b, d);
    } else if constexpr (N == 8) {
        C e[4] = {v[0], v[2], v[4], v[6]};
        C o[4] = {v[1], v[3], v[5], v[7]};
        dft<4, DIR>(e);
        dft<4, DIR>(o);
        o[1] = tw16<DIR, 2>(o[1]);
        o[2] = tw16<DIR, 4>(o[2]);
        o[3] = tw16<DIR, 6>(o[3]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = cadd(e[k], o[k]);
            v[k + 4] = csub(e[k], o[k]);
        }
    } else if constexpr (N == 16) {
        // n = n1 + 4 n2, k = k2 + 4 k1
        C a[4][4];
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) {
#pragma unroll
            for (int n2 = 0; n2 < 4; ++n2) a[n1][n2] = v[n1 + 4 * n2];
            dft<4, DIR>(a[n1]);
        }
        a[1][1] = tw16<DIR, 1>(a[1][1]); a[1][2] = tw16<DIR, 2>(a[1][2]); a[1][3] = tw16<DIR, 3>(a[1][3]);
        a[2][1] = tw16<DIR, 2>(a[2][1]); a[2][2] = tw16<DIR, 4>(a[2][2]); a[2][3] = tw16<DIR, 6>(a[2][3]);
        a[3][1] = tw16<DIR, 3>(a[3][1]); a[3][2] = tw16<DIR, 6>(a[3][2]); a[3][3] = tw16<DIR, 9>(a[3][3]);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
            C t[4] = {a[0][k2], a[1][k2], a[2][k2], a[3][k2]};
            dft<4, DIR>(t);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) v[k2 + 4 * k1] = t[k1];
        }
    }
}

template <int L> struct Split {
    static constexpr int N2 = L >= 128 ? 16 : (L >= 32 ? 8 : L);
    static constexpr int N1 = L / N2;
    static_assert(N1 * N2 == L && (N1 == 1 || N2 % N1 == 0), "unsupported length");
};

constexpr int pow2floor(int v) {
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}

// columns per workgroup: NF fields x NC columns x N1 threads <= 512 threads,
// NF x NC x CS elements <= 50 KB of LDS (CS: column stride, see below)
// Tile variants V (chosen per pass by the autotuner): bit 0 halves the
// columns per tile, bit 1 selects the persistent prefetching schedule.
template <typename T, int L, int NF, int V = 0> struct Geo {
    static constexpr int es = 2 * (int)sizeof(T);
    static constexpr int N1 = Split<L>::N1;
    static constexpr int GL = 128 / es;  // elements per 128 B LDS line
    static constexpr int CS = L >= GL ? L : L + 1;  // line-aligned columns (swizzled, see lsw)
    static constexpr int by_lds = (50 * 1024) / (NF * CS * es);
    static constexpr int by_thr = 512 / (NF * N1);
    static constexpr int NCMAX = pow2floor((by_lds < by_thr ? by_lds : by_thr) < 1 ? 1 : (by_lds < by_thr ? by_lds : by_thr));
    // V = 4 (spectral pass only): quarter-width tiles, one per workgroup
    static constexpr int NC = V == 4 ? (NCMAX >= 4 ? NCMAX / 4 : 1) : ((V & 1) && NCMAX > 1 ? NCMAX / 2 : NCMAX);
    static constexpr bool PERSIST = (V & 2) != 0;
    static constexpr int THREADS = ((NF * NC * N1 + 63) / 64) * 64;
    static constexpr int TILE = NF * NC * CS;  // complex elements of LDS tile
};

// XOR mask of the element index inside LDS tile column `col`.  Columns are
// unpadded, so every column starts on a 128 B line and a lane group that
// sweeps N1 consecutive elements of one column stays inside one line; the
// mask makes the GL consecutive columns that lanes read row by row (loads,
// stores, pack/unpack) hit distinct banks, and places the columns that share
// one GL-lane group in the FFT stages (GL / N1 of them) in disjoint quarters.
template <int L, typename C> __device__ __forceinline__ int lsw(int col) {
    constexpr int GL = 128 / (int)sizeof(C);
    if constexpr (L < GL) {
        return 0;
    } else {
        constexpr int N1 = Split<L>::N1;
        constexpr int P = N1 >= GL ? 1 : GL / N1;
        constexpr int Q = GL / P;
        return ((col % P) * (N1 >= GL ? 1 : N1)) | ((col / P) % Q);
    }
}

// LDS stores of this wave visible to its later loads (no other wave involved)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// FFT of `ncols` columns (stride CS) of an LDS tile in place.  twl holds the
// inter-stage twiddles as twl[ka * N1 + tau] = W_L^{tau ka}.  The exchange
// between the stages stores row r, entry c at r * N1 + (c ^ (r % N1)) so that
// the N1 threads of a column touch distinct LDS banks in both stages.  The N1
// threads of a column lie in one wavefront (N1 divides 64), so the exchange
// only needs wave-level ordering; one workgroup barrier at the end hands the
// transformed tile to the next stage.
template <int L, int DIR, int CS, typename C>
__device__ __forceinline__ void fft_cols(C* lds, int ncols, const C* twl, int s = threadIdx.x) {
    constexpr int N1 = Split<L>::N1, N2 = Split<L>::N2;
    const int col = s / N1, tau = s % N1;
    const bool act = col < ncols;
    C* base = lds + col * CS;
    const int sz = lsw<L, C>(col);
    C v[N2];
    if constexpr (N1 == 1) {
        if (act) {
#pragma unroll
            for (int q = 0; q < N2; ++q) v[q] = base[q ^ sz];
            dft<N2, DIR>(v);
#pragma unroll
            for (int q = 0; q < N2; ++q) base[q ^ sz] = v[q];
        }
        __syncthreads();
        return;
    } else {
        if (act) {
#pragma unroll
            for (int q = 0; q < N2; ++q) v[q] = base[(tau + N1 * q) ^ sz];
        }
        wave_lds_sync();
        if (act) {
            dft<N2, DIR>(v);
#pragma unroll
            for (int ka = 1; ka < N2; ++ka) {
                const C w = twl[ka * N1 + tau];
                v[ka] = DIR < 0 ? cmul(v[ka], w) : cmulc(v[ka], w);
            }
#pragma unroll
            for (int ka = 0; ka < N2; ++ka) base[(ka * N1 + (tau ^ (ka & (N1 - 1)))) ^ sz] = v[ka];
        }
        wave_lds_sync();
        constexpr int B = N2 / N1;
        if (act) {
#pragma unroll
            for (int b = 0; b < B; ++b)
#pragma unroll
                for (int t = 0; t < N1; ++t) v[b * N1 + t] = base[((tau + N1 * b) * N1 + (t ^ tau)) ^ sz];
        }
        wave_lds_sync();
        if (act) {
#pragma unroll
            for (int b = 0; b < B; ++b) {
                dft<N1, DIR>(v + b * N1);
#pragma unroll
                for (int kb = 0; kb < N1; ++kb) base[(tau + N1 * b + N2 * kb) ^ sz] = v[b * N1 + kb];
            }
        }
        __syncthreads();
    }
}

// inter-stage twiddles twl[ka * N1 + tau] = W_L^{tau ka} from the table tw[j] = W_L^j
template <int L, typename C>
__device__ __forceinline__ void load_twiddles(C* twl, const C* tw) {
    constexpr int N1 = Split<L>::N1;
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        const int ka = j / N1, tau = j % N1;
        twl[j] = tw[ka * tau];
    }
}

// The same table staged in two steps: loads into registers first, the LDS
// stores once the tile's own loads are in flight, so that the two memory
// latencies overlap instead of adding up.  Loads are unconditional (clamped
// index) so later waits stay exact.
template <int L, int TH, typename C> struct Twiddles {
    static constexpr int N = (L + TH - 1) / TH;
    C v[N];
    __device__ __forceinline__ void load(const C* tw, int tid) {
        constexpr int N1 = Split<L>::N1;
        sfor<0, N>([&](auto ic) __attribute__((always_inline)) {
            constexpr int i = ic;
            const int j = tid + i * TH < L ? tid + i * TH : 0;
            v[i] = ldg(tw + (j / N1) * (j % N1));
        });
    }
    __device__ __forceinline__ void store(C* twl, int tid) const {
        sfor<0, N>([&](auto ic) __attribute__((always_inline)) {
            constexpr int i = ic;
            if (tid + i * TH < L) twl[tid + i * TH] = v[i];
        });
    }
};

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

__device__ __forceinline__ double2 split_tw64(const AxisDesc& ax, const double2* __restrict__ tw64, int64_t j) {
    int64_t hi, lo;
    divmod_fast(j, ax.spB, hi, lo);
    const double2 a = tw64[ax.sp_off1 + lo];
    const double2 b = tw64[ax.sp_off2 + hi];
    return cmul(a, b);
}

template <typename C>
__device__ __forceinline__ C split_twiddle(const AxisDesc& ax, const double2* __restrict__ tw64, int64_t j) {
    const double2 w = split_tw64(ax, tw64, j);
    using T = decltype(C{}.x);
    return C{(T)w.x, (T)w.y};
}

// Four-step twiddles W^(Q l) along the positions l = l0, l0 + dl, ... that
// one thread visits in a column of fixed Q: the first one and the step from
// the two-level FP64 table, then a running FP64 product (one complex
// multiply per element instead of two table reads and an index division;
// the rounding grows by ~1e-16 per step over at most a few tens of steps).
struct TwiddleWalk {
    double2 w, step;
    __device__ __forceinline__ void start(const AxisDesc& ax, const double2* __restrict__ tw64, int64_t Q, int64_t l0,
                                          int64_t dl) {
        w = split_tw64(ax, tw64, Q * l0);
        step = split_tw64(ax, tw64, Q * dl);
    }
    // the twiddle of the current position, then advance
    template <typename C> __device__ __forceinline__ C next() {
        using T = decltype(C{}.x);
        const C out = C{(T)w.x, (T)w.y};
        w = cmul(w, step);
        return out;
    }
};

template <int DIM, int PH = PHYS_ELASTIC> using Comp = Fields<DIM, PH>;

template <typename T> __device__ __forceinline__ T* smem() {
    extern __shared__ __align__(16) unsigned char ahom_fast_smem[];
    return reinterpret_cast<T*>(ahom_fast_smem);
}

// Fixed-order sum of a double over the 64 lanes of a wavefront with DPP lane
// moves (VALU only, no LDS round trip): pairs, quads, half rows and rows by
// mirrors, then rows 0+1 and 2+3 by the row-15 broadcast and all four by the
// lane-31 broadcast.  The total is in lane 63.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_step(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
    return v + __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_sum_lane63(double v) {
    v = dpp_step<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
    v = dpp_step<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
    v = dpp_step<0x141, 0xf>(v);   // row_half_mirror
    v = dpp_step<0x140, 0xf>(v);   // row_mirror
    v = dpp_step<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_step<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    return v;
}

// Tile of schedule slot t (of n).  Workgroups are dealt to the 8 XCDs
// round-robin (slot t runs on XCD t % 8); give each XCD a contiguous range of
// tiles, so that tiles sharing HBM lines (neighbouring column blocks) meet in
// the same L2.  A bijection of [0, n).
__device__ __forceinline__ int64_t xcd_tile(int64_t t, int64_t n) {
    const int64_t per = n >> 3, rem = n & 7;
    const int64_t x = t & 7, i = t >> 3;
    return x * per + (x < rem ? x : rem) + i;
}

// Self-conjugate class test 2 kappa = 0 (mod e) per Smith axis.  The pass
// kernels enumerate reduced indices 0 <= kappa_s < e_s, for which the test is
// 2 kappa_s in {0, e_s}: no 64-bit division (kept as a fallback otherwise).
__device__ __forceinline__ bool self_conjugate(const FreqMap& f, const int64_t* kap, int dim) {
    bool ok = true;
    for (int s = 0; s < dim; ++s) {
        const int64_t k2 = 2 * kap[s], e = f.e[s];
        if (kap[s] >= 0 && kap[s] < e) ok = ok && (k2 == 0 || k2 == e);
        else ok = ok && (k2 % e == 0);
    }
    return ok;
}

// exact (A kappa) mod emax, centred; double path while products stay below 2^53
__device__ __forceinline__ int centred_numerators(const FreqMap& f, const int64_t* kap, int64_t* N, int dim) {
    int half = 0;
    const double inv = 1.0 / (double)f.emax;
    const double e = (double)f.emax;
    for (int i = 0; i < dim; ++i) {
        int64_t r;
        if (f.emax <= (int64_t(1) << 24)) {
            double x = 0.0;
            for (int s = 0; s < dim; ++s) x += (double)f.A[i][s] * (double)kap[s];
            double q = floor(x * inv);
            double rr = x - q * e;
            if (rr < 0) rr += e;
            if (rr >= e) rr -= e;
            r = (int64_t)rr;
        } else {
            r = 0;
            for (int s = 0; s < dim; ++s) r = (r + (f.A[i][s] % f.emax) * kap[s]) % f.emax;
        }
        if (2 * r >= f.emax) r -= f.emax;
        if (2 * r == -f.emax) half = 1;
        N[i] = r;
    }
    return half;
}

}  // namespace


// Work distribution of the pass kernels below: one tile per workgroup
// (variants 0/1), or a persistent grid that walks the tiles t = blockIdx.x,
// blockIdx.x + gridDim.x, ... with the next tile's loads in flight into
// registers (pre[]) while tile t is transformed (variants 2/3).  Tiles of
// load cases that have stopped are skipped.  Partial sums are written per
// (load, tile) and reduced in a fixed order.

// Value of a wave-uniform quantity kept in a scalar register, so that the
// loads it addresses (load states, plan fields) are scalar loads and never
// enter the vector-memory wait counter.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// =============================================================================
// real-space turnaround along axis 0
//
// Variants 0/1 run one tile per workgroup.  The persistent variants (2/3) run
// a software pipeline over the workgroup's tiles: while tile t is in its
// transforms and local law (LDS and registers only), the loads of tile t+1
// and the stores of tile t-1 are in flight.  A wave's counter of outstanding
// vector-memory operations covers loads and stores alike, and with both kinds
// in flight any wait on one of them waits for all; so nothing waits on global
// memory between the packing of a tile and the next packing: the law reads
// its Lame pairs from a copy of the phase table in LDS, and the stress sums
// go through LDS.  (Per-point Lame fields are read in the law directly: a
// slower path.)
// =============================================================================
template <typename T, int DIM, int L, int V, int PH>
__global__ void __launch_bounds__((Geo<T, L, Comp<DIM, PH>::NP, V>::THREADS)) kf_real(RealArgs a) {
    using C = typename CT<T>::t;
    constexpr int NCOMP = Comp<DIM, PH>::N, NP = Comp<DIM, PH>::NP;
    using G = Geo<T, L, NP, V>;
    constexpr int NC = G::NC, CS = G::CS, H = L / 2 + 1, TH = G::THREADS, NW = TH / 64;
    constexpr int EPT = (H * NC + TH - 1) / TH;     // half-spectrum rows per thread
    constexpr int EPL = (L * NC + TH - 1) / TH;     // law points per thread
    constexpr int TWT = (L + TH - 1) / TH;          // twiddles per thread
    constexpr int MTT = (2 * 256 + TH - 1) / TH;    // phase-table entries per thread (<= 256 phases)
    const Plan& P = *a.plan;
    const AxisDesc& ax = P.ax[0];
    const int64_t I = P.S / H;
    const int64_t nct = (I + NC - 1) / NC;
    const int64_t total = nct * a.nload;
    int tid = threadIdx.x;
    const int wave = tid >> 6;
    C* Z = smem<C>();
    C* twl = Z + G::TILE;
    double* red = reinterpret_cast<double*>(twl + L);   // [NCOMP + 1][NW] per-wave stress (and energy) sums
    T* mat = reinterpret_cast<T*>(red + (NCOMP + 1) * NW);   // [n_phase][2] Lame pairs
    const bool table = a.lame_pts_t == nullptr;
    const T lam0 = (T)a.lam0, mu0 = (T)a.mu0;

    // twiddles and phase table: loaded into registers, written to LDS once
    C twv[TWT];
    T mtv[MTT];
    auto load_tables = [&]() __attribute__((always_inline)) {
        const C* tw = reinterpret_cast<const C*>(a.tw) + ax.tw_off;
        sfor<0, TWT>([&](auto ic) __attribute__((always_inline)) {
            constexpr int i = ic;
            const int j = tid + i * TH < L ? tid + i * TH : 0;
            twv[i] = ldg(tw + (j / Split<L>::N1) * (j % Split<L>::N1));
        });
        if (table) {
            sfor<0, MTT>([&](auto ic) __attribute__((always_inline)) {
                constexpr int i = ic;
                const int j = tid + i * TH < 2 * a.n_phase ? tid + i * TH : 0;
                mtv[i] = (T)a.lame_tab[j];
            });
        }
    };
    auto store_tables = [&]() __attribute__((always_inline)) {
        sfor<0, TWT>([&](auto ic) __attribute__((always_inline)) {
            constexpr int i = ic;
            if (tid + i * TH < L) twl[tid + i * TH] = twv[i];
        });
        if (table) {
            sfor<0, MTT>([&](auto ic) __attribute__((always_inline)) {
                constexpr int i = ic;
                if (tid + i * TH < 2 * a.n_phase) mat[tid + i * TH] = mtv[i];
            });
        }
    };

    // A tile: load case, first column, columns, buffer parity of the iterate.
    struct Tile { int load, ncol, par; int64_t c0, ct; };
    auto tile_of = [&](int64_t t) __attribute__((always_inline)) -> Tile {
        Tile x;
        x.load = uni((int)(t / nct));
        x.ct = uni(t % nct);
        x.c0 = x.ct * NC;
        x.ncol = (int)((I - x.c0) < NC ? (I - x.c0) : NC);
        x.par = a.st[x.load].iter & 1;
        return x;
    };

    // Loads of a tile, phase ids first, then the spectra.  All loads are
    // issued unconditionally, out-of-tile slots clamped to an in-bounds
    // address (values unused), so the compiler's waits stay exact.
    C pre[EPT][NCOMP];
    uint8_t phq[EPL];
    auto fetch_loads = [&](const Tile& x) __attribute__((always_inline)) {
        if (table) {
            sfor<0, EPL>([&](auto qc) __attribute__((always_inline)) {
                constexpr int q = qc;
                const int e = tid + q * TH;
                const int j = e / L, n = e % L;
                const bool ok = e < L * NC && j < x.ncol;
                phq[q] = a.phase_t[ok ? (x.c0 + j) * (int64_t)L + n : x.c0 * (int64_t)L];
            });
        }
        // per field a uniform base and one 32-bit byte offset per slot (the
        // scalar-base addressing form: no 64-bit address per load)
        const C* src = reinterpret_cast<const C*>(x.par ? a.buf1 : a.buf0) + (int64_t)x.load * NCOMP * P.S;
        sfor<0, EPT>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = qc;
            const int e = tid + q * TH;
            const int k = e < H * NC ? e / NC : H - 1;
            const int j = e % NC < x.ncol ? e % NC : 0;
            const uint32_t off = (uint32_t)(((int64_t)k * I + x.c0 + j) * (int64_t)sizeof(C));
            sfor<0, NCOMP>([&](auto fc) __attribute__((always_inline)) {
                constexpr int f = fc;
                pre[q][f] = ldg(reinterpret_cast<const C*>(reinterpret_cast<const char*>(src + (int64_t)f * P.S) + off));
            });
        });
    };

    // packed full spectra Z_p = A + i B from the half spectra in pre[]
    // thread tid visits column j = tid % NC at rows k = tid / NC + q TH / NC
    static_assert(TH % NC == 0, "a thread keeps its column");
    TwiddleWalk walk;
    auto pack = [&](const Tile& x) __attribute__((always_inline)) {
        if (ax.split) walk.start(ax, a.tw64, div_fast(x.c0 + tid % NC, ax.qdiv), tid / NC, TH / NC);
        sfor<0, EPT>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = qc;
            const int e = tid + q * TH;
            const int k = e / NC, j = e % NC;
            C w = C{(T)1, (T)0};
            if (ax.split) w = walk.next<C>();
            if (e >= H * NC || j >= x.ncol) return;
            sfor<0, NP>([&](auto pc) __attribute__((always_inline)) {
                constexpr int p = pc;
                C A = pre[q][2 * p];
                C B = C{(T)0, (T)0};
                if constexpr (2 * p + 1 < NCOMP) B = pre[q][2 * p + 1];
                if (ax.split) { A = cmulc(A, w); B = cmulc(B, w); }
                if (k == 0 || 2 * k == L) { A.y = 0; B.y = 0; }
                C* Zp = Z + (p * NC + j) * CS;
                const int sz = lsw<L, C>(p * NC + j);
                Zp[k ^ sz] = C{A.x - B.y, A.y + B.x};
                if (k > 0 && 2 * k != L) Zp[(L - k) ^ sz] = C{A.x + B.y, B.x - A.y};
            });
        });
    };

    // local law on the tile in LDS; per-wave stress sums into red[] (and,
    // with a.en_part set, the sums of eps : tau)
    const bool energy = a.en_part != nullptr;
    auto law = [&](const Tile& x, const uint8_t (&ph)[EPL]) __attribute__((always_inline)) {
        double sig[NCOMP];
        double en = 0.0;
#pragma unroll
        for (int c = 0; c < NCOMP; ++c) sig[c] = 0.0;
        auto point = [&](int j, int n, T lam, T mu) __attribute__((always_inline)) {
            T eps[NCOMP];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const C z = Z[(p * NC + j) * CS + (n ^ lsw<L, C>(p * NC + j))];
                eps[2 * p] = z.x;
                if (2 * p + 1 < NCOMP) eps[2 * p + 1] = z.y;
            }
            T tau[NCOMP];
            if constexpr (PH == PHYS_THERMAL) {
                // flux q = k e, polarization (k - k0) e; k in the lambda slot
#pragma unroll
                for (int c = 0; c < NCOMP; ++c) {
                    sig[c] += (double)(lam * eps[c]);
                    tau[c] = (lam - lam0) * eps[c];
                }
            } else {
                const T tr = DIM == 3 ? eps[0] + eps[1] + eps[2] : eps[0] + eps[1];
                const T dl = lam - lam0, dm = (T)2 * (mu - mu0);
#pragma unroll
                for (int c = 0; c < NCOMP; ++c) {
                    const bool diag = DIM == 3 ? c < 3 : c < 2;
                    sig[c] += (double)((T)2 * mu * eps[c] + (diag ? lam * tr : (T)0));
                    tau[c] = dm * eps[c] + (diag ? dl * tr : (T)0);
                }
            }
            if (energy) {
#pragma unroll
                for (int c = 0; c < NCOMP; ++c) en += field_weight(PH, DIM, c) * (double)eps[c] * (double)tau[c];
            }
#pragma unroll
            for (int p = 0; p < NP; ++p)
                Z[(p * NC + j) * CS + (n ^ lsw<L, C>(p * NC + j))] = C{tau[2 * p], 2 * p + 1 < NCOMP ? tau[2 * p + 1] : (T)0};
        };
        // material arrays are stored column-major for this pass: one
        // contiguous block of NC * L entries per tile.  The two material paths
        // are separate loops, so the global loads of the per-point path are
        // waited for inside its own branch.
        if (table) {
            sfor<0, EPL>([&](auto qc) __attribute__((always_inline)) {
                constexpr int q = qc;
                const int e = tid + q * TH;
                const int j = e / L, n = e % L;
                if (e >= L * NC || j >= x.ncol) return;
                point(j, n, mat[2 * ph[q]], mat[2 * ph[q] + 1]);
            });
        } else {
            sfor<0, EPL>([&](auto qc) __attribute__((always_inline)) {
                constexpr int q = qc;
                const int e = tid + q * TH;
                const int j = e / L, n = e % L;
                if (e >= L * NC || j >= x.ncol) return;
                const int64_t pt_t = (x.c0 + j) * (int64_t)L + n;
                point(j, n, (T)a.lame_pts_t[2 * pt_t], (T)a.lame_pts_t[2 * pt_t + 1]);
            });
        }
        // fixed-order sums inside the wave, one entry per wave
#pragma unroll
        for (int c = 0; c < NCOMP; ++c) sig[c] = wave_sum_lane63(sig[c]);
        if (energy) en = wave_sum_lane63(en);
        if ((tid & 63) == 63) {
#pragma unroll
            for (int c = 0; c < NCOMP; ++c) red[c * NW + wave] = sig[c];
            red[NCOMP * NW + wave] = en;
        }
    };
    // tile's stress partial from the per-wave sums (thread 0, waves in order)
    auto write_sig = [&](const Tile& x) __attribute__((always_inline)) {
        if (tid == 0) {
            for (int c = 0; c < NCOMP; ++c) {
                double acc = 0.0;
                for (int w = 0; w < NW; ++w) acc += red[c * NW + w];
                a.sig_part[((int64_t)x.load * nct + x.ct) * NCOMP + c] = acc;
            }
            if (energy) {
                double acc = 0.0;
                for (int w = 0; w < NW; ++w) acc += red[NCOMP * NW + w];
                a.en_part[(int64_t)x.load * nct + x.ct] = acc;
            }
        }
    };

    // half spectra of the transformed tile into out[]
    C out[EPT][NCOMP];
    auto unpack = [&](const Tile& x) __attribute__((always_inline)) {
        if (ax.split) walk.start(ax, a.tw64, div_fast(x.c0 + tid % NC, ax.qdiv), tid / NC, TH / NC);
        sfor<0, EPT>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = qc;
            const int e = tid + q * TH;
            const bool ok = e < H * NC && e % NC < x.ncol;
            const int k = ok ? e / NC : 0, j = e % NC;
            C w = C{(T)1, (T)0};
            if (ax.split) w = walk.next<C>();
            const int km = k == 0 ? 0 : L - k;
            sfor<0, NP>([&](auto pc) __attribute__((always_inline)) {
                constexpr int p = pc;
                const C* Zp = Z + (p * NC + j) * CS;
                const int sz = lsw<L, C>(p * NC + j);
                const C zk = Zp[k ^ sz], zm = Zp[km ^ sz];
                C A = C{(T)0.5 * (zk.x + zm.x), (T)0.5 * (zk.y - zm.y)};
                C B = C{(T)0.5 * (zk.y + zm.y), (T)0.5 * (zm.x - zk.x)};
                if (ax.split) { A = cmul(A, w); B = cmul(B, w); }
                out[q][2 * p] = A;
                if constexpr (2 * p + 1 < NCOMP) out[q][2 * p + 1] = B;
            });
        });
    };
    auto store = [&](const Tile& x) __attribute__((always_inline)) {
        C* dst = reinterpret_cast<C*>(x.par ? a.buf0 : a.buf1) + (int64_t)x.load * NCOMP * P.S;
        sfor<0, EPT>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = qc;
            const int e = tid + q * TH;
            const int k = e / NC, j = e % NC;
            if (e >= H * NC || j >= x.ncol) return;
            const uint32_t off = (uint32_t)(((int64_t)k * I + x.c0 + j) * (int64_t)sizeof(C));
            sfor<0, NCOMP>([&](auto fc) __attribute__((always_inline)) {
                constexpr int f = fc;
                stg(reinterpret_cast<C*>(reinterpret_cast<char*>(dst + (int64_t)f * P.S) + off), out[q][f]);
            });
        });
    };

    int64_t t = blockIdx.x;
    if constexpr (!G::PERSIST) {
        // one tile per workgroup; a workgroup without work leaves at once
        if (t >= total) return;
        const Tile x = tile_of(xcd_tile(t, total));
        if (a.st[x.load].done) return;
        load_tables();
        fetch_loads(x);
        pack(x);
        store_tables();                 // older than the tile's loads: no further wait
        __syncthreads();
        fft_cols<L, +1, CS>(Z, NP * NC, twl);
        law(x, phq);
        __syncthreads();
        write_sig(x);
        fft_cols<L, -1, CS>(Z, NP * NC, twl);
        unpack(x);
        store(x);
    } else {
        load_tables();
        store_tables();
        Tile x = t < total ? tile_of(xcd_tile(t, total)) : Tile{0, 0, 0, 0, 0};
        bool have = t < total && !a.st[x.load].done;
        if (have) fetch_loads(x);
        Tile prev = x;
        bool pend = false;
        uint8_t phc[EPL];
        for (; t < total; t += gridDim.x) {
            // a fresh (opaque) copy of the thread index per tile: keeps the
            // per-thread LDS offsets from being hoisted out of the loop and
            // held in registers across all stages
            asm volatile("" : "=v"(tid) : "0"(tid));
            const bool cur = have;
            if (cur) {
                pack(x);
                sfor<0, EPL>([&](auto qc) __attribute__((always_inline)) { phc[qc] = phq[qc]; });
            }
            __syncthreads();
            if (pend) store(prev);      // tile t-1, in flight during this tile's work
            pend = false;
            const Tile xc = x;
            const int64_t tn = t + gridDim.x;
            have = false;
            if (tn < total) {
                x = tile_of(xcd_tile(tn, total));
                have = !a.st[x.load].done;
                if (have) fetch_loads(x);   // tile t+1, in flight during this tile's work
            }
            if (!cur) continue;
            fft_cols<L, +1, CS>(Z, NP * NC, twl, tid);
            law(xc, phc);
            __syncthreads();
            write_sig(xc);
            fft_cols<L, -1, CS>(Z, NP * NC, twl, tid);
            unpack(xc);
            __syncthreads();            // the tile is read out: LDS free for the next packing
            prev = xc;
            pend = true;
        }
        if (pend) store(prev);
    }
}

// =============================================================================
// real-space turnaround, register-resident variant: one wave owns a tile of
// 64 / N1 columns and all packed transforms of it; the columns stay in
// registers from the gather to the scatter, the local law runs on them in
// place, and LDS only carries the FFT exchange and the final half-spectrum
// split, in a region private to the wave (no workgroup barrier per stage).
// =============================================================================
template <typename T, int L> struct RR {
    static constexpr int N1 = Split<L>::N1, N2 = Split<L>::N2, B = N2 / N1;
    static constexpr int NCW = 64 / N1;      // columns per wave
    static constexpr int W = 4;              // waves (independent tiles) per workgroup
    static constexpr int CS = L + 1;
    static constexpr int REGION = NCW * CS;  // complex elements of one wave's LDS region
};

// FFT of one column held by the N1 threads tau of it: v[q] = x[tau + N1 q] in,
// v[b N1 + kb] = X[tau + N1 b + N2 kb] out; base = the column's LDS region.
template <int L, int DIR, typename C>
__device__ __forceinline__ void fft_reg(C* v, C* base, int tau, const C* twl) {
    constexpr int N1 = Split<L>::N1, N2 = Split<L>::N2, B = N2 / N1;
    dft<N2, DIR>(v);
    sfor<1, N2>([&](auto kc) __attribute__((always_inline)) {
        constexpr int ka = kc;
        const C w = twl[ka * N1 + tau];
        v[ka] = DIR < 0 ? cmul(v[ka], w) : cmulc(v[ka], w);
    });
    wave_lds_sync();
    sfor<0, N2>([&](auto kc) __attribute__((always_inline)) {
        constexpr int ka = kc;
        base[ka * N1 + (tau ^ (ka & (N1 - 1)))] = v[ka];
    });
    wave_lds_sync();
    sfor<0, B>([&](auto bc) __attribute__((always_inline)) {
        constexpr int b = bc;
        sfor<0, N1>([&](auto tc) __attribute__((always_inline)) {
            constexpr int t = tc;
            v[b * N1 + t] = base[(tau + N1 * b) * N1 + (t ^ tau)];
        });
        dft<N1, DIR>(v + b * N1);
    });
}

template <typename T, int DIM, int L>
__global__ void __launch_bounds__(256) kf_real_rr(RealArgs a) {
    using C = typename CT<T>::t;
    using R = RR<T, L>;
    constexpr int NCOMP = Comp<DIM>::N, NP = Comp<DIM>::NP;
    constexpr int N1 = R::N1, N2 = R::N2, B = R::B, NCW = R::NCW, CS = R::CS, H = L / 2 + 1;
    constexpr int TW = NCW * R::W;          // columns per workgroup tile
    const Plan& P = *a.plan;
    const AxisDesc& ax = P.ax[0];
    const int64_t I = P.S / H;
    const int64_t nct = (I + TW - 1) / TW;
    const int64_t total = nct * a.nload;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tau = lane % N1, jj = lane / N1;
    C* twl = smem<C>();
    C* X = twl + L + wave * R::REGION + jj * CS;
    double* red = reinterpret_cast<double*>(twl + L + R::W * R::REGION);
    load_twiddles<L>(twl, reinterpret_cast<const C*>(a.tw) + ax.tw_off);
    __syncthreads();
    const int64_t tt = xcd_tile(blockIdx.x, total);
    const int load = (int)(tt / nct);
    const LoadState& st = a.st[load];
    if (st.done) return;
    const int64_t col = (tt % nct) * TW + wave * NCW + jj;
    const bool act = col < I;
    const int64_t colc = act ? col : 0;
    const C* src = reinterpret_cast<const C*>((st.iter & 1) ? a.buf1 : a.buf0) + (int64_t)load * NCOMP * P.S;
    C* dst = reinterpret_cast<C*>((st.iter & 1) ? a.buf0 : a.buf1) + (int64_t)load * NCOMP * P.S;

    // gather the packed full spectra Z_p[k] = A + i B, k = tau + N1 q (rows above
    // L/2 from the conjugate half-spectrum row L - k)
    C v[NP][N2];
    sfor<0, N2>([&](auto qc) __attribute__((always_inline)) {
        constexpr int q = qc;
        const int k = tau + N1 * q;
        const bool upper = 2 * k > L;
        const int kr = upper ? L - k : k;
        C w = C{(T)1, (T)0};
        if (ax.split) w = split_twiddle<C>(ax, a.tw64, div_fast(colc, ax.qdiv) * (int64_t)kr);
        sfor<0, NP>([&](auto pc) __attribute__((always_inline)) {
            constexpr int p = pc;
            C A = ldg(src + (int64_t)(2 * p) * P.S + (int64_t)kr * I + colc);
            C Bv = C{(T)0, (T)0};
            if constexpr (2 * p + 1 < NCOMP) Bv = ldg(src + (int64_t)(2 * p + 1) * P.S + (int64_t)kr * I + colc);
            if (ax.split) { A = cmulc(A, w); Bv = cmulc(Bv, w); }
            if (kr == 0 || 2 * kr == L) { A.y = 0; Bv.y = 0; }
            v[p][q] = upper ? C{A.x + Bv.y, Bv.x - A.y} : C{A.x - Bv.y, A.y + Bv.x};
        });
    });
    sfor<0, NP>([&](auto pc) __attribute__((always_inline)) { fft_reg<L, +1>(v[decltype(pc)::value], X, tau, twl); });

    // local law at x_n, n = tau + N1 (b + B kb) for v[.][b N1 + kb]; then the
    // forward transforms take the samples back in the order n = tau + N1 q
    const T lam0 = (T)a.lam0, mu0 = (T)a.mu0;
    double sig[NCOMP];
#pragma unroll
    for (int c = 0; c < NCOMP; ++c) sig[c] = 0.0;
    C u[NP][N2];
    sfor<0, N2>([&](auto ic) __attribute__((always_inline)) {
        constexpr int i = ic;
        constexpr int b = i / N1, kb = i % N1;
        constexpr int qpos = b + B * kb;
        const int n = tau + N1 * qpos;
        const int64_t pt_t = colc * (int64_t)L + n;
        T lam, mu;
        if (a.lame_pts_t) {
            lam = (T)a.lame_pts_t[2 * pt_t];
            mu = (T)a.lame_pts_t[2 * pt_t + 1];
        } else {
            const int ph = a.phase_t[pt_t];
            lam = (T)a.lame_tab[2 * ph];
            mu = (T)a.lame_tab[2 * ph + 1];
        }
        T eps[NCOMP];
        sfor<0, NP>([&](auto pc) __attribute__((always_inline)) {
            constexpr int p = pc;
            eps[2 * p] = v[p][i].x;
            if constexpr (2 * p + 1 < NCOMP) eps[2 * p + 1] = v[p][i].y;
        });
        const T tr = DIM == 3 ? eps[0] + eps[1] + eps[2] : eps[0] + eps[1];
        const T dl = lam - lam0, dm = (T)2 * (mu - mu0);
        T tv[NCOMP];
#pragma unroll
        for (int c = 0; c < NCOMP; ++c) {
            const bool diag = DIM == 3 ? c < 3 : c < 2;
            if (act) sig[c] += (double)((T)2 * mu * eps[c] + (diag ? lam * tr : (T)0));
            tv[c] = dm * eps[c] + (diag ? dl * tr : (T)0);
        }
        sfor<0, NP>([&](auto pc) __attribute__((always_inline)) {
            constexpr int p = pc;
            u[p][qpos] = C{tv[2 * p], 2 * p + 1 < NCOMP ? tv[2 * p + 1] : (T)0};
        });
    });

    // forward transforms and the half-spectrum split A_k, B_k (k <= L/2),
    // rows k = tau + N1 r of this thread's column
    sfor<0, NP>([&](auto pc) __attribute__((always_inline)) {
        constexpr int p = pc;
        fft_reg<L, -1>(u[p], X, tau, twl);
        wave_lds_sync();
        sfor<0, N2>([&](auto ic) __attribute__((always_inline)) {
            constexpr int i = ic;
            constexpr int b = i / N1, kb = i % N1;
            X[tau + N1 * b + N2 * kb] = u[p][i];
        });
        wave_lds_sync();
        sfor<0, (H + N1 - 1) / N1>([&](auto rc) __attribute__((always_inline)) {
            constexpr int r = rc;
            const int k = tau + N1 * r;
            if (k < H && act) {
                const int km = k == 0 ? 0 : L - k;
                const C zk = X[k], zm = X[km];
                C A = C{(T)0.5 * (zk.x + zm.x), (T)0.5 * (zk.y - zm.y)};
                C Bv = C{(T)0.5 * (zk.y + zm.y), (T)0.5 * (zm.x - zk.x)};
                if (ax.split) {
                    const C w = split_twiddle<C>(ax, a.tw64, div_fast(col, ax.qdiv) * (int64_t)k);
                    A = cmul(A, w);
                    Bv = cmul(Bv, w);
                }
                stg(dst + (int64_t)(2 * p) * P.S + (int64_t)k * I + col, A);
                if constexpr (2 * p + 1 < NCOMP) stg(dst + (int64_t)(2 * p + 1) * P.S + (int64_t)k * I + col, Bv);
            }
        });
    });

    // mean-stress partial sums: wave butterflies, then the waves in order
#pragma unroll
    for (int c = 0; c < NCOMP; ++c) {
        double x = sig[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        sig[c] = x;
    }
    if (lane == 0)
        for (int c = 0; c < NCOMP; ++c) red[wave * NCOMP + c] = sig[c];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int c = 0; c < NCOMP; ++c) {
            double acc = 0.0;
            for (int w2 = 0; w2 < R::W; ++w2) acc += red[w2 * NCOMP + c];
            a.sig_part[((int64_t)load * nct + tt % nct) * NCOMP + c] = acc;
        }
}

// =============================================================================
// middle axes
// =============================================================================
template <typename T, int L, int DIR, int V>
__global__ void __launch_bounds__((Geo<T, L, 1, V>::THREADS)) kf_axis(AxisArgs a) {
    using C = typename CT<T>::t;
    using G = Geo<T, L, 1, V>;
    constexpr int NC = G::NC, CS = G::CS, TH = G::THREADS;
    constexpr int EPT = (NC * L + TH - 1) / TH;
    const Plan& P = *a.plan;
    const AxisDesc& ax = P.ax[a.axis];
    int64_t O = 1, I = 1;
    for (int b = 0; b < a.axis; ++b) O *= (a.slen0_full && b == 0) ? P.ax[0].len : P.ax[b].slen;
    for (int b = a.axis + 1; b < P.D; ++b) I *= P.ax[b].slen;
    const int64_t ncols = O * I;
    const int64_t nct = (ncols + NC - 1) / NC;
    const int64_t total = nct * a.nfield * a.nload;
    const bool rowmajor = I >= NC;
    const bool aligned = rowmajor && (I % NC) == 0;
    int tid = threadIdx.x;
    C* X = smem<C>();
    C* twl = X + G::TILE;
    Twiddles<L, TH, C> twr;
    twr.load(reinterpret_cast<const C*>(a.tw) + ax.tw_off, tid);

    // element e of a tile -> (column j, position l)
    auto map = [&](int e, int& j, int& l) __attribute__((always_inline)) {
        if (rowmajor) { l = e / NC; j = e % NC; } else { j = e / L; l = e % L; }
    };
    auto addr = [&](int64_t c0, int64_t cbase_aligned, int j, int l) __attribute__((always_inline)) -> int64_t {
        if (aligned) return cbase_aligned + j + (int64_t)l * I;
        int64_t cq, cr;
        divmod_fast(c0 + j, I, cq, cr);
        return cq * (int64_t)L * I + cr + (int64_t)l * I;
    };
    auto tile_base = [&](int64_t t, int& load, int64_t& c0) __attribute__((always_inline)) -> C* {
        const int64_t ct = t % nct;
        const int64_t rest = t / nct;
        const int field = (int)(rest % a.nfield);
        load = (int)(rest / a.nfield);
        c0 = ct * NC;
        int par = 0;
        if (a.st) par = (a.st[load].iter + 1) & 1;
        return reinterpret_cast<C*>(par ? a.buf1 : a.buf0) + (int64_t)load * a.load_stride + (int64_t)field * a.field_stride;
    };

    C pre[EPT];
    auto fetch = [&](int64_t t) __attribute__((always_inline)) -> bool {
        int load;
        int64_t c0;
        const C* base = tile_base(t, load, c0);
        if (a.st && a.st[load].done) return false;
        if (aligned && TH % NC == 0) {
            // thread keeps its column j; position advances by TH / NC per step
            const int j = tid % NC, l0 = tid / NC;
            const C* p0 = base + (c0 / I) * (int64_t)L * I + (c0 % I) + j + (int64_t)l0 * I;
            const int64_t step = (int64_t)(TH / NC) * I;
            // unconditional loads, out-of-tile slots clamped to the first
            // position (values unused): keeps later waits on older loads exact
            sfor<0, EPT>([&](auto qc) __attribute__((always_inline)) {
                constexpr int q = qc;
                pre[q] = ldg(tid + q * TH < NC * L ? p0 + q * step : p0);
            });
            return true;
        }
        const int64_t cb = aligned ? (c0 / I) * (int64_t)L * I + (c0 % I) : 0;
        sfor<0, EPT>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = qc;
            const int e = tid + q * TH;
            int j, l;
            map(e, j, l);
            if (!(e < NC * L && c0 + j < ncols)) { j = 0; l = 0; }
            pre[q] = ldg(base + addr(c0, cb, j, l));
        });
        return true;
    };

    // transformed tile (LDS) -> out[] -> HBM; the persistent variants defer
    // the stores of tile t until tile t+1 is packed (software pipeline: the
    // loads of t+1 and the stores of t-1 are in flight during the transform
    // of t, and the wait for the next tile's loads never waits for stores
    // issued just before it)
    C out[EPT];
    // rows of a tile (row-major tiles): thread tid keeps column j = tid % NC
    // at positions l = tid / NC + q TH / NC, so its four-step twiddles walk
    static_assert(TH % NC == 0, "a thread keeps its column");
    const bool walk_ok = ax.split && rowmajor;
    TwiddleWalk walk;
    auto unpack = [&](int64_t c0, int ncol) __attribute__((always_inline)) {
        if (DIR < 0 && walk_ok) walk.start(ax, a.tw64, div_fast(mod_fast(c0 + tid % NC, I), ax.qdiv), tid / NC, TH / NC);
        sfor<0, EPT>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = qc;
            const int e = tid + q * TH;
            int j, l;
            map(e, j, l);
            const bool ok = e < NC * L && j < ncol;
            C w = C{(T)1, (T)0};
            if (DIR < 0 && walk_ok) w = walk.next<C>();
            if (!ok) { j = 0; l = 0; }
            C v = X[j * CS + (l ^ lsw<L, C>(j))];
            if (DIR < 0 && ax.split && ok)
                v = cmul(v, walk_ok ? w : split_twiddle<C>(ax, a.tw64, div_fast(mod_fast(c0 + j, I), ax.qdiv) * (int64_t)l));
            out[q] = v;
        });
    };
    auto store_out = [&](C* base, int64_t c0, int ncol) __attribute__((always_inline)) {
        const int64_t cb = aligned ? (c0 / I) * (int64_t)L * I + (c0 % I) : 0;
        sfor<0, EPT>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = qc;
            const int e = tid + q * TH;
            int j, l;
            map(e, j, l);
            if (e >= NC * L || j >= ncol) return;
            stg(base + addr(c0, cb, j, l), out[q]);
        });
    };
    auto pack = [&](int64_t c0, int ncol) __attribute__((always_inline)) {
        if (DIR > 0 && walk_ok) walk.start(ax, a.tw64, div_fast(mod_fast(c0 + tid % NC, I), ax.qdiv), tid / NC, TH / NC);
        sfor<0, EPT>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = qc;
            const int e = tid + q * TH;
            int j, l;
            map(e, j, l);
            C w = C{(T)1, (T)0};
            if (DIR > 0 && walk_ok) w = walk.next<C>();
            if (e >= NC * L || j >= ncol) return;
            C v = pre[q];
            if (DIR > 0 && ax.split)
                v = cmulc(v, walk_ok ? w : split_twiddle<C>(ax, a.tw64, div_fast(mod_fast(c0 + j, I), ax.qdiv) * (int64_t)l));
            X[j * CS + (l ^ lsw<L, C>(j))] = v;
        });
    };

    int64_t t = blockIdx.x;
    if constexpr (!G::PERSIST) {
        // one tile per workgroup: a workgroup without work leaves here, so the
        // tile's loads lie on the only path below (exact load waits)
        if (t >= total || !fetch(xcd_tile(t, total))) return;
        int load;
        int64_t c0;
        C* base = tile_base(xcd_tile(t, total), load, c0);
        const int ncol = (int)((ncols - c0) < NC ? (ncols - c0) : NC);
        pack(c0, ncol);
        twr.store(twl, tid);   // older than the tile's loads
        __syncthreads();
        fft_cols<L, DIR, CS>(X, NC, twl);
        unpack(c0, ncol);
        store_out(base, c0, ncol);
    } else {
        twr.store(twl, tid);
        bool have = t < total ? fetch(xcd_tile(t, total)) : false;
        bool pend = false;
        C* pbase = nullptr;
        int64_t pc0 = 0;
        int pncol = 0;
        for (; t < total; t += gridDim.x) {
            // a fresh (opaque) copy of the thread index per tile: keeps the
            // per-thread offsets from being hoisted out of the loop and held
            // in registers across all stages
            asm volatile("" : "=v"(tid) : "0"(tid));
            const bool cur = have;
            int load;
            int64_t c0;
            C* base = tile_base(xcd_tile(t, total), load, c0);
            const int ncol = (int)((ncols - c0) < NC ? (ncols - c0) : NC);
            if (cur) pack(c0, ncol);
            __syncthreads();
            if (pend) store_out(pbase, pc0, pncol);   // tile t-1
            pend = false;
            const int64_t tn = t + gridDim.x;
            have = tn < total ? fetch(xcd_tile(tn, total)) : false;   // tile t+1
            if (!cur) continue;
            fft_cols<L, DIR, CS>(X, NC, twl, tid);
            unpack(c0, ncol);
            __syncthreads();   // the tile is read out: LDS free for the next packing
            pend = true;
            pbase = base;
            pc0 = c0;
            pncol = ncol;
        }
        if (pend) store_out(pbase, pc0, pncol);
    }
}

// =============================================================================
// spectral turnaround along the last axis
// =============================================================================
template <typename T, int DIM, int L, int V, int PH>
__global__ void __launch_bounds__((Geo<T, L, Comp<DIM, PH>::N, V>::THREADS)) kf_spec(SpecArgs a) {
    using C = typename CT<T>::t;
    constexpr int NCOMP = Comp<DIM, PH>::N, NT = Comp<DIM, PH>::NT;
    using G = Geo<T, L, NCOMP, V>;
    constexpr int NC = G::NC, CS = G::CS, TH = G::THREADS;
    constexpr int EPT = (NC * L + TH - 1) / TH;
    const Plan& P = *a.plan;
    const int D = P.D;
    const int64_t ncols = P.S / L;
    const int64_t nct = (ncols + NC - 1) / NC;
    const int64_t total = nct * a.nload;
    const int tid = threadIdx.x;
    constexpr int NW = TH / 64;
    C* F = smem<C>();
    C* twl = F + G::TILE;
    int64_t* kb = reinterpret_cast<int64_t*>(twl + L);   // [NC][4]: kappa base (3) + weight
    double* nbd = reinterpret_cast<double*>(kb + NC * 4); // [NC][3]: base numerators (exact doubles)
    double* red = nbd + NC * 3;                           // [2][NW] per-wave residual and Cauchy sums
    Twiddles<L, TH, C> twr;
    twr.load(reinterpret_cast<const C*>(a.tw) + P.ax[D - 1].tw_off, tid);
    const T inv_m = (T)(1.0 / (double)P.m);
    const T mu0 = (T)a.mu0, beta = (T)a.beta;
    // Cauchy step |eps_hat(n+1) - eps_hat(n)|^2: (|dt|^2 + c1 |xi . dt|^2) / (2 mu0^2)
    // in elasticity, |dt|^2 / k0^2 for conductivity
    const double cau_c1 = PH == PHYS_THERMAL ? 0.0 : 1.0 - 4.0 * a.beta + 2.0 * a.beta * a.beta;
    const int last_snf = P.ax[D - 1].snf;
    const int64_t last_mult = P.ax[D - 1].mult;
    // Along a column only the last axis moves: kappa = kappa_b + l mult u_snf,
    // so the centred numerators are (A kappa_b + l A u mult) mod emax.  With
    // emax <= 2^24 every term is an integer below 2^53 and the reduction in
    // doubles is exact (the same integers as the plain 64-bit formula).
    // (A has entries in [0, emax) and mult < e_s <= emax, so every product
    // below is an integer < 2^48 and sums of three stay < 2^53.)
    const int64_t emax = P.fm.emax;
    const bool nfast = emax <= (int64_t(1) << 24);
    const double emax_d = (double)emax, inv_e = 1.0 / emax_d;
    auto dmod = [&](double x) __attribute__((always_inline)) -> double {   // x mod emax, x integer >= 0
        double r = x - floor(x * inv_e) * emax_d;
        if (r < 0) r += emax_d;
        if (r >= emax_d) r -= emax_d;
        return r;
    };
    double Ad[3][3], Gd[3][3], stepd[3];
#pragma unroll
    for (int i2 = 0; i2 < 3; ++i2)
#pragma unroll
        for (int r2 = 0; r2 < 3; ++r2) {
            Ad[i2][r2] = (i2 < DIM && r2 < DIM) ? (double)P.fm.A[i2][r2] : 0.0;
            Gd[i2][r2] = (i2 < DIM && r2 < DIM) ? P.fm.G[i2][r2] : 0.0;
        }
#pragma unroll
    for (int i2 = 0; i2 < 3; ++i2) {
        double a_s = 0.0;
#pragma unroll
        for (int r2 = 0; r2 < 3; ++r2) a_s = r2 == last_snf ? Ad[i2][r2] : a_s;
        stepd[i2] = nfast ? dmod(a_s * (double)last_mult) : 0.0;
    }

    // previous traction of a tile (and, in FP32, the restart's traction
    // offset): the one-tile variants fetch them with the tile's spectra, the
    // persistent ones after packing (in flight during the forward transform)
    constexpr bool HOIST_OFF = sizeof(T) == 4;
    C oldv[EPT][NT];
    C offv[HOIST_OFF ? EPT : 1][NT];
    auto load_old = [&](int load, int64_t c0, int iter) __attribute__((always_inline)) {
        const C* tb = reinterpret_cast<const C*>(a.tbuf) + (int64_t)load * NT * P.S;
        const C* to = reinterpret_cast<const C*>(a.toff) + (int64_t)load * NT * P.S;
        if (ahom_check_iter(iter, a.resid_period, a.max_iter)) {
            sfor<0, EPT>([&](auto qc) __attribute__((always_inline)) {
                constexpr int q = qc;
                const int e = tid + q * TH;
                const int64_t addr = c0 * L + ((e < NC * L && c0 + e / L < ncols) ? e : 0);
                sfor<0, NT>([&](auto cc) __attribute__((always_inline)) {
                    constexpr int c = cc;
                    oldv[q][c] = ldg(tb + (int64_t)c * P.S + addr);
                });
            });
        }
        if constexpr (HOIST_OFF) {
            if (a.toff) {
                sfor<0, EPT>([&](auto qc) __attribute__((always_inline)) {
                    constexpr int q = qc;
                    const int e = tid + q * TH;
                    const int64_t addr = c0 * L + ((e < NC * L && c0 + e / L < ncols) ? e : 0);
                    sfor<0, NT>([&](auto cc) __attribute__((always_inline)) {
                        constexpr int c = cc;
                        offv[q][c] = ldg(to + (int64_t)c * P.S + addr);
                    });
                });
            }
        }
    };

    C pre[EPT][NCOMP];
    auto fetch = [&](int64_t t) __attribute__((always_inline)) -> bool {
        const int load = (int)(t / nct);
        const int64_t c0 = (t % nct) * NC;
        const LoadState& st = a.st[load];
        if (st.done) return false;
        const C* base = reinterpret_cast<const C*>(((st.iter + 1) & 1) ? a.buf1 : a.buf0) + (int64_t)load * NCOMP * P.S;
        // unconditional loads, out-of-tile slots clamped to the tile's first
        // element (values unused): keeps later waits on older loads exact
        sfor<0, EPT>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = qc;
            const int e = tid + q * TH;
            const int64_t addr = c0 * L + ((e < NC * L && c0 + e / L < ncols) ? e : 0);
            sfor<0, NCOMP>([&](auto fc) __attribute__((always_inline)) {
                constexpr int f = fc;
                pre[q][f] = ldg(base + (int64_t)f * P.S + addr);
            });
        });
        if constexpr (!G::PERSIST) load_old(load, c0, st.iter);
        return true;
    };

    int64_t t = blockIdx.x;
    bool have;
    if constexpr (!G::PERSIST) {
        // one tile per workgroup: a workgroup without work leaves here, so the
        // tile's loads lie on the only path below (exact load waits)
        if (t >= total || !fetch(xcd_tile(t, total))) return;
        have = true;
    } else {
        twr.store(twl, tid);
        have = t < total ? fetch(xcd_tile(t, total)) : false;
    }
    for (; t < total; t += gridDim.x) {
        const bool cur = have;
        const int64_t tt = xcd_tile(t, total);
        const int load = (int)(tt / nct);
        const int64_t c0 = (tt % nct) * NC;
        const int ncol = (int)((ncols - c0) < NC ? (ncols - c0) : NC);
        if (cur) {
            // per-column Smith indices of the other axes (while the tile's
            // loads are in flight); 32-bit division where the column count fits
            if (tid < NC) {
                int64_t k0 = 0, kq0 = 0, kq1 = 0, kq2 = 0;
                auto acc = [&](int b, int64_t kk) __attribute__((always_inline)) {
                    const int64_t v = P.ax[b].mult * kk;
                    const int sn = P.ax[b].snf;
                    kq0 += sn == 0 ? v : 0;
                    kq1 += sn == 1 ? v : 0;
                    kq2 += sn == 2 ? v : 0;
                    if (b == 0) k0 = kk;
                };
                if (ncols < (int64_t(1) << 31)) {
                    uint32_t o = (uint32_t)(c0 + tid);
                    for (int b = D - 2; b >= 0; --b) {
                        const uint32_t sl = (uint32_t)P.ax[b].slen;
                        acc(b, (int64_t)(o % sl));
                        o /= sl;
                    }
                } else {
                    int64_t o = c0 + tid;
                    for (int b = D - 2; b >= 0; --b) {
                        const int64_t sl = P.ax[b].slen;
                        acc(b, o % sl);
                        o /= sl;
                    }
                }
                kb[tid * 4 + 0] = kq0;
                kb[tid * 4 + 1] = kq1;
                kb[tid * 4 + 2] = kq2;
                kb[tid * 4 + 3] = (k0 == 0 || 2 * k0 == P.ax[0].len) ? 1 : 2;
                if (nfast) {
                    const double kq[3] = {(double)kq0, (double)kq1, (double)kq2};
#pragma unroll
                    for (int i2 = 0; i2 < DIM; ++i2) {
                        double acc = 0.0;
#pragma unroll
                        for (int s2 = 0; s2 < DIM; ++s2) acc += Ad[i2][s2] * kq[s2];
                        nbd[tid * 3 + i2] = dmod(acc);
                    }
                }
            }
            sfor<0, EPT>([&](auto qc) __attribute__((always_inline)) {
                constexpr int q = qc;
                const int e = tid + q * TH;
                const int j = e / L, l = e % L;
                if (e >= NC * L || j >= ncol) return;
                sfor<0, NCOMP>([&](auto fc) __attribute__((always_inline)) {
                    constexpr int f = fc;
                    F[(f * NC + j) * CS + (l ^ lsw<L, C>(f * NC + j))] = pre[q][f];
                });
            });
        }
        if constexpr (!G::PERSIST) twr.store(twl, tid);   // older than the tile's loads
        __syncthreads();
        const int64_t tn = t + gridDim.x;
        if constexpr (G::PERSIST) have = tn < total ? fetch(xcd_tile(tn, total)) : false;
        else have = false;
        if (!cur) {
            if constexpr (!G::PERSIST) break;
            continue;
        }
        const LoadState& st = a.st[load];
        C* base = reinterpret_cast<C*>(((st.iter + 1) & 1) ? a.buf1 : a.buf0) + (int64_t)load * NCOMP * P.S;
        C* tb = reinterpret_cast<C*>(a.tbuf) + (int64_t)load * NT * P.S;
        const bool chk = ahom_check_iter(st.iter, a.resid_period, a.max_iter);
        const bool wrt = ahom_write_traction(st.iter, a.resid_period, a.max_iter);
        const C* to = reinterpret_cast<const C*>(a.toff) + (int64_t)load * NT * P.S;
        if constexpr (G::PERSIST) load_old(load, c0, st.iter);
        fft_cols<L, -1, CS>(F, NCOMP * NC, twl);

        const double* eb = a.eps_bar + (int64_t)load * NCOMP;
        double res = 0.0, cau = 0.0;
        sfor<0, EPT>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = qc;
            const int e = tid + q * TH;
            const int j = e / L, l = e % L;
            if (e >= NC * L || j >= ncol) return;
            const int64_t add = last_mult * l;
            int64_t kap[3] = {kb[j * 4 + 0] + (last_snf == 0 ? add : 0), kb[j * 4 + 1] + (last_snf == 1 ? add : 0),
                              kb[j * 4 + 2] + (last_snf == 2 ? add : 0)};
            C* fp[NCOMP];
#pragma unroll
            for (int f = 0; f < NCOMP; ++f) fp[f] = F + (f * NC + j) * CS + (l ^ lsw<L, C>(f * NC + j));
            if (kap[0] == 0 && kap[1] == 0 && kap[2] == 0) {
#pragma unroll
                for (int f = 0; f < NCOMP; ++f) *fp[f] = C{(T)eb[f], (T)0};
                return;
            }
            double Nd[3];
            int half = 0;
            if (nfast) {
#pragma unroll
                for (int i = 0; i < DIM; ++i) {
                    double r = dmod(nbd[j * 3 + i] + (double)l * stepd[i]);
                    if (2 * r >= emax_d) r -= emax_d;
                    if (2 * r == -emax_d) half = 1;
                    Nd[i] = r;
                }
            } else {
                int64_t N[3];
                half = centred_numerators(P.fm, kap, N, DIM);
#pragma unroll
                for (int i = 0; i < DIM; ++i) Nd[i] = (double)N[i];
            }
            if (half && !self_conjugate(P.fm, kap, DIM)) {
#pragma unroll
                for (int f = 0; f < NCOMP; ++f) *fp[f] = C{(T)0, (T)0};
                return;
            }
            double hd[DIM];
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                hd[i] = 0.0;
#pragma unroll
                for (int r = 0; r < DIM; ++r) hd[i] += Gd[i][r] * Nd[r];
            }
            double hn = 0.0;
#pragma unroll
            for (int i = 0; i < DIM; ++i) hn += hd[i] * hd[i];
            hn = rsqrt(hn);
            T xi[DIM];
#pragma unroll
            for (int i = 0; i < DIM; ++i) xi[i] = (T)(hd[i] * hn);
            C tv[NCOMP];
#pragma unroll
            for (int f = 0; f < NCOMP; ++f) { C v = *fp[f]; tv[f] = C{v.x * inv_m, v.y * inv_m}; }
            C tt[NT];
            if constexpr (PH == PHYS_THERMAL) {
                tt[0] = C{(T)0, (T)0};
#pragma unroll
                for (int i = 0; i < DIM; ++i) { tt[0].x += tv[i].x * xi[i]; tt[0].y += tv[i].y * xi[i]; }
            } else if constexpr (DIM == 3) {
                const C T00 = tv[0], T11 = tv[1], T22 = tv[2], T12 = tv[3], T02 = tv[4], T01 = tv[5];
                tt[0] = C{T00.x * xi[0] + T01.x * xi[1] + T02.x * xi[2], T00.y * xi[0] + T01.y * xi[1] + T02.y * xi[2]};
                tt[1] = C{T01.x * xi[0] + T11.x * xi[1] + T12.x * xi[2], T01.y * xi[0] + T11.y * xi[1] + T12.y * xi[2]};
                tt[2] = C{T02.x * xi[0] + T12.x * xi[1] + T22.x * xi[2], T02.y * xi[0] + T12.y * xi[1] + T22.y * xi[2]};
            } else {
                const C T00 = tv[0], T11 = tv[1], T01 = tv[2];
                tt[0] = C{T00.x * xi[0] + T01.x * xi[1], T00.y * xi[0] + T01.y * xi[1]};
                tt[1] = C{T01.x * xi[0] + T11.x * xi[1], T01.y * xi[0] + T11.y * xi[1]};
            }
            const int64_t spos = c0 * L + e;
            // residual and Cauchy terms of this frequency; accumulated once
            // below, outside the branches (per-branch updates of the two sums
            // were merged by the compiler into a store through a selected
            // address, which put both sums in scratch memory)
            double r2 = 0.0, c2 = 0.0;
            if (a.cg_alpha) {
                // conjugate gradients: traction of the updated iterate t + alpha t_p
                const T cg_a = (T)a.cg_alpha[load];
#pragma unroll
                for (int c = 0; c < NT; ++c) {
                    const C nt = C{oldv[q][c].x + cg_a * tt[c].x, oldv[q][c].y + cg_a * tt[c].y};
                    r2 += (double)nt.x * (double)nt.x + (double)nt.y * (double)nt.y;
                    stg(tb + (int64_t)c * P.S + spos, nt);
                }
            } else if (chk) {
                double xdx = 0.0, xdy = 0.0;
#pragma unroll
                for (int c = 0; c < NT; ++c) {
                    const double dx = (double)tt[c].x - (double)oldv[q][c].x, dy = (double)tt[c].y - (double)oldv[q][c].y;
                    r2 += dx * dx + dy * dy;
                    xdx += (double)xi[c] * dx;
                    xdy += (double)xi[c] * dy;
                    if (a.dout) {
                        const int64_t o = ((int64_t)load * NT + c) * P.S + spos;
                        reinterpret_cast<float2*>(a.dout)[o] = float2{(float)dx, (float)dy};
                        reinterpret_cast<float2*>(a.dneg)[o] = float2{(float)-dx, (float)-dy};
                    }
                }
                // Cauchy term |eps_hat(n+1) - eps_hat(n)|^2 up to 1 / (2 mu0^2)
                c2 = r2 + cau_c1 * (xdx * xdx + xdy * xdy);
            }
            const double wk = (double)kb[j * 4 + 3];
            res += wk * r2;
            cau += wk * c2;
            if (wrt && !a.cg_alpha) {
#pragma unroll
                for (int c = 0; c < NT; ++c) stg(tb + (int64_t)c * P.S + spos, tt[c]);
            }
            if (a.toff) {
#pragma unroll
                for (int c = 0; c < NT; ++c) {
                    C o;
                    if constexpr (HOIST_OFF) o = offv[q][c];
                    else o = ldg(to + (int64_t)c * P.S + spos);
                    tt[c] = C{tt[c].x + o.x, tt[c].y + o.y};
                }
            }
            const T im0 = (T)1 / mu0;
            if constexpr (PH == PHYS_THERMAL) {
                // e_hat = -xi (tau_hat . xi) / k0
#pragma unroll
                for (int i = 0; i < DIM; ++i) *fp[i] = C{-xi[i] * tt[0].x * im0, -xi[i] * tt[0].y * im0};
            } else {
                C xt = C{(T)0, (T)0};
#pragma unroll
                for (int i = 0; i < DIM; ++i) { xt.x += xi[i] * tt[i].x; xt.y += xi[i] * tt[i].y; }
                C v[DIM];
#pragma unroll
                for (int i = 0; i < DIM; ++i) v[i] = C{(tt[i].x - beta * xt.x * xi[i]) * im0, (tt[i].y - beta * xt.y * xi[i]) * im0};
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
                    *fp[2] = C{(T)-0.5 * (xi[0] * v[1].x + xi[1] * v[0].x), (T)-0.5 * (xi[0] * v[1].y + xi[1] * v[0].y)};
                }
            }
        });
        // fixed-order residual and Cauchy sums: inside the wave, then waves in order
        res = wave_sum_lane63(res);
        cau = wave_sum_lane63(cau);
        if ((tid & 63) == 63) {
            red[tid >> 6] = res;
            red[NW + (tid >> 6)] = cau;
        }
        __syncthreads();
        if (tid == 0) {
            double acc = 0.0, acc2 = 0.0;
            for (int w = 0; w < NW; ++w) {
                acc += red[w];
                acc2 += red[NW + w];
            }
            a.res_part[(int64_t)load * nct + tt % nct] = acc;
            if (a.cau_part) a.cau_part[(int64_t)load * nct + tt % nct] = acc2;
        }
        fft_cols<L, +1, CS>(F, NCOMP * NC, twl);
        // read the tile out into registers, then store (the LDS reads go out
        // back to back instead of alternating with the stores)
        C out[EPT][NCOMP];
        sfor<0, EPT>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = qc;
            const int e = tid + q * TH;
            const bool ok = e < NC * L && e / L < ncol;
            const int j = ok ? e / L : 0, l = e % L;
            sfor<0, NCOMP>([&](auto fc) __attribute__((always_inline)) {
                constexpr int f = fc;
                out[q][f] = F[(f * NC + j) * CS + (l ^ lsw<L, C>(f * NC + j))];
            });
        });
        sfor<0, EPT>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = qc;
            const int e = tid + q * TH;
            if (e >= NC * L || e / L >= ncol) return;
            const int64_t addr = c0 * L + e;
            sfor<0, NCOMP>([&](auto fc) __attribute__((always_inline)) {
                constexpr int f = fc;
                stg(base + (int64_t)f * P.S + addr, out[q][f]);
            });
        });
        if constexpr (!G::PERSIST) break;  // one tile per workgroup
        __syncthreads();                   // LDS free for the next tile
    }
}

// ----------------------------------------------------------------- dispatch
// The launchers are explicit template instantiations split over several
// compilation parts (AHOM_FAST_PART, see the build script) so that the many
// kernel instantiations compile in parallel; part "dispatch" holds the
// exported entry points.
namespace ahom_fast_detail {

template <typename T, int L, int NF, int V>
FastGeom geom_of(int kind) {
    using G = Geo<T, L, NF, V>;
    FastGeom g;
    g.NC = G::NC;
    g.threads = G::THREADS;
    g.persistent = G::PERSIST;
    // tile + twiddles + per-column integers (spec: kappa + weight) or
    // per-wave stress sums (real; the phase table is added at launch)
    size_t extra = kind == FAST_SPEC ? (size_t)G::NC * (32 + 24) + (size_t)(G::THREADS / 64) * 16
                                     : (kind == FAST_REAL ? (size_t)7 * (G::THREADS / 64) * 8 : 0);
    size_t lds = (size_t)G::TILE * G::es + (size_t)L * G::es + extra;
    // block reduction of the other passes reuses the tile: one double per thread
    const size_t red = (size_t)G::THREADS * 8;
    g.lds = lds > red ? lds : red;
    return g;
}

// lengths with tile variants; shorter transforms use variant 0 only
constexpr bool tuned_length(int L) { return L >= 32; }

// fields held by a tile: packed transforms (real-space pass), components
// (spectral pass) or one field (middle axes)
inline int tile_fields(int kind, int dim, int phys) {
    const int n = phys == PHYS_THERMAL ? dim : (dim == 3 ? 6 : 3);
    return kind == FAST_REAL ? (n + 1) / 2 : (kind == FAST_SPEC ? n : 1);
}

template <typename T, int V>
bool geom_TV(int kind, int dim, int L, FastGeom* g, int phys = PHYS_ELASTIC) {
    const int nf = tile_fields(kind, dim, phys);
#define AHOM_G(LL)                                                     \
    case LL:                                                           \
        if (nf == 1) *g = geom_of<T, LL, 1, V>(kind);                  \
        else if (nf == 2) *g = geom_of<T, LL, 2, V>(kind);             \
        else if (nf == 3) *g = geom_of<T, LL, 3, V>(kind);             \
        else *g = geom_of<T, LL, 6, V>(kind);                          \
        return true;
    switch (L) {
        AHOM_G(1) AHOM_G(2) AHOM_G(4) AHOM_G(8) AHOM_G(16) AHOM_G(32) AHOM_G(64) AHOM_G(128) AHOM_G(256)
        default: return false;
    }
#undef AHOM_G
}

// Geometry of the kernel that a launch of variant V runs for length L: axes
// shorter than the tuned lengths instantiate variant 0 only, so their launch
// geometry (threads, LDS, grid) must be variant 0's as well.
template <typename T, int V>
bool geom_launch(int kind, int dim, int L, FastGeom* g, int phys) {
    return tuned_length(L) ? geom_TV<T, V>(kind, dim, L, g, phys) : geom_TV<T, 0>(kind, dim, L, g, phys);
}

// Set the LDS attribute and return the grid: one workgroup per tile, or for
// the persistent schedule the workgroups that fit on the device at once
// (occupancy API: registers, LDS and threads), capped by the tiles.
template <typename F>
int prepare(F fn, const FastGeom& g, int64_t total, int ncu) {
    if (g.lds > 64 * 1024)
        if (hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds) != hipSuccess) return -1;
    if (!g.persistent) return (int)total;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, g.threads, g.lds) != hipSuccess || per_cu < 1) per_cu = 1;
    int64_t grid = (int64_t)ncu * per_cu;
    if (grid > total) grid = total;
    return (int)(grid < 1 ? 1 : grid);
}

template <typename F, typename A>
int go(F fn, const FastGeom& g, int64_t total, int ncu, hipStream_t s, const A& a) {
    const int nb = prepare(fn, g, total, ncu);
    if (nb < 0) return -1;
    hipLaunchKernelGGL(fn, dim3(nb), dim3(g.threads), g.lds, s, a);
    return 0;
}

template <typename T, int V, int PH>
int real_TV(int dim, int L, const RealArgs& a, int64_t total, int ncu, hipStream_t s) {
    FastGeom g;
    if (!geom_launch<T, V>(FAST_REAL, dim, L, &g, PH)) return -1;
    // the phase table (Lame pairs in the working precision) follows in LDS
    if (!a.lame_pts_t && (a.n_phase < 1 || a.n_phase > 256 || !a.lame_tab)) return -1;
    if (!a.lame_pts_t) g.lds += (size_t)a.n_phase * 2 * sizeof(T);
#define AHOM_FR(LL)                                                                    \
    case LL:                                                                           \
        return dim == 3 ? go(kf_real<T, 3, LL, (tuned_length(LL) ? V : 0), PH>, g, total, ncu, s, a) \
                        : go(kf_real<T, 2, LL, (tuned_length(LL) ? V : 0), PH>, g, total, ncu, s, a);
    switch (L) {
        AHOM_FR(1) AHOM_FR(2) AHOM_FR(4) AHOM_FR(8) AHOM_FR(16) AHOM_FR(32) AHOM_FR(64) AHOM_FR(128) AHOM_FR(256)
        default: return -1;
    }
#undef AHOM_FR
}

template <typename T, int V>
int axis_TV(int dir, int L, const AxisArgs& a, int64_t total, int ncu, hipStream_t s) {
    FastGeom g;
    if (!geom_launch<T, V>(FAST_AXIS, 3, L, &g, PHYS_ELASTIC)) return -1;
#define AHOM_FA(LL)                                                                    \
    case LL:                                                                           \
        return dir < 0 ? go(kf_axis<T, LL, -1, (tuned_length(LL) ? V : 0)>, g, total, ncu, s, a) \
                       : go(kf_axis<T, LL, 1, (tuned_length(LL) ? V : 0)>, g, total, ncu, s, a);
    switch (L) {
        AHOM_FA(1) AHOM_FA(2) AHOM_FA(4) AHOM_FA(8) AHOM_FA(16) AHOM_FA(32) AHOM_FA(64) AHOM_FA(128) AHOM_FA(256)
        default: return -1;
    }
#undef AHOM_FA
}

template <typename T, int V, int PH>
int spec_TV(int dim, int L, const SpecArgs& a, int64_t total, int ncu, hipStream_t s) {
    FastGeom g;
    if (!geom_launch<T, V>(FAST_SPEC, dim, L, &g, PH)) return -1;
#define AHOM_FS(LL)                                                                    \
    case LL:                                                                           \
        return dim == 3 ? go(kf_spec<T, 3, LL, (tuned_length(LL) ? V : 0), PH>, g, total, ncu, s, a) \
                        : go(kf_spec<T, 2, LL, (tuned_length(LL) ? V : 0), PH>, g, total, ncu, s, a);
    switch (L) {
        AHOM_FS(1) AHOM_FS(2) AHOM_FS(4) AHOM_FS(8) AHOM_FS(16) AHOM_FS(32) AHOM_FS(64) AHOM_FS(128) AHOM_FS(256)
        default: return -1;
    }
#undef AHOM_FS
}

}  // namespace ahom_fast_detail

namespace ahom_fast_detail {
// register-resident real-space variant (tile variant 4)
constexpr int kRRVariant = 4;
constexpr bool rr_length(int L) { return L >= 32 && L <= 256; }

template <typename T, int LL>
FastGeom geom_rr(int dim) {
    using R = RR<T, LL>;
    FastGeom g;
    g.NC = R::NCW * R::W;
    g.threads = 64 * R::W;
    g.persistent = false;
    g.lds = (size_t)(LL + R::W * R::REGION) * 2 * sizeof(T) + (size_t)R::W * 6 * 8;
    (void)dim;
    return g;
}

template <typename T>
bool geom_rr_T(int dim, int L, FastGeom* g) {
    switch (L) {
        case 32: *g = geom_rr<T, 32>(dim); return true;
        case 64: *g = geom_rr<T, 64>(dim); return true;
        case 128: *g = geom_rr<T, 128>(dim); return true;
        case 256: *g = geom_rr<T, 256>(dim); return true;
        default: return false;
    }
}

template <typename T>
int real_RR(int dim, int L, const RealArgs& a, int64_t total, int ncu, hipStream_t s);

template <typename T>
bool geom_T(int kind, int dim, int L, int v, FastGeom* g, int phys) {
    if (v == kRRVariant) {
        // variant 4: the register-resident real-space pass, the quarter-width spectral pass
        if (kind == FAST_REAL) return phys == PHYS_ELASTIC && rr_length(L) && geom_rr_T<T>(dim, L, g);
        if (kind != FAST_SPEC) return false;
        return tuned_length(L) ? geom_TV<T, 4>(kind, dim, L, g, phys) : geom_TV<T, 0>(kind, dim, L, g, phys);
    }
    if (v > kRRVariant) return false;
    if (!tuned_length(L)) v = 0;
    switch (v) {
        case 0: return geom_TV<T, 0>(kind, dim, L, g, phys);
        case 1: return geom_TV<T, 1>(kind, dim, L, g, phys);
        case 2: return geom_TV<T, 2>(kind, dim, L, g, phys);
        default: return geom_TV<T, 3>(kind, dim, L, g, phys);
    }
}

#define AHOM_DECL_TV(T, V)                                                                                          \
    extern template int real_TV<T, V, PHYS_ELASTIC>(int, int, const RealArgs&, int64_t, int, hipStream_t);       \
    extern template int real_TV<T, V, PHYS_THERMAL>(int, int, const RealArgs&, int64_t, int, hipStream_t);       \
    extern template int axis_TV<T, V>(int, int, const AxisArgs&, int64_t, int, hipStream_t);                     \
    extern template int spec_TV<T, V, PHYS_ELASTIC>(int, int, const SpecArgs&, int64_t, int, hipStream_t);       \
    extern template int spec_TV<T, V, PHYS_THERMAL>(int, int, const SpecArgs&, int64_t, int, hipStream_t);
#define AHOM_INST_REAL(T, V, PH) template int real_TV<T, V, PH>(int, int, const RealArgs&, int64_t, int, hipStream_t);
#define AHOM_INST_AXIS(T, V) template int axis_TV<T, V>(int, int, const AxisArgs&, int64_t, int, hipStream_t);
#define AHOM_INST_SPEC(T, V, PH) template int spec_TV<T, V, PH>(int, int, const SpecArgs&, int64_t, int, hipStream_t);

#if defined(AHOM_FAST_PART)
#if AHOM_FAST_PART == 0
AHOM_INST_REAL(double, 0, PHYS_ELASTIC) AHOM_INST_REAL(double, 1, PHYS_ELASTIC) AHOM_INST_REAL(double, 2, PHYS_ELASTIC) AHOM_INST_REAL(double, 3, PHYS_ELASTIC)
#elif AHOM_FAST_PART == 1
AHOM_INST_REAL(float, 0, PHYS_ELASTIC) AHOM_INST_REAL(float, 1, PHYS_ELASTIC) AHOM_INST_REAL(float, 2, PHYS_ELASTIC) AHOM_INST_REAL(float, 3, PHYS_ELASTIC)
#elif AHOM_FAST_PART == 2
AHOM_INST_AXIS(double, 0) AHOM_INST_AXIS(double, 1) AHOM_INST_AXIS(double, 2) AHOM_INST_AXIS(double, 3)
#elif AHOM_FAST_PART == 3
AHOM_INST_AXIS(float, 0) AHOM_INST_AXIS(float, 1) AHOM_INST_AXIS(float, 2) AHOM_INST_AXIS(float, 3)
#elif AHOM_FAST_PART == 4
AHOM_INST_SPEC(double, 0, PHYS_ELASTIC) AHOM_INST_SPEC(double, 1, PHYS_ELASTIC)
#elif AHOM_FAST_PART == 5
AHOM_INST_SPEC(double, 2, PHYS_ELASTIC) AHOM_INST_SPEC(double, 3, PHYS_ELASTIC) AHOM_INST_SPEC(double, 4, PHYS_ELASTIC)
#elif AHOM_FAST_PART == 6
AHOM_INST_SPEC(float, 0, PHYS_ELASTIC) AHOM_INST_SPEC(float, 1, PHYS_ELASTIC) AHOM_INST_SPEC(float, 2, PHYS_ELASTIC) AHOM_INST_SPEC(float, 3, PHYS_ELASTIC)
AHOM_INST_SPEC(float, 4, PHYS_ELASTIC)
#elif AHOM_FAST_PART == 8
AHOM_INST_REAL(double, 0, PHYS_THERMAL) AHOM_INST_REAL(double, 1, PHYS_THERMAL) AHOM_INST_REAL(double, 2, PHYS_THERMAL) AHOM_INST_REAL(double, 3, PHYS_THERMAL)
#elif AHOM_FAST_PART == 9
AHOM_INST_REAL(float, 0, PHYS_THERMAL) AHOM_INST_REAL(float, 1, PHYS_THERMAL) AHOM_INST_REAL(float, 2, PHYS_THERMAL) AHOM_INST_REAL(float, 3, PHYS_THERMAL)
#elif AHOM_FAST_PART == 10
AHOM_INST_SPEC(double, 0, PHYS_THERMAL) AHOM_INST_SPEC(double, 1, PHYS_THERMAL) AHOM_INST_SPEC(double, 2, PHYS_THERMAL) AHOM_INST_SPEC(double, 3, PHYS_THERMAL)
AHOM_INST_SPEC(double, 4, PHYS_THERMAL)
#elif AHOM_FAST_PART == 11
AHOM_INST_SPEC(float, 0, PHYS_THERMAL) AHOM_INST_SPEC(float, 1, PHYS_THERMAL) AHOM_INST_SPEC(float, 2, PHYS_THERMAL) AHOM_INST_SPEC(float, 3, PHYS_THERMAL)
AHOM_INST_SPEC(float, 4, PHYS_THERMAL)
#elif AHOM_FAST_PART == 7
template <typename T>
int real_RR(int dim, int L, const RealArgs& a, int64_t total, int ncu, hipStream_t s) {
    FastGeom g;
    if (a.en_part || !geom_rr_T<T>(dim, L, &g)) return -1;   // no energy sums in this variant
#define AHOM_FRR(LL)                                                                 \
    case LL:                                                                         \
        return dim == 3 ? go(kf_real_rr<T, 3, LL>, g, total, ncu, s, a) : go(kf_real_rr<T, 2, LL>, g, total, ncu, s, a);
    switch (L) {
        AHOM_FRR(32) AHOM_FRR(64) AHOM_FRR(128) AHOM_FRR(256)
        default: return -1;
    }
#undef AHOM_FRR
}
template int real_RR<double>(int, int, const RealArgs&, int64_t, int, hipStream_t);
template int real_RR<float>(int, int, const RealArgs&, int64_t, int, hipStream_t);
#endif
#else
AHOM_DECL_TV(double, 0) AHOM_DECL_TV(double, 1) AHOM_DECL_TV(double, 2) AHOM_DECL_TV(double, 3)
AHOM_DECL_TV(float, 0) AHOM_DECL_TV(float, 1) AHOM_DECL_TV(float, 2) AHOM_DECL_TV(float, 3)
extern template int spec_TV<double, 4, PHYS_ELASTIC>(int, int, const SpecArgs&, int64_t, int, hipStream_t);
extern template int spec_TV<double, 4, PHYS_THERMAL>(int, int, const SpecArgs&, int64_t, int, hipStream_t);
extern template int spec_TV<float, 4, PHYS_ELASTIC>(int, int, const SpecArgs&, int64_t, int, hipStream_t);
extern template int spec_TV<float, 4, PHYS_THERMAL>(int, int, const SpecArgs&, int64_t, int, hipStream_t);
extern template int real_RR<double>(int, int, const RealArgs&, int64_t, int, hipStream_t);
extern template int real_RR<float>(int, int, const RealArgs&, int64_t, int, hipStream_t);
#endif

}  // namespace ahom_fast_detail

#if !defined(AHOM_FAST_PART)
using namespace ahom_fast_detail;

bool ahom_fast_geom(int prec, int kind, int dim, int L, int variant, FastGeom* g, int phys) {
    return prec == 0 ? geom_T<double>(kind, dim, L, variant, g, phys) : geom_T<float>(kind, dim, L, variant, g, phys);
}

#define AHOM_VSWITCH(FN, ...)                                                  \
    do {                                                                       \
        if (prec == 0) {                                                       \
            switch (variant) {                                                 \
                case 0: return FN<double, 0>(__VA_ARGS__);                     \
                case 1: return FN<double, 1>(__VA_ARGS__);                     \
                case 2: return FN<double, 2>(__VA_ARGS__);                     \
                default: return FN<double, 3>(__VA_ARGS__);                    \
            }                                                                  \
        }                                                                      \
        switch (variant) {                                                     \
            case 0: return FN<float, 0>(__VA_ARGS__);                          \
            case 1: return FN<float, 1>(__VA_ARGS__);                          \
            case 2: return FN<float, 2>(__VA_ARGS__);                          \
            default: return FN<float, 3>(__VA_ARGS__);                         \
        }                                                                      \
    } while (0)
// the same with the physics as a third template argument
#define AHOM_VPSWITCH(FN, PH, ...)                                             \
    do {                                                                       \
        if (prec == 0) {                                                       \
            switch (variant) {                                                 \
                case 0: return FN<double, 0, PH>(__VA_ARGS__);                 \
                case 1: return FN<double, 1, PH>(__VA_ARGS__);                 \
                case 2: return FN<double, 2, PH>(__VA_ARGS__);                 \
                default: return FN<double, 3, PH>(__VA_ARGS__);                \
            }                                                                  \
        }                                                                      \
        switch (variant) {                                                     \
            case 0: return FN<float, 0, PH>(__VA_ARGS__);                      \
            case 1: return FN<float, 1, PH>(__VA_ARGS__);                      \
            case 2: return FN<float, 2, PH>(__VA_ARGS__);                      \
            default: return FN<float, 3, PH>(__VA_ARGS__);                     \
        }                                                                      \
    } while (0)

int ahom_launch_fast_real(int prec, int dim, int L, int variant, const RealArgs& a, int64_t total, int ncu, hipStream_t s) {
    int rc;
    if (variant == kRRVariant) {
        if (a.phys != PHYS_ELASTIC) return -1;   // the register-resident variant is elastic only
        rc = prec == 0 ? real_RR<double>(dim, L, a, total, ncu, s) : real_RR<float>(dim, L, a, total, ncu, s);
        return rc == 0 && hipGetLastError() == hipSuccess ? 0 : -1;
    }
    auto run = [&]() -> int {
        if (a.phys == PHYS_THERMAL) AHOM_VPSWITCH(real_TV, PHYS_THERMAL, dim, L, a, total, ncu, s);
        AHOM_VPSWITCH(real_TV, PHYS_ELASTIC, dim, L, a, total, ncu, s);
    };
    rc = run();
    return rc == 0 && hipGetLastError() == hipSuccess ? 0 : -1;
}

int ahom_launch_fast_axis(int prec, int dir, int L, int variant, const AxisArgs& a, int64_t total, int ncu, hipStream_t s) {
    int rc;
    auto run = [&]() -> int { AHOM_VSWITCH(axis_TV, dir, L, a, total, ncu, s); };
    rc = run();
    return rc == 0 && hipGetLastError() == hipSuccess ? 0 : -1;
}

int ahom_launch_fast_spec(int prec, int dim, int L, int variant, const SpecArgs& a, int64_t total, int ncu, hipStream_t s) {
    int rc;
    if (variant == 4) {   // quarter-width tiles (tuned lengths only; shorter axes run variant 0)
        if (prec == 0)
            rc = a.phys == PHYS_THERMAL ? spec_TV<double, 4, PHYS_THERMAL>(dim, L, a, total, ncu, s)
                                        : spec_TV<double, 4, PHYS_ELASTIC>(dim, L, a, total, ncu, s);
        else
            rc = a.phys == PHYS_THERMAL ? spec_TV<float, 4, PHYS_THERMAL>(dim, L, a, total, ncu, s)
                                        : spec_TV<float, 4, PHYS_ELASTIC>(dim, L, a, total, ncu, s);
        return rc == 0 && hipGetLastError() == hipSuccess ? 0 : -1;
    }
    auto run = [&]() -> int {
        if (a.phys == PHYS_THERMAL) AHOM_VPSWITCH(spec_TV, PHYS_THERMAL, dim, L, a, total, ncu, s);
        AHOM_VPSWITCH(spec_TV, PHYS_ELASTIC, dim, L, a, total, ncu, s);
    };
    rc = run();
    return rc == 0 && hipGetLastError() == hipSuccess ? 0 : -1;
}
#endif  // !AHOM_FAST_PART
