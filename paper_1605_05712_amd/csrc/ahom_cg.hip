// Conjugate-gradient scheme on the pattern Lippmann-Schwinger system.
//
// The operator A p = Gamma0 * (C : p) is one sweep of the Basic Scheme's
// passes with the law C : eps (reference Lame constants zero in the real-space
// pass) and the mean set to zero in the spectral pass; these kernels add the
// vector updates and the scalar recurrences of CG in the C0 inner product
// <u, v>_C0 = sum_x u : C0 : v.  For compatible p, <p, A p>_C0 = sum_x p : C : p
// (Gamma0 C0 is the C0-orthogonal projection on compatible zero-mean fields),
// so the real-space pass supplies it as a by-product.  The equilibrium
// residual of the iterate eps_bar + x is kept exact by linearity: the
// spectral pass updates the traction t = sigma_hat xi of the iterate by
// alpha (C p)^ xi and sums |t|^2, the mean stress follows <sigma> += alpha <C p>.
//
// Fields are in the state layout (per load and component: half spectrum
// along axis 0, the other axes in point order), where point sums are
// Parseval sums: sum_x u v = L0 sum_k w(k) Re(u_k conj v_k), w = 1 at k = 0
// and k = L0/2, 2 elsewhere.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "ahom_internal.h"
#include "ahom_kernels.h"

namespace {

constexpr int kWG = 256;
constexpr int kMaxBlocks = 1024;    // workgroups per load of the vector kernels

template <typename T> struct CT;
template <> struct CT<double> { using t = double2; };
template <> struct CT<float> { using t = float2; };

template <int DIM, int PH> struct NComp { static constexpr int N = Fields<DIM, PH>::N; };

// block-wide fixed-order sum of NV doubles per thread; result in thread 0
template <int NV>
__device__ void cg_block_sum(double* vals, double* scratch) {
    const int tid = threadIdx.x;
    for (int c = 0; c < NV; ++c) scratch[c * kWG + tid] = vals[c];
    __syncthreads();
    for (int off = kWG / 2; off > 0; off >>= 1) {
        if (tid < off)
            for (int c = 0; c < NV; ++c) scratch[c * kWG + tid] += scratch[c * kWG + tid + off];
        __syncthreads();
    }
    if (tid == 0)
        for (int c = 0; c < NV; ++c) vals[c] = scratch[c * kWG];
}

// alpha = <r, r>_C0 / <p, C p> (1 for the start), and the mean stress
// recurrence <sigma> += alpha <C p>
template <int DIM, int PH>
__global__ void __launch_bounds__(kWG) k_cg_alpha(CgArgs a) {
    constexpr int NC = NComp<DIM, PH>::N;
    __shared__ double scratch[(NC + 1) * kWG];
    const int load = blockIdx.x;
    LoadState& st = a.st[load];
    if (st.done) return;
    const int tid = threadIdx.x;
    double v[NC + 1];
    for (int c = 0; c <= NC; ++c) v[c] = 0.0;
    for (int w = tid; w < a.n_real; w += kWG) {
        for (int c = 0; c < NC; ++c) v[c] += a.sig_part[((int64_t)load * a.n_real + w) * NC + c];
        v[NC] += a.en_part[(int64_t)load * a.n_real + w];
    }
    cg_block_sum<NC + 1>(v, scratch);
    if (tid != 0) return;
    CgScalars& g = a.cg[load];
    double al = 1.0;
    if (!a.start) al = (v[NC] > 0.0 && g.rr > 0.0) ? g.rr / v[NC] : 0.0;   // no step once r = 0 exactly
    g.alpha = al;
    g.pcp = v[NC];
    a.alpha[load] = al;
    const double inv_m = 1.0 / (double)a.m;
    for (int c = 0; c < NC; ++c) st.mean[c] = (a.start ? 0.0 : st.mean[c]) + al * v[c] * inv_m;
}

// Start: r = p = q (q = -Gamma0 C eps_bar, the operator output), no x update.
// Update: x += alpha p, r += alpha q (q = -A p).  Both: partial sums of
// <r, r>_C0 per workgroup.  The iteration itself never reads x (the residual
// and the mean stress follow their own recurrences), so with no_x the x
// update and its 3 of the update's 6 field streams are left out.
template <typename T, int DIM, int PH>
__global__ void __launch_bounds__(kWG) k_cg_update(CgArgs a) {
    using C = typename CT<T>::t;
    constexpr int NC = NComp<DIM, PH>::N;
    __shared__ double scratch[kWG];
    const int load = blockIdx.y;
    const LoadState& st = a.st[load];
    if (st.done) return;
    const int par = st.iter & 1;
    const int64_t per_load = (int64_t)NC * a.S;
    C* P = reinterpret_cast<C*>(par ? a.buf1 : a.buf0) + load * per_load;
    const C* Q = reinterpret_cast<const C*>(par ? a.buf0 : a.buf1) + load * per_load;
    C* X = reinterpret_cast<C*>(a.xbuf) + load * per_load;
    C* R = reinterpret_cast<C*>(a.rbuf) + load * per_load;
    const T al = (T)a.cg[load].alpha;
    const double lam0 = a.lam0, two_mu0 = 2.0 * a.mu0;
    double acc = 0.0;
    for (int64_t s = (int64_t)blockIdx.x * kWG + threadIdx.x; s < a.S; s += (int64_t)gridDim.x * kWG) {
        double e = 0.0, trx = 0.0, try_ = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int64_t i = (int64_t)c * a.S + s;
            const C q = Q[i];
            C r;
            if (a.start) {
                r = q;
                P[i] = q;
            } else {
                if (!a.no_x) {
                    const C p = P[i];
                    const C x = X[i];
                    X[i] = C{x.x + al * p.x, x.y + al * p.y};
                }
                const C r0 = R[i];
                r = C{r0.x + al * q.x, r0.y + al * q.y};
            }
            R[i] = r;
            e += field_weight(PH, DIM, c) * ((double)r.x * (double)r.x + (double)r.y * (double)r.y);
            if (c < DIM) { trx += (double)r.x; try_ += (double)r.y; }
        }
        const int64_t k0 = s / a.I;
        const double w = (k0 == 0 || 2 * k0 == a.L0) ? 1.0 : 2.0;
        // r : C0 : r = lambda0 |tr r|^2 + 2 mu0 |r|^2 (elasticity), k0 |r|^2 (conductivity, k0 = mu0)
        acc += w * (PH == PHYS_THERMAL ? a.mu0 * e : two_mu0 * e + lam0 * (trx * trx + try_ * try_));
    }
    cg_block_sum<1>(&acc, scratch);
    if (threadIdx.x == 0) a.rr_part[(int64_t)load * gridDim.x + blockIdx.x] = acc;
}

// <r, r>_C0, beta, the equilibrium residual of the iterate, stop decision
template <int DIM, int PH>
__global__ void __launch_bounds__(kWG) k_cg_reduce(CgArgs a) {
    constexpr int NC = NComp<DIM, PH>::N;
    __shared__ double scratch[2 * kWG];
    const int load = blockIdx.x;
    LoadState& st = a.st[load];
    if (st.done) return;
    const int tid = threadIdx.x;
    double v[2] = {0.0, 0.0};
    for (int w = tid; w < a.nblk; w += kWG) v[0] += a.rr_part[(int64_t)load * a.nblk + w];
    for (int w = tid; w < a.n_spec; w += kWG) v[1] += a.res_part[(int64_t)load * a.n_spec + w];
    cg_block_sum<2>(v, scratch);
    if (tid != 0) return;
    CgScalars& g = a.cg[load];
    const double rr = (double)a.L0 * v[0];
    const bool inner = a.rr_stop > 0.0;
    if (a.start) g.rr0 = rr;
    double r;
    if (inner) {
        // inner solve: the C0 norm of the CG residual relative to its start
        r = g.rr0 > 0.0 ? sqrt(rr / g.rr0) : 0.0;
    } else {
        double fro = 0.0;
        for (int c = 0; c < NC; ++c) fro += field_weight(PH, DIM, c) * st.mean[c] * st.mean[c];
        r = sqrt(v[1]) / sqrt(fro);
    }
    const int n = a.start ? 0 : st.iter + 1;
    if (a.start) {
        g.beta = 0.0;
        st.r0 = r;
    } else {
        g.beta = g.rr > 0.0 ? rr / g.rr : 0.0;
    }
    g.rr = rr;
    if (n < a.hist_cap) a.hist[(int64_t)load * a.hist_cap + n] = r;
    st.resid = r;
    st.iter = n;
    const bool bad = !(r == r) || isinf(r) || (st.r0 > 0.0 && r > 1e3 * st.r0);
    if (bad) { st.done = 1; st.status = 2; return; }
    if (r <= (inner ? a.rr_stop : a.tol)) { st.done = 1; st.status = 0; return; }
    if (n >= a.max_iter) { st.done = 1; st.status = 1; return; }
}

// p(n) = r(n) + beta p(n - 1): from buf[(n - 1) & 1] into buf[n & 1]
template <typename T, int DIM, int PH>
__global__ void __launch_bounds__(kWG) k_cg_direction(CgArgs a) {
    using C = typename CT<T>::t;
    constexpr int NC = NComp<DIM, PH>::N;
    const int load = blockIdx.y;
    const LoadState& st = a.st[load];
    if (st.done) return;
    const int par = st.iter & 1;
    const int64_t per_load = (int64_t)NC * a.S;
    const C* Pold = reinterpret_cast<const C*>(par ? a.buf0 : a.buf1) + load * per_load;
    C* Pnew = reinterpret_cast<C*>(par ? a.buf1 : a.buf0) + load * per_load;
    const C* R = reinterpret_cast<const C*>(a.rbuf) + load * per_load;
    const T be = (T)a.cg[load].beta;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < per_load; i += (int64_t)gridDim.x * kWG) {
        const C r = R[i], p = Pold[i];
        Pnew[i] = C{r.x + be * p.x, r.y + be * p.y};
    }
}

__global__ void __launch_bounds__(kWG) k_cg_demote(const double2* __restrict__ in, float2* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG)
        out[i] = float2{(float)in[i].x, (float)in[i].y};
}

__global__ void __launch_bounds__(kWG) k_cg_sub(double2* __restrict__ x, const double2* __restrict__ d, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG) {
        const double2 v = x[i], w = d[i];
        x[i] = double2{v.x - w.x, v.y - w.y};
    }
}

}  // namespace

int ahom_launch_cg_sub(double2* x, const double2* d, int64_t n, hipStream_t s) {
    int64_t blocks = (n + kWG - 1) / kWG;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_cg_sub, dim3((unsigned)blocks), dim3(kWG), 0, s, x, d, n);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int ahom_launch_cg_demote(const double2* in, float2* out, int64_t n, hipStream_t s) {
    int64_t blocks = (n + kWG - 1) / kWG;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_cg_demote, dim3((unsigned)blocks), dim3(kWG), 0, s, in, out, n);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int ahom_cg_blocks(int64_t S) {
    const int64_t b = (S + kWG - 1) / kWG;
    return (int)(b < kMaxBlocks ? (b < 1 ? 1 : b) : kMaxBlocks);
}

// kernel of the given precision, dimension and physics
#define AHOM_CG_PICK(K, ...)                                                                      \
    (a.phys == PHYS_THERMAL ? (dim == 3 ? K<__VA_ARGS__ 3, PHYS_THERMAL> : K<__VA_ARGS__ 2, PHYS_THERMAL>) \
                            : (dim == 3 ? K<__VA_ARGS__ 3, PHYS_ELASTIC> : K<__VA_ARGS__ 2, PHYS_ELASTIC>))

int ahom_launch_cg_alpha(int dim, const CgArgs& a, int nload, hipStream_t s) {
    hipLaunchKernelGGL(AHOM_CG_PICK(k_cg_alpha, ), dim3(nload), dim3(kWG), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int ahom_launch_cg_update(int prec, int dim, const CgArgs& a, int nload, hipStream_t s) {
    const dim3 grid(a.nblk, nload);
    if (prec == 0) hipLaunchKernelGGL(AHOM_CG_PICK(k_cg_update, double, ), grid, dim3(kWG), 0, s, a);
    else hipLaunchKernelGGL(AHOM_CG_PICK(k_cg_update, float, ), grid, dim3(kWG), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int ahom_launch_cg_reduce(int dim, const CgArgs& a, int nload, hipStream_t s) {
    hipLaunchKernelGGL(AHOM_CG_PICK(k_cg_reduce, ), dim3(nload), dim3(kWG), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int ahom_launch_cg_direction(int prec, int dim, const CgArgs& a, int nload, hipStream_t s) {
    const dim3 grid(a.nblk, nload);
    if (prec == 0) hipLaunchKernelGGL(AHOM_CG_PICK(k_cg_direction, double, ), grid, dim3(kWG), 0, s, a);
    else hipLaunchKernelGGL(AHOM_CG_PICK(k_cg_direction, float, ), grid, dim3(kWG), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
