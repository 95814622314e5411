// C ABI of libahom: patterns (host-only), the bare pattern DFT and the
// Algorithm 1 solver (device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/ahom.h"
#include "ahom_internal.h"
#include "ahom_kernels.h"

namespace {
thread_local std::string g_err;

// a roctx range over the enclosing scope (shown by rocprofv3 --marker-trace)
struct RoctxRange {
    explicit RoctxRange(const char* name) { roctxRangePushA(name); }
    ~RoctxRange() { roctxRangePop(); }
};

constexpr int kLmax = 256;          // longest transform held by one pass
constexpr size_t kLdsCap = 150 * 1024;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return fail(AHOM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

// field index (11,22,33,23,13,12) / (11,22,12) -> position in a 3x3 row-major tensor
const int kComp3[6] = {0, 4, 8, 5, 2, 1};
const int kComp2[3] = {0, 4, 1};
}  // namespace

void ahom_set_error(const std::string& msg) { g_err = msg; }

// ---------------------------------------------------------------------------
// Scratch of the allocation-free pattern DFT (ahom_dft_noalloc): the plan,
// the twiddle tables (FP64 and their FP32 rounding) and one working array of
// up to kScratchMaxPoints complex doubles.  Each GPU holds its own copy from
// load until the process ends; every call on a GPU shares it.  Host code
// never passes the array's name to a kernel: it takes the device address
// from hipGetSymbolAddress once per device (scratch_base below).
constexpr size_t kScratchPlanBytes = 4096;
constexpr size_t kScratchTableBytes = size_t(1) << 20;       // plan + both twiddle tables
constexpr int64_t kScratchMaxPoints = int64_t(1) << 21;
constexpr size_t kScratchBytes = kScratchTableBytes + (size_t)kScratchMaxPoints * 16;
static_assert(sizeof(Plan) <= kScratchPlanBytes, "plan does not fit its scratch slot");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
constexpr int kScratchMaxDevices = 64;
void* g_scratch_ptr[kScratchMaxDevices] = {};

// device address of `scratch` on the current device (resolved once per device)
int scratch_base(void** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchMaxDevices) return fail(AHOM_E_DEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(AHOM_E_DEVICE, "no device address for the DFT scratch");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return AHOM_OK;
}

__global__ void k_twiddles_to_f32(const double2* __restrict__ in, float2* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = float2{(float)in[i].x, (float)in[i].y};
}
}  // namespace

struct DeviceTables {
    int device = -1;
    Plan* plan = nullptr;
    double2* tw64 = nullptr;
    float2* tw32 = nullptr;
};

struct ahom_pattern {
    SmithForm sf;
    Plan plan;
    std::vector<double> tw;
    DeviceTables dev;

    int ensure_device() {
        int cur = 0;
        HIPCHK(hipGetDevice(&cur));
        if (dev.plan && dev.device == cur) return AHOM_OK;
        if (dev.plan) return fail(AHOM_E_DEVICE, "pattern used on a second device");
        HIPCHK(hipMalloc((void**)&dev.plan, sizeof(Plan)));
        HIPCHK(hipMemcpy(dev.plan, &plan, sizeof(Plan), hipMemcpyHostToDevice));
        const size_t n = tw.size() / 2;
        HIPCHK(hipMalloc((void**)&dev.tw64, std::max<size_t>(n, 1) * sizeof(double2)));
        HIPCHK(hipMalloc((void**)&dev.tw32, std::max<size_t>(n, 1) * sizeof(float2)));
        std::vector<float> t32(tw.size());
        for (size_t i = 0; i < tw.size(); ++i) t32[i] = (float)tw[i];
        if (n) {
            HIPCHK(hipMemcpy(dev.tw64, tw.data(), n * sizeof(double2), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(dev.tw32, t32.data(), n * sizeof(float2), hipMemcpyHostToDevice));
        }
        dev.device = cur;
        return AHOM_OK;
    }

    ~ahom_pattern() {
        dfree(dev.plan);
        dfree(dev.tw64);
        dfree(dev.tw32);
    }
};

namespace {

struct PassGeom {
    int NC = 1, CS = 1, nwg = 1;
    size_t lds = 0;
};

// Choose columns per workgroup for a pass over columns of length L.
int choose_geom(int L, int64_t ncols, int nbuf, size_t extra, size_t es, int prec, PassGeom* g) {
    const int target = prec == AHOM_FP64 ? 1024 : 2048;
    int NC = std::max(1, target / L);
    if (ncols < NC) NC = (int)std::max<int64_t>(1, ncols);
    const int CS = L + 1;
    extra += (size_t)L * es;   // LDS copy of the axis's twiddle table
    while (NC > 1 && (size_t)nbuf * NC * CS * es + extra > kLdsCap) NC /= 2;
    size_t lds = (size_t)nbuf * NC * CS * es + extra;
    if (lds > 160 * 1024) return fail(AHOM_E_UNSUPPORTED_SIZE, "transform length too long for one LDS tile");
    g->NC = NC;
    g->CS = CS;
    g->lds = lds;
    g->nwg = (int)((ncols + NC - 1) / NC);
    return AHOM_OK;
}

}  // namespace

struct ahom_solver {
    ahom_pattern* pat = nullptr;
    ahom_config cfg{};
    int prec = 0, dim = 3, ncomp = 6, npack = 3, nt = 3;
    int phys = PHYS_ELASTIC;           // elasticity or conductivity (k and k0 in the Lame slots)
    hipStream_t stream = nullptr;
    // material
    bool has_material = false, ref_set = false;
    int n_phase = 0;
    double lam0 = 0, mu0 = 0;
    double lam_lo = 0, lam_hi = 0, mu_lo = 0, mu_hi = 0;
    uint8_t* d_phase = nullptr;
    uint8_t* d_phase_t = nullptr;      // transposed copies for the real-space pass
    double* d_lame_pts_t = nullptr;
    double* d_lame_tab = nullptr;
    double* d_lame_pts = nullptr;
    // buffers
    int cap = 0;
    void* d_buf0 = nullptr;
    void* d_buf1 = nullptr;
    void* d_tbuf = nullptr;
    LoadState* d_st = nullptr;
    LoadState* h_st = nullptr;
    double* d_sig = nullptr;
    double* d_res = nullptr;
    double* d_hist = nullptr;
    double* d_cau = nullptr;       // [load][wg] Cauchy-measure partial sums
    double* d_chist = nullptr;     // [load][hist_cap] Cauchy measure per iteration
    double* d_norm0 = nullptr;     // [load] |eps(0)| of the plain start
    double* d_epsbar = nullptr;
    double* d_real = nullptr;
    int hist_cap = 0;
    // FP32 defect-correction restarts: an FP64 solver on the same pattern that
    // borrows this solver's material arrays, the FP32 traction offset and the
    // mean stress of the FP64 iterate
    ahom_solver* ref64 = nullptr;
    bool borrowed = false;
    void* d_toff = nullptr;
    double* d_sigbase = nullptr;
    // conjugate gradients (cfg.scheme == AHOM_SCHEME_CG): iterate, residual
    // field, scalars, and the partial sums of <p, C p> and <r, r>_C0
    bool cg = false;
    void* d_x = nullptr;
    void* d_r = nullptr;
    CgScalars* d_cg = nullptr;
    double* d_alpha = nullptr;
    double* d_en = nullptr;
    double* d_rr = nullptr;
    double* d_zero6 = nullptr;     // [load][ncomp] zeros: the mean of the operator output
    // mixed-precision CG: the homogeneous reference medium (all points phase
    // 0, table entry C0) that the FP64 companion projects corrections with
    uint8_t* d_zero_phase = nullptr;
    double* d_c0tab = nullptr;
    int cg_nblk = 1;
    double cg_rr_stop = 0.0;       // > 0: inner solves of the mixed-precision scheme
    bool cg_no_x = false;          // the current CG solve returns no field: x is not formed
    // per-stage settings read by the launches
    double cur_tol = 0.0;
    const void* spec_toff = nullptr;
    void* spec_dout = nullptr;
    void* spec_dneg = nullptr;
    const double* red_sig_base = nullptr;
    // geometry: generic kernels (always available) and the power-of-two fast path
    PassGeom g_real, g_spec, g_axis[AHOM_MAX_AXES];
    bool f_real = false, f_spec = false, f_axis[AHOM_MAX_AXES] = {};
    int fn_real = 0, fn_spec = 0, fn_axis[AHOM_MAX_AXES] = {};   // tiles per load (and field)
    size_t fl_real = 0, fl_spec = 0, fl_axis[AHOM_MAX_AXES] = {}; // LDS bytes per workgroup
    int v_real = 0, v_spec = 0, v_axis[AHOM_MAX_AXES] = {};       // tile variants (autotuned)
    bool tuned = false;
    int ncu = 256;
    bool use_fast = true;
    // tiles per load (and field) of each fast pass for the chosen variants
    void apply_variants() {
        const Plan& P = pat->plan;
        FastGeom fg;
        if (f_real && ahom_fast_geom(prec, FAST_REAL, dim, P.ax[0].len, v_real, &fg, phys)) {
            const int64_t I = P.S / P.ax[0].slen;
            fn_real = (int)((I + fg.NC - 1) / fg.NC);
            fl_real = fg.lds;
        }
        if (f_spec && ahom_fast_geom(prec, FAST_SPEC, dim, P.ax[P.D - 1].len, v_spec, &fg, phys)) {
            const int64_t nc = P.S / P.ax[P.D - 1].len;
            fn_spec = (int)((nc + fg.NC - 1) / fg.NC);
            fl_spec = fg.lds;
        }
        for (int a = 1; a <= P.D - 2; ++a)
            if (f_axis[a] && ahom_fast_geom(prec, FAST_AXIS, dim, P.ax[a].len, v_axis[a], &fg)) {
                int64_t O = 1, I = 1;
                for (int b = 0; b < a; ++b) O *= P.ax[b].slen;
                for (int b = a + 1; b < P.D; ++b) I *= P.ax[b].slen;
                fn_axis[a] = (int)((O * I + fg.NC - 1) / fg.NC);
                fl_axis[a] = fg.lds;
            }
    }
    // largest tile count over all variants (partial-sum buffers)
    int max_tiles(int kind, int L, int64_t ncols) const {
        int best = 1;
        for (int v = 0; v < AHOM_FAST_VARIANTS; ++v) {
            FastGeom fg;
            if (ahom_fast_geom(prec, kind, dim, L, v, &fg, phys)) best = std::max<int>(best, (int)((ncols + fg.NC - 1) / fg.NC));
        }
        return best;
    }
    int autotune(int nload);
    int n_real_wg() const { return f_real ? fn_real : g_real.nwg; }
    int n_spec_wg() const { return f_spec ? fn_spec : g_spec.nwg; }
    // timing
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double last_ms = 0;
    int last_enqueued = 0;
    int last_nload = 0;
    int last_restarts = 0;
    std::vector<int> last_start;       // per load of the last solve: 1 guessed start kept, 0 plain start

    size_t es() const { return prec == AHOM_FP64 ? 16 : 8; }

    int release_buffers() {
        dfree(d_buf0); dfree(d_buf1); dfree(d_tbuf); dfree(d_st); dfree(d_sig);
        dfree(d_res); dfree(d_hist); dfree(d_cau); dfree(d_chist); dfree(d_norm0); dfree(d_epsbar); dfree(d_real); dfree(d_toff); dfree(d_sigbase);
        dfree(d_x); dfree(d_r); dfree(d_cg); dfree(d_alpha); dfree(d_en); dfree(d_rr); dfree(d_zero6);
        if (h_st) (void)hipHostFree(h_st);
        h_st = nullptr;
        cap = 0;
        return AHOM_OK;
    }

    int ensure_real_staging() {
        if (d_real) return AHOM_OK;
        HIPCHK(hipMalloc((void**)&d_real, (size_t)cap * ncomp * pat->plan.m * sizeof(double)));
        return AHOM_OK;
    }

    int ensure_capacity(int nload) {
        if (nload <= cap) return AHOM_OK;
        release_buffers();
        const Plan& P = pat->plan;
        const size_t fb = (size_t)nload * ncomp * P.S * es();
        HIPCHK(hipMalloc(&d_buf0, fb));
        HIPCHK(hipMalloc(&d_buf1, fb));
        HIPCHK(hipMalloc(&d_tbuf, (size_t)nload * nt * P.S * es()));
        HIPCHK(hipMalloc((void**)&d_st, nload * sizeof(LoadState)));
        HIPCHK(hipHostMalloc((void**)&h_st, nload * sizeof(LoadState), hipHostMallocDefault));
        const int mt_real = max_tiles(FAST_REAL, P.ax[0].len, P.S / P.ax[0].slen);
        const int mt_spec = max_tiles(FAST_SPEC, P.ax[P.D - 1].len, P.S / P.ax[P.D - 1].len);
        HIPCHK(hipMalloc((void**)&d_sig, (size_t)nload * std::max(g_real.nwg, mt_real) * ncomp * sizeof(double)));
        HIPCHK(hipMalloc((void**)&d_res, (size_t)nload * std::max(g_spec.nwg, mt_spec) * sizeof(double)));
        HIPCHK(hipMalloc((void**)&d_cau, (size_t)nload * std::max(g_spec.nwg, mt_spec) * sizeof(double)));
        hist_cap = cfg.max_iter + 1;
        HIPCHK(hipMalloc((void**)&d_hist, (size_t)nload * hist_cap * sizeof(double)));
        HIPCHK(hipMalloc((void**)&d_chist, (size_t)nload * hist_cap * sizeof(double)));
        HIPCHK(hipMalloc((void**)&d_norm0, (size_t)nload * sizeof(double)));
        HIPCHK(hipMalloc((void**)&d_epsbar, (size_t)nload * ncomp * sizeof(double)));
        HIPCHK(hipMalloc((void**)&d_sigbase, (size_t)nload * ncomp * sizeof(double)));
        if (prec == AHOM_FP32_MIXED && cfg.refine > 0.0) {
            const size_t tb = (size_t)nload * nt * P.S * sizeof(float2);
            HIPCHK(hipMalloc(&d_toff, tb));
            HIPCHK(hipMemset(d_toff, 0, tb));
        }
        if (cg) {
            cg_nblk = ahom_cg_blocks(P.S);
            HIPCHK(hipMalloc(&d_x, fb));
            HIPCHK(hipMalloc(&d_r, fb));
            HIPCHK(hipMalloc((void**)&d_cg, (size_t)nload * sizeof(CgScalars)));
            HIPCHK(hipMalloc((void**)&d_alpha, (size_t)nload * sizeof(double)));
            HIPCHK(hipMalloc((void**)&d_en, (size_t)nload * std::max(g_real.nwg, mt_real) * sizeof(double)));
            HIPCHK(hipMalloc((void**)&d_rr, (size_t)nload * cg_nblk * sizeof(double)));
            HIPCHK(hipMalloc((void**)&d_zero6, (size_t)nload * ncomp * sizeof(double)));
            HIPCHK(hipMemset(d_zero6, 0, (size_t)nload * ncomp * sizeof(double)));
        }
        cap = nload;
        return AHOM_OK;
    }

    ~ahom_solver() {
        release_buffers();
        delete ref64;
        if (borrowed) {
            d_phase = d_phase_t = nullptr;
            d_lame_tab = d_lame_pts = d_lame_pts_t = nullptr;
        }
        dfree(d_phase); dfree(d_lame_tab); dfree(d_lame_pts); dfree(d_phase_t); dfree(d_lame_pts_t);
        dfree(d_zero_phase); dfree(d_c0tab);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
    }

    RealArgs real_args(int mode) const {
        RealArgs a{};
        a.phys = phys;
        a.plan = pat->dev.plan;
        a.buf0 = d_buf0;
        a.buf1 = d_buf1;
        a.tw = prec == AHOM_FP64 ? (const void*)pat->dev.tw64 : (const void*)pat->dev.tw32;
        a.tw64 = pat->dev.tw64;
        a.st = d_st;
        a.phase = d_phase;
        a.lame_tab = d_lame_tab;
        a.lame_pts = d_lame_pts;
        a.phase_t = d_phase_t;
        a.lame_pts_t = d_lame_pts_t;
        a.n_phase = d_lame_pts_t ? 0 : n_phase;
        // conjugate gradients apply C itself (reference constants zero) and
        // collect <p, C p>
        a.lam0 = cg ? 0.0 : lam0;
        a.mu0 = cg ? 0.0 : mu0;
        a.en_part = cg ? d_en : nullptr;
        a.sig_part = d_sig;
        a.real_io = d_real;
        a.eps_bar = d_epsbar;
        a.NC = g_real.NC;
        a.CS = g_real.CS;
        (void)mode;
        return a;
    }

    AxisArgs axis_args(int axis) const {
        AxisArgs a{};
        a.plan = pat->dev.plan;
        a.buf0 = d_buf0;
        a.buf1 = d_buf1;
        a.tw = prec == AHOM_FP64 ? (const void*)pat->dev.tw64 : (const void*)pat->dev.tw32;
        a.tw64 = pat->dev.tw64;
        a.st = d_st;
        a.load_stride = (int64_t)ncomp * pat->plan.S;
        a.field_stride = pat->plan.S;
        a.axis = axis;
        a.slen0_full = 0;
        a.NC = g_axis[axis].NC;
        a.CS = g_axis[axis].CS;
        return a;
    }

    SpecArgs spec_args() const {
        SpecArgs a{};
        a.phys = phys;
        a.plan = pat->dev.plan;
        a.buf0 = d_buf0;
        a.buf1 = d_buf1;
        a.tbuf = d_tbuf;
        a.tw = prec == AHOM_FP64 ? (const void*)pat->dev.tw64 : (const void*)pat->dev.tw32;
        a.st = d_st;
        a.eps_bar = d_epsbar;
        a.mu0 = mu0;
        a.beta = (lam0 + mu0) / (lam0 + 2.0 * mu0);
        a.res_part = d_res;
        a.cau_part = d_cau;
        a.NC = g_spec.NC;
        a.CS = g_spec.CS;
        a.resid_period = cfg.resid_period;
        a.max_iter = cfg.max_iter;
        a.toff = spec_toff;
        a.dout = spec_dout;
        a.dneg = spec_dneg;
        if (cg) {
            // operator output of zero mean, traction recurrence every iteration
            a.eps_bar = d_zero6;
            a.cg_alpha = d_alpha;
            a.resid_period = 1;
        }
        return a;
    }

    int launch_real_turn(int nload, hipStream_t s) {
        if (f_real) {
            RealArgs ra = real_args(REAL_TURN);
            ra.nload = nload;
            return ahom_launch_fast_real(prec, dim, pat->plan.ax[0].len, v_real, ra, (int64_t)fn_real * nload, ncu, s);
        }
        return ahom_launch_real(prec, dim, REAL_TURN, real_args(REAL_TURN), g_real.nwg, nload, g_real.lds, s);
    }
    int launch_axis(int a, int dir, int nload, hipStream_t s) {
        if (f_axis[a]) {
            AxisArgs aa = axis_args(a);
            aa.nload = nload;
            aa.nfield = ncomp;
            return ahom_launch_fast_axis(prec, dir, pat->plan.ax[a].len, v_axis[a], aa, (int64_t)fn_axis[a] * ncomp * nload, ncu, s);
        }
        return ahom_launch_axis(prec, dir, axis_args(a), g_axis[a].nwg, ncomp, nload, g_axis[a].lds, s);
    }
    int launch_spec(int nload, hipStream_t s) {
        if (f_spec) {
            SpecArgs sa = spec_args();
            sa.nload = nload;
            return ahom_launch_fast_spec(prec, dim, pat->plan.ax[pat->plan.D - 1].len, v_spec, sa, (int64_t)fn_spec * nload, ncu, s);
        }
        return ahom_launch_spec(prec, dim, spec_args(), g_spec.nwg, nload, g_spec.lds, s);
    }

    int enqueue_iteration(int nload) {
        const Plan& P = pat->plan;
        hipStream_t s = stream;
        if (launch_real_turn(nload, s)) return fail(AHOM_E_DEVICE, "launch real-space pass failed");
        for (int a = 1; a <= P.D - 2; ++a)
            if (launch_axis(a, -1, nload, s)) return fail(AHOM_E_DEVICE, "launch axis pass failed");
        if (launch_spec(nload, s)) return fail(AHOM_E_DEVICE, "launch spectral pass failed");
        for (int a = P.D - 2; a >= 1; --a)
            if (launch_axis(a, +1, nload, s)) return fail(AHOM_E_DEVICE, "launch axis pass failed");
        ReduceArgs r{};
        r.phys = phys;
        r.st = d_st;
        r.sig_part = d_sig;
        r.res_part = d_res;
        r.hist = d_hist;
        r.n_real = n_real_wg();
        r.n_spec = n_spec_wg();
        r.hist_cap = hist_cap;
        r.m = P.m;
        r.tol = cur_tol;
        r.max_iter = cfg.max_iter;
        r.resid_period = cfg.resid_period;
        r.sig_base = red_sig_base;
        r.cau_part = d_cau;
        r.chist = d_chist;
        r.norm0 = d_norm0;
        // |eps(n+1) - eps(n)|^2 = m sum |delta eps_hat|^2: 1/(2 mu0^2) of the kernel sums in
        // elasticity, 1/k0^2 for conductivity (k0 in mu0)
        r.cau_scale = (double)P.m / ((phys == PHYS_THERMAL ? 1.0 : 2.0) * mu0 * mu0);
        r.stop_cauchy = cfg.stop_rule == AHOM_STOP_CAUCHY;
        if (ahom_launch_reduce(dim, r, nload, s)) return fail(AHOM_E_DEVICE, "launch k_reduce failed");
        return AHOM_OK;
    }
};

// ------------------------------------------------------- conjugate gradients
// One CG update per load (see ahom_cg.hip): the operator sweep on the
// direction p(n) (buf[n & 1] -> -A p(n) in buf[(n + 1) & 1]), alpha, the
// vector update of x and r, <r, r>_C0, beta and the stop test, the new
// direction.  With start = 1: the sweep on eps_bar gives r(0) = p(0) and the
// residual r(0) of eps_bar.
namespace {
int cg_sweep(ahom_solver* s, int nload, int start) {
    const Plan& P = s->pat->plan;
    hipStream_t st = s->stream;
    CgArgs c{};
    c.phys = s->phys;
    c.st = s->d_st;
    c.cg = s->d_cg;
    c.alpha = s->d_alpha;
    c.buf0 = s->d_buf0;
    c.buf1 = s->d_buf1;
    c.xbuf = s->d_x;
    c.rbuf = s->d_r;
    c.sig_part = s->d_sig;
    c.en_part = s->d_en;
    c.res_part = s->d_res;
    c.rr_part = s->d_rr;
    c.hist = s->d_hist;
    c.n_real = s->n_real_wg();
    c.n_spec = s->n_spec_wg();
    c.nblk = s->cg_nblk;
    c.hist_cap = s->hist_cap;
    c.S = P.S;
    c.I = P.S / P.ax[0].slen;
    c.m = P.m;
    c.L0 = P.ax[0].len;
    c.lam0 = s->lam0;
    c.mu0 = s->mu0;
    c.tol = s->cfg.tol;
    c.max_iter = s->cfg.max_iter;
    c.start = start;
    c.rr_stop = s->cg_rr_stop;
    c.no_x = s->cg_no_x ? 1 : 0;
    if (start == 2) {
        // start of an inner solve from a given residual field r(0), stored
        // in buf1: r = p = r(0), <r, r>_C0 (no operator sweep)
        c.start = 1;
        if (ahom_launch_cg_update(s->prec, s->dim, c, nload, st)) return fail(AHOM_E_DEVICE, "launch k_cg_update failed");
        if (ahom_launch_cg_reduce(s->dim, c, nload, st)) return fail(AHOM_E_DEVICE, "launch k_cg_reduce failed");
        return AHOM_OK;
    }
    if (s->launch_real_turn(nload, st)) return fail(AHOM_E_DEVICE, "launch real-space pass failed");
    if (ahom_launch_cg_alpha(s->dim, c, nload, st)) return fail(AHOM_E_DEVICE, "launch k_cg_alpha failed");
    for (int a = 1; a <= P.D - 2; ++a)
        if (s->launch_axis(a, -1, nload, st)) return fail(AHOM_E_DEVICE, "launch axis pass failed");
    if (s->launch_spec(nload, st)) return fail(AHOM_E_DEVICE, "launch spectral pass failed");
    for (int a = P.D - 2; a >= 1; --a)
        if (s->launch_axis(a, +1, nload, st)) return fail(AHOM_E_DEVICE, "launch axis pass failed");
    if (ahom_launch_cg_update(s->prec, s->dim, c, nload, st)) return fail(AHOM_E_DEVICE, "launch k_cg_update failed");
    if (ahom_launch_cg_reduce(s->dim, c, nload, st)) return fail(AHOM_E_DEVICE, "launch k_cg_reduce failed");
    if (!start && ahom_launch_cg_direction(s->prec, s->dim, c, nload, st))
        return fail(AHOM_E_DEVICE, "launch k_cg_direction failed");
    return AHOM_OK;
}
}  // namespace

// ---------------------------------------------------------------- autotuner
// Times every compiled tile variant of each power-of-two pass on the solver's
// own buffers and keeps the fastest.  Results are cached per process by
// (pass, precision, dimension, length, columns, loads), so later solvers of
// the same shape reuse them without timing.
namespace {
struct TuneKey {
    int kind, prec, dim, L, axis, nload;
    int64_t ncols;
    int phys;
    bool operator<(const TuneKey& o) const {
        return std::tie(kind, prec, dim, L, axis, nload, ncols, phys) <
               std::tie(o.kind, o.prec, o.dim, o.L, o.axis, o.nload, o.ncols, o.phys);
    }
};
std::map<TuneKey, int>& tune_cache() {
    static std::map<TuneKey, int> c;
    return c;
}
std::mutex& tune_mutex() {
    static std::mutex m;
    return m;
}
}  // namespace

int ahom_solver::autotune(int nload) {
    if (tuned || !use_fast) {
        if ((cg || phys != PHYS_ELASTIC) && v_real == 4) { v_real = 0; apply_variants(); }
        return AHOM_OK;
    }
    const Plan& P = pat->plan;
    hipStream_t st = stream;
    const char* venv = getenv("AHOM_VERBOSE");
    const bool verbose = venv && venv[0] == '1';
    if (ahom_launch_reset(d_st, nload, st)) return fail(AHOM_E_DEVICE, "reset");
    auto time_pass = [&](auto&& launch, float* best_ms) -> int {
        // one warm launch, then the minimum of three timed launches
        if (launch()) return -1;
        float best = 1e30f;
        for (int r = 0; r < 3; ++r) {
            if (hipEventRecord(ev0, st) != hipSuccess) return -1;
            if (launch()) return -1;
            if (hipEventRecord(ev1, st) != hipSuccess || hipEventSynchronize(ev1) != hipSuccess) return -1;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev0, ev1) != hipSuccess) return -1;
            best = std::min(best, ms);
        }
        *best_ms = best;
        return 0;
    };
    auto tune_one = [&](int kind, int L, int axis, int64_t ncols, int* vsel, auto&& launch_v) -> int {
        TuneKey key{kind, prec, dim, L, axis, nload, ncols, phys};
        {
            std::lock_guard<std::mutex> g(tune_mutex());
            auto it = tune_cache().find(key);
            if (it != tune_cache().end()) { *vsel = it->second; return AHOM_OK; }
        }
        int best_v = 0;
        float best = 1e30f;
        std::vector<FastGeom> seen;
        for (int v = 0; v < AHOM_FAST_VARIANTS; ++v) {
            FastGeom fg;
            if (!ahom_fast_geom(prec, kind, dim, L, v, &fg, phys)) continue;
            bool dup = false;
            // same launch shape = same kernel work (the register-resident
            // real pass can report the column count of another variant)
            for (auto& o : seen)
                dup = dup || (o.NC == fg.NC && o.persistent == fg.persistent && o.threads == fg.threads && o.lds == fg.lds);
            if (dup) continue;
            seen.push_back(fg);
            // the register-resident variant has neither <p, C p> sums nor the conductivity law
            if ((cg || phys != PHYS_ELASTIC) && kind == FAST_REAL && v == 4) continue;
            *vsel = v;
            apply_variants();
            float ms = 0.f;
            if (time_pass([&]() { return launch_v(); }, &ms)) return fail(AHOM_E_DEVICE, "autotune launch failed");
            if (verbose)
                fprintf(stderr, "[ahom tune] pass %d L %d axis %d variant %d (NC %d, %s): %.4f ms\n", kind, L, axis, v, fg.NC,
                        fg.persistent ? "persistent" : "one tile per WG", ms);
            if (ms < best) { best = ms; best_v = v; }
        }
        *vsel = best_v;
        apply_variants();
        std::lock_guard<std::mutex> g(tune_mutex());
        tune_cache()[key] = best_v;
        return AHOM_OK;
    };
    int rc;
    if (f_real && (rc = tune_one(FAST_REAL, P.ax[0].len, 0, P.S / P.ax[0].slen, &v_real, [&]() { return launch_real_turn(nload, st); }))) return rc;
    for (int a = 1; a <= P.D - 2; ++a) {
        int64_t O = 1, I = 1;
        for (int b = 0; b < a; ++b) O *= P.ax[b].slen;
        for (int b = a + 1; b < P.D; ++b) I *= P.ax[b].slen;
        if (f_axis[a] && (rc = tune_one(FAST_AXIS, P.ax[a].len, a, O * I, &v_axis[a], [&]() { return launch_axis(a, -1, nload, st); }))) return rc;
    }
    if (f_spec && (rc = tune_one(FAST_SPEC, P.ax[P.D - 1].len, P.D - 1, P.S / P.ax[P.D - 1].len, &v_spec, [&]() { return launch_spec(nload, st); }))) return rc;
    if ((cg || phys != PHYS_ELASTIC) && v_real == 4) v_real = 0;   // a cached or pinned choice of another solver
    apply_variants();  // tile counts must follow the chosen variants (also on cache hits)
    tuned = true;
    return AHOM_OK;
}

// ============================================================================ API
namespace {
int create_solver(ahom_pattern* p, const ahom_config* cfg, ahom_solver** out) {
    *out = nullptr;
    if (p->sf.m < 2) return fail(AHOM_E_ARG, "trivial pattern (m = 1): the strain is eps_bar");
    int rc = p->ensure_device();
    if (rc) return rc;
    ahom_solver* s = new (std::nothrow) ahom_solver();
    if (!s) return fail(AHOM_E_NOMEM, "host allocation failed");
    s->pat = p;
    s->cfg = *cfg;
    s->cur_tol = cfg->tol;
    // default restart factor: 1e-3 for the Basic Scheme's FP32 stages; CG
    // restarts lose the Krylov space, so its FP32 solves of elasticity run
    // longer (1e-4: fewest updates in total on the 128^3 Hashin and
    // contrast-100 sphere cells; the conductivity cell does best at 1e-3)
    if (s->cfg.refine == 0.0)
        s->cfg.refine = cfg->scheme == AHOM_SCHEME_CG && cfg->physics != AHOM_CONDUCTIVITY ? 1e-4 : 1e-3;
    if (s->cfg.check_period < 1) s->cfg.check_period = 1;
    if (s->cfg.resid_period < 1) s->cfg.resid_period = 1;
    s->prec = cfg->precision;
    s->dim = p->sf.d;
    s->phys = cfg->physics == AHOM_CONDUCTIVITY ? PHYS_THERMAL : PHYS_ELASTIC;
    s->ncomp = s->phys == PHYS_THERMAL ? s->dim : (s->dim == 3 ? 6 : 3);
    s->npack = (s->ncomp + 1) / 2;
    s->nt = s->phys == PHYS_THERMAL ? 1 : s->dim;
    s->stream = (hipStream_t)cfg->stream;
    s->cg = cfg->scheme == AHOM_SCHEME_CG;
    const Plan& P = p->plan;
    const size_t es = s->es();
    auto bad = [&](int code) { delete s; return code; };
    if ((rc = choose_geom(P.ax[0].len, P.S / P.ax[0].slen, 2 * s->npack, (size_t)(s->ncomp + 1) * AHOM_WG * 8, es, s->prec, &s->g_real))) return bad(rc);
    if ((rc = choose_geom(P.ax[P.D - 1].len, P.S / P.ax[P.D - 1].len, 2 * s->ncomp, (size_t)2 * AHOM_WG * 8, es, s->prec, &s->g_spec))) return bad(rc);
    for (int a = 1; a <= P.D - 2; ++a) {
        int64_t O = 1, I = 1;
        for (int b = 0; b < a; ++b) O *= P.ax[b].slen;
        for (int b = a + 1; b < P.D; ++b) I *= P.ax[b].slen;
        if ((rc = choose_geom(P.ax[a].len, O * I, 2, 0, es, s->prec, &s->g_axis[a]))) return bad(rc);
    }
    {
        const char* env = getenv("AHOM_GENERIC_ONLY");
        s->use_fast = !(env && env[0] == '1');
    }
    {
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            int n = 0;
            if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0) s->ncu = n;
        }
    }
    if (s->use_fast) {
        FastGeom fg;
        if (ahom_fast_geom(s->prec, FAST_REAL, s->dim, P.ax[0].len, 0, &fg, s->phys)) s->f_real = true;
        if (ahom_fast_geom(s->prec, FAST_SPEC, s->dim, P.ax[P.D - 1].len, 0, &fg, s->phys)) s->f_spec = true;
        for (int a = 1; a <= P.D - 2; ++a)
            if (ahom_fast_geom(s->prec, FAST_AXIS, s->dim, P.ax[a].len, 0, &fg)) s->f_axis[a] = true;
        const char* venv = getenv("AHOM_FAST_VARIANT");
        if (venv && venv[0] >= '0' && venv[0] <= '4') {
            const int v = venv[0] - '0';
            FastGeom fg4;
            const bool rr_ok = ahom_fast_geom(s->prec, FAST_REAL, s->dim, P.ax[0].len, v, &fg4, s->phys);
            s->v_real = rr_ok ? v : 0;          // variant 4 exists for the real-space pass only
            FastGeom fgs;
            s->v_spec = (v < 4 || ahom_fast_geom(s->prec, FAST_SPEC, s->dim, P.ax[P.D - 1].len, v, &fgs, s->phys)) ? v : 0;
            for (int a = 0; a < AHOM_MAX_AXES; ++a) s->v_axis[a] = v < 4 ? v : 0;
            s->tuned = true;
        }
        // per-pass pin "real,spec,axis" (profiling runs that must execute the
        // kernels another run tuned); a variant a pass lacks falls back to 0
        const char* penv = getenv("AHOM_FAST_VARIANTS");
        int vr = -1, vs = -1, va = -1;
        if (penv && std::sscanf(penv, "%d,%d,%d", &vr, &vs, &va) == 3 && vr >= 0 && vr <= 4 && vs >= 0 && vs <= 4 &&
            va >= 0 && va <= 3) {
            FastGeom fgp;
            s->v_real = ahom_fast_geom(s->prec, FAST_REAL, s->dim, P.ax[0].len, vr, &fgp, s->phys) ? vr : 0;
            s->v_spec = vs;
            for (int a = 0; a < AHOM_MAX_AXES; ++a) s->v_axis[a] = va;
            s->tuned = true;
        }
        s->apply_variants();
    }
    if (hipEventCreate(&s->ev0) != hipSuccess || hipEventCreate(&s->ev1) != hipSuccess)
        return bad(fail(AHOM_E_DEVICE, "event create"));
    *out = s;
    return AHOM_OK;
}

// FP64 companion of an FP32 solver for the defect-correction restarts: two
// updates per restart, no stop on the residual, the parent's material arrays
int ensure_ref64(ahom_solver* s, int nload) {
    if (!s->ref64) {
        ahom_config c = s->cfg;
        c.precision = AHOM_FP64;
        c.max_iter = 1;
        c.resid_period = 1;
        c.check_period = 2;
        c.refine = -1.0;
        int rc = create_solver(s->pat, &c, &s->ref64);
        if (rc) return rc;
        s->ref64->borrowed = true;
        s->ref64->cur_tol = -1.0;
    }
    ahom_solver* r = s->ref64;
    r->d_phase = s->d_phase;
    r->d_phase_t = s->d_phase_t;
    r->d_lame_tab = s->d_lame_tab;
    r->d_lame_pts = s->d_lame_pts;
    r->d_lame_pts_t = s->d_lame_pts_t;
    r->n_phase = s->n_phase;
    r->lam0 = s->lam0;
    r->mu0 = s->mu0;
    r->has_material = true;
    int rc = r->ensure_capacity(nload);
    if (rc) return rc;
    return r->autotune(nload);
}

// The homogeneous reference medium of solver s (every point phase 0, table
// entry C0 = (lambda0, mu0), or (k0, k0) for conductivity), in which a CG start
// sweep is the projection: r = -Gamma0 C0 buf0 = -P buf0.
int ensure_c0_medium(ahom_solver* s) {
    if (!s->d_zero_phase) {
        HIPCHK(hipMalloc((void**)&s->d_zero_phase, (size_t)s->pat->sf.m));
        HIPCHK(hipMemset(s->d_zero_phase, 0, (size_t)s->pat->sf.m));
        HIPCHK(hipMalloc((void**)&s->d_c0tab, 2 * sizeof(double)));
    }
    const double c0[2] = {s->lam0, s->mu0};
    HIPCHK(hipMemcpy(s->d_c0tab, c0, sizeof c0, hipMemcpyHostToDevice));
    return AHOM_OK;
}

// r->d_r = -P (r->d_buf0): one FP64 CG start sweep of r in the reference
// medium of `owner` (r's own material pointers are restored afterwards).
// Clobbers r's state, traction and buf1.
int project_sweep(ahom_solver* owner, ahom_solver* r, int n_load) {
    const Plan& P = r->pat->plan;
    hipStream_t st = r->stream;
    uint8_t* sv_ph = r->d_phase;
    uint8_t* sv_pht = r->d_phase_t;
    double* sv_tab = r->d_lame_tab;
    double* sv_pts = r->d_lame_pts;
    double* sv_ptst = r->d_lame_pts_t;
    const int sv_np = r->n_phase;
    const bool sv_nox = r->cg_no_x;
    r->d_phase = r->d_phase_t = owner->d_zero_phase;
    r->d_lame_tab = owner->d_c0tab;
    r->d_lame_pts = r->d_lame_pts_t = nullptr;
    r->n_phase = 1;
    r->cg_no_x = true;
    int rc = ahom_launch_reset(r->d_st, n_load, st) || ahom_launch_zero(AHOM_FP64, r->d_tbuf, (int64_t)n_load * r->nt * P.S, st)
                 ? fail(AHOM_E_DEVICE, "reset")
                 : cg_sweep(r, n_load, 1);
    r->d_phase = sv_ph;
    r->d_phase_t = sv_pht;
    r->d_lame_tab = sv_tab;
    r->d_lame_pts = sv_pts;
    r->d_lame_pts_t = sv_ptst;
    r->n_phase = sv_np;
    r->cg_no_x = sv_nox;
    return rc;
}

// CG start from a guess: the FP64 iterate r->d_x = eps_bar + P init (init:
// the fluctuation, component-major per load, host or device doubles).  Only
// the compatible zero-mean part of a guess is a CG iterate, so the guess is
// projected first (any field is accepted).  stage: solver whose real-space
// staging buffer takes a host init.
int cg_start_from_init(ahom_solver* owner, ahom_solver* r, ahom_solver* stage, int n_load, const void* init,
                       int mem_flags) {
    const Plan& P = r->pat->plan;
    const int nc = r->ncomp;
    hipStream_t st = r->stream;
    int rc;
    if ((rc = ensure_c0_medium(owner))) return rc;
    RealArgs fr = r->real_args(REAL_FROM_REAL);      // buf0 = state of eps_bar + init
    fr.buf0 = fr.buf1 = r->d_buf0;
    if (mem_flags == AHOM_MEM_DEVICE) {
        fr.real_io = const_cast<double*>(static_cast<const double*>(init));
    } else {
        if ((rc = stage->ensure_real_staging())) return rc;
        HIPCHK(hipMemcpyAsync(stage->d_real, init, (size_t)n_load * nc * P.m * sizeof(double), hipMemcpyHostToDevice, st));
        fr.real_io = stage->d_real;
    }
    if (ahom_launch_real(AHOM_FP64, r->dim, REAL_FROM_REAL, fr, r->g_real.nwg, n_load, r->g_real.lds, st))
        return fail(AHOM_E_DEVICE, "launch from_real");
    if ((rc = project_sweep(owner, r, n_load))) return rc;
    if (ahom_launch_cg_sub(static_cast<double2*>(r->d_x), static_cast<const double2*>(r->d_r), (int64_t)n_load * nc * P.S, st))
        return fail(AHOM_E_DEVICE, "launch cg sub");
    return AHOM_OK;
}

int solve_cg_mixed(ahom_solver* s, int n_load, const double* ebc, const void* init, void* strain_out, int* iters,
                   double* resid, double* mean_out, int mem_flags);

// Conjugate gradients for n_load strains (cfg.scheme == AHOM_SCHEME_CG).
int solve_cg(ahom_solver* s, int n_load, const double* ebc, const void* init, void* strain_out, int* iters,
             double* resid, double* mean_out, int mem_flags) {
    if (s->prec == AHOM_FP32_MIXED)
        return solve_cg_mixed(s, n_load, ebc, init, strain_out, iters, resid, mean_out, mem_flags);
    int rc = s->ensure_capacity(n_load);
    if (rc) return rc;
    s->spec_toff = nullptr;
    s->spec_dout = s->spec_dneg = nullptr;
    s->red_sig_base = nullptr;
    s->cur_tol = s->cfg.tol;
    if ((rc = s->autotune(n_load))) return rc;
    const Plan& P = s->pat->plan;
    const int nc = s->ncomp;
    hipStream_t st = s->stream;
    HIPCHK(hipMemcpyAsync(s->d_epsbar, ebc, (size_t)n_load * nc * sizeof(double), hipMemcpyHostToDevice, st));
    if (ahom_launch_reset(s->d_st, n_load, st)) return fail(AHOM_E_DEVICE, "reset");
    if (ahom_launch_zero(s->prec, s->d_tbuf, (int64_t)n_load * s->nt * P.S, st)) return fail(AHOM_E_DEVICE, "zero");
    FillArgs f{};
    f.eps_bar = s->d_epsbar;
    f.S = P.S;
    f.row = P.S / P.ax[0].slen;
    f.nfield = nc;
    f.buf = s->d_x;                    // x(0) = 0: the iterate eps_bar
    if (ahom_launch_fill(s->prec, f, n_load, st)) return fail(AHOM_E_DEVICE, "fill");
    HIPCHK(hipEventRecord(s->ev0, st));
    if (init) {                        // x(0) = P init
        if ((rc = cg_start_from_init(s, s, s, n_load, init, mem_flags))) return rc;
        if (ahom_launch_reset(s->d_st, n_load, st)) return fail(AHOM_E_DEVICE, "reset");
        if (ahom_launch_zero(s->prec, s->d_tbuf, (int64_t)n_load * s->nt * P.S, st)) return fail(AHOM_E_DEVICE, "zero");
    }
    // the start's operator input: the iterate
    HIPCHK(hipMemcpyAsync(s->d_buf0, s->d_x, (size_t)n_load * nc * P.S * s->es(), hipMemcpyDeviceToDevice, st));
    // C_eff alone (no field asked) needs only the residual and mean-stress
    // recurrences: the iterate is then not formed
    s->cg_no_x = strain_out == nullptr;
    if ((rc = cg_sweep(s, n_load, 1))) { s->cg_no_x = false; return rc; }
    int enq = 1;
    const int limit = s->cfg.max_iter + 1;
    bool all_done = false;
    while (!all_done) {
        HIPCHK(hipMemcpyAsync(s->h_st, s->d_st, n_load * sizeof(LoadState), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        all_done = true;
        for (int l = 0; l < n_load; ++l) all_done = all_done && s->h_st[l].done;
        if (all_done) break;
        if (enq > limit + 2 * s->cfg.check_period) return fail(AHOM_E_DEVICE, "loop control did not terminate");
        const int k = std::min(s->cfg.check_period, std::max(1, limit - enq + 1));
        for (int i = 0; i < k; ++i) {
            if ((rc = cg_sweep(s, n_load, 0))) { s->cg_no_x = false; return rc; }
            ++enq;
        }
    }
    s->cg_no_x = false;
    float ms = 0.f;
    HIPCHK(hipEventRecord(s->ev1, st));
    HIPCHK(hipEventSynchronize(s->ev1));
    HIPCHK(hipEventElapsedTime(&ms, s->ev0, s->ev1));
    s->last_ms = ms;
    s->last_enqueued = enq;
    s->last_nload = n_load;
    s->last_restarts = 0;
    s->last_start.assign(n_load, 0);
    if (strain_out) {
        if (mem_flags != AHOM_MEM_DEVICE && (rc = s->ensure_real_staging())) return rc;
        RealArgs ra = s->real_args(REAL_TO_REAL);
        ra.buf0 = ra.buf1 = s->d_x;
        ra.real_io = mem_flags == AHOM_MEM_DEVICE ? static_cast<double*>(strain_out) : s->d_real;
        if (ahom_launch_real(s->prec, s->dim, REAL_TO_REAL, ra, s->g_real.nwg, n_load, s->g_real.lds, st))
            return fail(AHOM_E_DEVICE, "launch to_real");
        if (mem_flags != AHOM_MEM_DEVICE)
            HIPCHK(hipMemcpyAsync(strain_out, s->d_real, (size_t)n_load * nc * P.m * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    int ret = AHOM_OK;
    for (int l = 0; l < n_load; ++l) {
        const LoadState& ls = s->h_st[l];
        if (iters) iters[l] = ls.iter;
        if (resid) resid[l] = ls.resid;
        if (mean_out)
            for (int c = 0; c < nc; ++c) mean_out[(size_t)l * nc + c] = ls.mean[c];
        if (ls.status == 2) ret = AHOM_E_DIVERGED;
        else if (ls.status == 1 && ret == AHOM_OK) ret = AHOM_W_NOT_CONVERGED;
    }
    if (ret == AHOM_E_DIVERGED) g_err = "residual diverged";
    return ret;
}

// Mixed precision CG (AHOM_FP32_MIXED): defect correction with FP32 inner
// CG solves.  The FP64 iterate eps_b (the FP64 companion's x buffer) gets
// its exact residual field r_b = -A eps_b, equilibrium residual and mean
// stress from one FP64 operator sweep (the companion's CG start on eps_b);
// an FP32 CG solve of A e = r_b from e = 0, stopped when its residual has
// dropped by `refine` in the C0 norm, gives the correction, eps_b += P e with
// P the projection onto compatible zero-mean fields (one more FP64 sweep);
// until the FP64 equilibrium residual of eps_b meets tol.  n counts the FP32
// updates; the FP64 sweeps are the restarts.
int solve_cg_mixed(ahom_solver* s, int n_load, const double* ebc, const void* init, void* strain_out, int* iters,
                   double* resid, double* mean_out, int mem_flags) {
    int rc = s->ensure_capacity(n_load);
    if (rc) return rc;
    s->spec_toff = nullptr;
    s->spec_dout = s->spec_dneg = nullptr;
    s->red_sig_base = nullptr;
    if ((rc = s->autotune(n_load))) return rc;
    if ((rc = ensure_ref64(s, n_load))) return rc;
    ahom_solver* r = s->ref64;
    const Plan& P = s->pat->plan;
    const int nc = s->ncomp;
    const size_t per = (size_t)nc * P.S;
    // the reference medium C0 of this solve (stiffness or conductivity)
    if ((rc = ensure_c0_medium(s))) return rc;
    hipStream_t st = s->stream;
    HIPCHK(hipMemcpyAsync(r->d_epsbar, ebc, (size_t)n_load * nc * sizeof(double), hipMemcpyHostToDevice, st));
    FillArgs f{};
    f.eps_bar = r->d_epsbar;
    f.S = P.S;
    f.row = P.S / P.ax[0].slen;
    f.nfield = nc;
    f.buf = r->d_x;                    // eps_b = eps_bar
    if (ahom_launch_fill(AHOM_FP64, f, n_load, st)) return fail(AHOM_E_DEVICE, "fill");
    std::vector<LoadState> fin(n_load);            // FP64 result per load (resid, mean, status)
    std::vector<int> done(n_load, 0), nupd(n_load, 0);
    std::vector<std::vector<std::pair<int, double>>> hrec(n_load);   // (updates so far, FP64 residual) per sweep
    int nrestart = 0, total = 0;
    HIPCHK(hipEventRecord(s->ev0, st));
    if (init && (rc = cg_start_from_init(s, r, s, n_load, init, mem_flags))) return rc;   // eps_b = eps_bar + P init
    for (;;) {
        // FP64 sweep on eps_b: r_b, its traction, residual and mean stress
        HIPCHK(hipMemcpyAsync(r->d_buf0, r->d_x, (size_t)n_load * per * 16, hipMemcpyDeviceToDevice, st));
        if (ahom_launch_reset(r->d_st, n_load, st)) return fail(AHOM_E_DEVICE, "reset");
        if (ahom_launch_zero(AHOM_FP64, r->d_tbuf, (int64_t)n_load * r->nt * P.S, st)) return fail(AHOM_E_DEVICE, "zero");
        if ((rc = cg_sweep(r, n_load, 1))) return rc;
        HIPCHK(hipMemcpyAsync(r->h_st, r->d_st, n_load * sizeof(LoadState), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        bool all = true;
        for (int l = 0; l < n_load; ++l) {
            if (done[l]) continue;
            LoadState ls = r->h_st[l];
            hrec[l].emplace_back(nupd[l], ls.resid);
            const bool bad = !(ls.resid == ls.resid) || std::isinf(ls.resid);
            ls.iter = nupd[l];
            if (bad) { ls.status = 2; done[l] = 1; }
            else if (ls.resid <= s->cfg.tol) { ls.status = 0; done[l] = 1; }
            else if (nupd[l] >= s->cfg.max_iter) { ls.status = 1; done[l] = 1; }
            fin[l] = ls;
            all = all && done[l];
        }
        if (all) break;
        ++nrestart;
        // FP32 inner CG on A e = r_b for the loads still running
        if (ahom_launch_reset(s->d_st, n_load, st)) return fail(AHOM_E_DEVICE, "reset");
        HIPCHK(hipMemcpyAsync(s->h_st, s->d_st, n_load * sizeof(LoadState), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int l = 0; l < n_load; ++l) s->h_st[l].done = done[l];
        HIPCHK(hipMemcpyAsync(s->d_st, s->h_st, n_load * sizeof(LoadState), hipMemcpyHostToDevice, st));
        if (ahom_launch_cg_demote(static_cast<const double2*>(r->d_r), static_cast<float2*>(s->d_buf1),
                                  (int64_t)n_load * per, st))
            return fail(AHOM_E_DEVICE, "demote");
        if (ahom_launch_zero(s->prec, s->d_x, (int64_t)n_load * per, st)) return fail(AHOM_E_DEVICE, "zero");
        if (ahom_launch_zero(s->prec, s->d_tbuf, (int64_t)n_load * s->nt * P.S, st)) return fail(AHOM_E_DEVICE, "zero");
        s->cg_rr_stop = s->cfg.refine;
        rc = cg_sweep(s, n_load, 2);
        int local = 0;
        while (!rc) {
            HIPCHK(hipMemcpyAsync(s->h_st, s->d_st, n_load * sizeof(LoadState), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            bool inner_done = true;
            for (int l = 0; l < n_load; ++l) inner_done = inner_done && s->h_st[l].done;
            if (inner_done) break;
            if (local > s->cfg.max_iter + 2 * s->cfg.check_period) { rc = fail(AHOM_E_DEVICE, "loop control did not terminate"); break; }
            for (int i = 0; i < s->cfg.check_period && !rc; ++i, ++local) rc = cg_sweep(s, n_load, 0);
        }
        s->cg_rr_stop = 0.0;
        if (rc) return rc;
        for (int l = 0; l < n_load; ++l)
            if (!done[l]) { nupd[l] += s->h_st[l].iter; total += s->h_st[l].iter; }
        // eps_b += P e (loads that are done have e = 0).  The FP32 updates
        // leave rounding noise in e also where the operator never looks: the
        // mean and the classes the Hermitian rule zeroes.  No later residual
        // sees it, yet it shifts <sigma> (~1e-7 relative), so e enters the
        // iterate only through its C0-orthogonal projection P onto compatible
        // zero-mean fields, taken in FP64: the companion's CG start sweep on
        // e in the homogeneous reference medium gives r = -Gamma0 C0 e = -P e.
        GatherArgs ga{};
        ga.out = static_cast<double2*>(r->d_buf0);     // e in FP64
        ga.base = nullptr;
        ga.in0 = ga.in1 = static_cast<const float2*>(s->d_x);
        ga.st = s->d_st;
        ga.per_load = (int64_t)per;
        if (ahom_launch_refine_gather(ga, n_load, st)) return fail(AHOM_E_DEVICE, "launch refine gather");
        rc = project_sweep(s, r, n_load);
        if (rc) return rc;
        if (ahom_launch_cg_sub(static_cast<double2*>(r->d_x), static_cast<const double2*>(r->d_r), (int64_t)n_load * per, st))
            return fail(AHOM_E_DEVICE, "launch cg sub");
    }
    float ms = 0.f;
    HIPCHK(hipEventRecord(s->ev1, st));
    HIPCHK(hipEventSynchronize(s->ev1));
    HIPCHK(hipEventElapsedTime(&ms, s->ev0, s->ev1));
    s->last_ms = ms;
    s->last_enqueued = total + nrestart + 1;
    s->last_nload = n_load;
    s->last_restarts = nrestart;
    s->last_start.assign(n_load, 0);
    // history: the FP64 residual at the update counts where a sweep evaluated it, -1 between
    std::vector<double> hh((size_t)n_load * s->hist_cap, -1.0);
    for (int l = 0; l < n_load; ++l)
        for (const auto& pr : hrec[l])
            if (pr.first < s->hist_cap) hh[(size_t)l * s->hist_cap + pr.first] = pr.second;
    HIPCHK(hipMemcpyAsync(s->d_hist, hh.data(), hh.size() * sizeof(double), hipMemcpyHostToDevice, st));
    for (int l = 0; l < n_load; ++l) s->h_st[l] = fin[l];
    if (strain_out) {
        if (mem_flags != AHOM_MEM_DEVICE && (rc = s->ensure_real_staging())) return rc;
        RealArgs ra = r->real_args(REAL_TO_REAL);
        ra.buf0 = ra.buf1 = r->d_x;
        ra.real_io = mem_flags == AHOM_MEM_DEVICE ? static_cast<double*>(strain_out) : s->d_real;
        if (ahom_launch_real(AHOM_FP64, r->dim, REAL_TO_REAL, ra, r->g_real.nwg, n_load, r->g_real.lds, st))
            return fail(AHOM_E_DEVICE, "launch to_real");
        if (mem_flags != AHOM_MEM_DEVICE)
            HIPCHK(hipMemcpyAsync(strain_out, s->d_real, (size_t)n_load * nc * P.m * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    int ret = AHOM_OK;
    for (int l = 0; l < n_load; ++l) {
        const LoadState& ls = fin[l];
        if (iters) iters[l] = ls.iter;
        if (resid) resid[l] = ls.resid;
        if (mean_out)
            for (int c = 0; c < nc; ++c) mean_out[(size_t)l * nc + c] = ls.mean[c];
        if (ls.status == 2) ret = AHOM_E_DIVERGED;
        else if (ls.status == 1 && ret == AHOM_OK) ret = AHOM_W_NOT_CONVERGED;
    }
    if (ret == AHOM_E_DIVERGED) g_err = "residual diverged";
    return ret;
}

}  // namespace

extern "C" {

int ahom_version(void) { return (0 << 16) | (1 << 8) | 0; }

const char* ahom_last_error(void) { return g_err.c_str(); }

int ahom_pattern_create(int d, const int64_t* M, ahom_pattern** out) {
    if (!M || !out) return fail(AHOM_E_ARG, "null argument");
    *out = nullptr;
    ahom_pattern* p = new (std::nothrow) ahom_pattern();
    if (!p) return fail(AHOM_E_NOMEM, "host allocation failed");
    std::string err;
    int rc = ahom_smith_form(d, M, &p->sf, &err);
    if (rc != AHOM_OK) { delete p; return fail(rc, err); }
    if (p->sf.m > 1) {
        rc = ahom_build_plan(p->sf, kLmax, &p->plan, &err);
        if (rc != AHOM_OK) { delete p; return fail(rc, err); }
        ahom_build_twiddles(&p->plan, &p->tw);
    } else {
        p->plan = Plan{};
        p->plan.d = d;
        p->plan.m = 1;
    }
    *out = p;
    return AHOM_OK;
}

int ahom_pattern_create_transformed(int d, const int64_t* M, const double* L, ahom_pattern** out) {
    if (!M || !L || !out) return fail(AHOM_E_ARG, "null argument");
    *out = nullptr;
    if (d != 2 && d != 3) return fail(AHOM_E_ARG, "d must be 2 or 3");
    Plan probe{};
    std::string err;
    if (int rc = ahom_plan_set_cell(&probe, d, L, &err)) return fail(rc, err);   // validate L first
    const int rc = ahom_pattern_create(d, M, out);
    if (rc != AHOM_OK) return rc;
    if ((*out)->sf.m > 1) ahom_plan_set_cell(&(*out)->plan, d, L, &err);
    return AHOM_OK;
}

void ahom_pattern_destroy(ahom_pattern* p) { delete p; }

int ahom_pattern_info(const ahom_pattern* p, int64_t* m, int* dM, int64_t* e, int64_t* Q, int64_t* R) {
    if (!p) return fail(AHOM_E_ARG, "null pattern");
    const int d = p->sf.d;
    if (m) *m = p->sf.m;
    if (dM) *dM = p->sf.dM;
    for (int i = 0; i < d; ++i) {
        if (e) e[i] = p->sf.e[i];
        for (int j = 0; j < d; ++j) {
            if (Q) Q[i * d + j] = p->sf.Q[i][j];
            if (R) R[i * d + j] = p->sf.R[i][j];
        }
    }
    return AHOM_OK;
}

int ahom_pattern_points(const ahom_pattern* p, int64_t* num) {
    if (!p || !num) return fail(AHOM_E_ARG, "null argument");
    ahom_canonical_points(p->sf, num);
    return AHOM_OK;
}

int ahom_pattern_freqs(const ahom_pattern* p, int64_t* h) {
    if (!p || !h) return fail(AHOM_E_ARG, "null argument");
    if (p->sf.m == 1) {
        for (int i = 0; i < p->sf.d; ++i) h[i] = 0;
        return AHOM_OK;
    }
    ahom_canonical_freqs(p->sf, p->plan.fm, h);
    return AHOM_OK;
}

int ahom_dft(const ahom_pattern* pc, int sign, int prec, const void* in, void* out, int mem_flags, void* stream) {
    if (!pc || !in || !out || (sign != -1 && sign != 1)) return fail(AHOM_E_ARG, "bad argument");
    if (prec != AHOM_FP64 && prec != AHOM_FP32_MIXED) return fail(AHOM_E_ARG, "bad precision");
    ahom_pattern* p = const_cast<ahom_pattern*>(pc);
    const int64_t m = p->sf.m;
    const size_t es = prec == AHOM_FP64 ? 16 : 8;
    hipStream_t s = (hipStream_t)stream;
    if (m == 1) {
        if (mem_flags == AHOM_MEM_DEVICE) HIPCHK(hipMemcpyAsync(out, in, es, hipMemcpyDeviceToDevice, s));
        else std::memcpy(out, in, es);
        return AHOM_OK;
    }
    int rc = p->ensure_device();
    if (rc) return rc;
    const Plan& P = p->plan;
    void* X = nullptr;
    void* Y = nullptr;
    HIPCHK(hipMalloc(&X, m * es));
    HIPCHK(hipMalloc(&Y, m * es));
    auto cleanup = [&]() { (void)hipFree(X); (void)hipFree(Y); };
    const hipMemcpyKind kin = mem_flags == AHOM_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const hipMemcpyKind kout = mem_flags == AHOM_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (hipMemcpyAsync(sign < 0 ? X : Y, in, m * es, kin, s) != hipSuccess) { cleanup(); return fail(AHOM_E_DEVICE, "copy in"); }
    ReorderArgs ro{};
    ro.plan = p->dev.plan;
    if (sign > 0) {  // canonical frequency order -> kernel positions
        ro.in = Y; ro.out = X; ro.dir = 1; ro.scale = 1.0;
        if (ahom_launch_reorder(prec, ro, m, s)) { cleanup(); return fail(AHOM_E_DEVICE, "reorder"); }
    }
    for (int t = 0; t < P.D; ++t) {
        const int a = sign < 0 ? t : P.D - 1 - t;
        int64_t O = 1, I = 1;
        for (int b = 0; b < a; ++b) O *= P.ax[b].len;
        for (int b = a + 1; b < P.D; ++b) I *= P.ax[b].len;
        PassGeom g;
        if ((rc = choose_geom(P.ax[a].len, O * I, 2, 0, es, prec, &g))) { cleanup(); return rc; }
        AxisArgs aa{};
        aa.plan = p->dev.plan;
        aa.buf0 = X;
        aa.buf1 = X;
        aa.tw = prec == AHOM_FP64 ? (const void*)p->dev.tw64 : (const void*)p->dev.tw32;
        aa.tw64 = p->dev.tw64;
        aa.st = nullptr;
        aa.axis = a;
        aa.slen0_full = 1;
        aa.NC = g.NC;
        aa.CS = g.CS;
        if (ahom_launch_axis(prec, sign, aa, g.nwg, 1, 1, g.lds, s)) { cleanup(); return fail(AHOM_E_DEVICE, "axis launch"); }
    }
    if (sign < 0) {
        ro.in = X; ro.out = Y; ro.dir = 0; ro.scale = 1.0 / (double)m;
        if (ahom_launch_reorder(prec, ro, m, s)) { cleanup(); return fail(AHOM_E_DEVICE, "reorder"); }
    }
    if (hipMemcpyAsync(out, sign < 0 ? Y : X, m * es, kout, s) != hipSuccess) { cleanup(); return fail(AHOM_E_DEVICE, "copy out"); }
    if (hipStreamSynchronize(s) != hipSuccess) { cleanup(); return fail(AHOM_E_DEVICE, "sync"); }
    cleanup();
    return AHOM_OK;
}

int ahom_dft_noalloc(const ahom_pattern* p, int sign, int prec, const void* in, void* out, void* stream) {
    if (!p || !in || !out || (sign != -1 && sign != 1)) return fail(AHOM_E_ARG, "bad argument");
    if (prec != AHOM_FP64 && prec != AHOM_FP32_MIXED) return fail(AHOM_E_ARG, "bad precision");
    const int64_t m = p->sf.m;
    const size_t es = prec == AHOM_FP64 ? 16 : 8;
    hipStream_t s = (hipStream_t)stream;
    if (m > kScratchMaxPoints)
        return fail(AHOM_E_ARG, "pattern of " + std::to_string(m) + " points exceeds the 2^21-point scratch of the allocation-free DFT");
    if (m == 1) {
        HIPCHK(hipMemcpyAsync(out, in, es, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        return AHOM_OK;
    }
    const size_t ntw = p->tw.size() / 2;
    const size_t off64 = kScratchPlanBytes;
    const size_t off32 = (off64 + ntw * 16 + 255) / 256 * 256;
    if (off32 + ntw * 8 > kScratchTableBytes) return fail(AHOM_E_ARG, "twiddle tables exceed the scratch of the allocation-free DFT");
    void* base = nullptr;
    int rc = scratch_base(&base);
    if (rc) return rc;
    unsigned char* b = static_cast<unsigned char*>(base);
    Plan* dplan = reinterpret_cast<Plan*>(b);
    double2* tw64 = reinterpret_cast<double2*>(b + off64);
    float2* tw32 = reinterpret_cast<float2*>(b + off32);
    void* X = b + kScratchTableBytes;
    const Plan& P = p->plan;
    HIPCHK(hipMemcpyAsync(dplan, &P, sizeof(Plan), hipMemcpyHostToDevice, s));
    if (ntw) {
        HIPCHK(hipMemcpyAsync(tw64, p->tw.data(), ntw * 16, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_twiddles_to_f32, dim3((unsigned)std::min<size_t>((ntw + 255) / 256, 256)), dim3(256), 0, s,
                           (const double2*)tw64, tw32, (int64_t)ntw);
        HIPCHK(hipGetLastError());
    }
    ReorderArgs ro{};
    ro.plan = dplan;
    if (sign < 0) {
        HIPCHK(hipMemcpyAsync(X, in, m * es, hipMemcpyDeviceToDevice, s));
    } else {  // canonical frequency order -> kernel positions
        ro.in = in; ro.out = X; ro.dir = 1; ro.scale = 1.0;
        if (ahom_launch_reorder(prec, ro, m, s)) return fail(AHOM_E_DEVICE, "reorder");
    }
    for (int t = 0; t < P.D; ++t) {
        const int a = sign < 0 ? t : P.D - 1 - t;
        int64_t O = 1, I = 1;
        for (int q = 0; q < a; ++q) O *= P.ax[q].len;
        for (int q = a + 1; q < P.D; ++q) I *= P.ax[q].len;
        PassGeom g;
        if ((rc = choose_geom(P.ax[a].len, O * I, 2, 0, es, prec, &g))) return rc;
        AxisArgs aa{};
        aa.plan = dplan;
        aa.buf0 = X;
        aa.buf1 = X;
        aa.tw = prec == AHOM_FP64 ? (const void*)tw64 : (const void*)tw32;
        aa.tw64 = tw64;
        aa.st = nullptr;
        aa.axis = a;
        aa.slen0_full = 1;
        aa.NC = g.NC;
        aa.CS = g.CS;
        if (ahom_launch_axis(prec, sign, aa, g.nwg, 1, 1, g.lds, s)) return fail(AHOM_E_DEVICE, "axis launch");
    }
    if (sign < 0) {
        ro.in = X; ro.out = out; ro.dir = 0; ro.scale = 1.0 / (double)m;
        if (ahom_launch_reorder(prec, ro, m, s)) return fail(AHOM_E_DEVICE, "reorder");
    } else {
        HIPCHK(hipMemcpyAsync(out, X, m * es, hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return AHOM_OK;
}

int ahom_solver_create(const ahom_pattern* pc, const ahom_config* cfg, ahom_solver** out) {
    if (!pc || !cfg || !out) return fail(AHOM_E_ARG, "null argument");
    *out = nullptr;
    if (cfg->precision != AHOM_FP64 && cfg->precision != AHOM_FP32_MIXED) return fail(AHOM_E_ARG, "bad precision");
    if (cfg->max_iter < 0 || !(cfg->tol >= 0.0)) return fail(AHOM_E_ARG, "bad tol/max_iter");
    if (cfg->nyquist != AHOM_NYQUIST_HERMITIAN) return fail(AHOM_E_ARG, "unsupported Nyquist rule");
    if (!(cfg->refine < 1.0)) return fail(AHOM_E_ARG, "refine must be < 1");
    if (cfg->stop_rule != AHOM_STOP_RESIDUAL && cfg->stop_rule != AHOM_STOP_CAUCHY) return fail(AHOM_E_ARG, "unknown stop rule");
    if (cfg->stop_rule == AHOM_STOP_CAUCHY && cfg->precision == AHOM_FP32_MIXED && !(cfg->refine < 0.0))
        return fail(AHOM_E_ARG, "the Cauchy stop rule in FP32 needs refine < 0 (no restarts)");
    if (cfg->scheme != AHOM_SCHEME_BASIC && cfg->scheme != AHOM_SCHEME_CG) return fail(AHOM_E_ARG, "unknown scheme");
    if (cfg->physics != AHOM_ELASTICITY && cfg->physics != AHOM_CONDUCTIVITY) return fail(AHOM_E_ARG, "unknown physics");
    if (cfg->guess_probe < 0 || cfg->guess_probe > cfg->max_iter) return fail(AHOM_E_ARG, "guess_probe must be in [0, max_iter]");
    if (cfg->scheme == AHOM_SCHEME_CG && cfg->stop_rule != AHOM_STOP_RESIDUAL)
        return fail(AHOM_E_ARG, "the conjugate-gradient scheme stops on the residual");
    if (cfg->scheme == AHOM_SCHEME_CG && cfg->precision == AHOM_FP32_MIXED && !(cfg->refine >= 0.0))
        return fail(AHOM_E_ARG, "the conjugate-gradient scheme in FP32 runs with FP64 corrections (refine >= 0)");
    return create_solver(const_cast<ahom_pattern*>(pc), cfg, out);
}

void ahom_solver_destroy(ahom_solver* s) { delete s; }

}  // extern "C"

namespace {
// phase table (pairs per phase) and phase ids on the device; the default
// reference is the mean of the extreme values of each slot
int upload_table(ahom_solver* s, int n_phase, const double* lame, const uint8_t* phase, int mem_flags);
}  // namespace

extern "C" {

int ahom_solver_set_material(ahom_solver* s, int n_phase, const double* lame, const uint8_t* phase, int mem_flags) {
    if (!s || !lame || !phase || n_phase < 1 || n_phase > 256) return fail(AHOM_E_ARG, "bad material arguments");
    if (s->phys != PHYS_ELASTIC) return fail(AHOM_E_ARG, "a conductivity solver: use ahom_solver_set_conductivity");
    for (int k = 0; k < n_phase; ++k) {
        const double l = lame[2 * k], mu = lame[2 * k + 1];
        if (!(mu > 0.0) || !(3.0 * l + 2.0 * mu > 0.0)) return fail(AHOM_E_MATERIAL, "phase " + std::to_string(k) + ": need mu > 0 and 3 lambda + 2 mu > 0");
    }
    return upload_table(s, n_phase, lame, phase, mem_flags);
}

int ahom_solver_set_conductivity(ahom_solver* s, int n_phase, const double* k, const uint8_t* phase, int mem_flags) {
    if (!s || !k || !phase || n_phase < 1 || n_phase > 256) return fail(AHOM_E_ARG, "bad material arguments");
    if (s->phys != PHYS_THERMAL) return fail(AHOM_E_ARG, "an elasticity solver: use ahom_solver_set_material");
    double tab[512];
    for (int q = 0; q < n_phase; ++q) {
        if (!(k[q] > 0.0) || !std::isfinite(k[q])) return fail(AHOM_E_MATERIAL, "phase " + std::to_string(q) + ": need 0 < k < inf");
        tab[2 * q] = tab[2 * q + 1] = k[q];
    }
    return upload_table(s, n_phase, tab, phase, mem_flags);
}

int ahom_solver_set_reference_conductivity(ahom_solver* s, double k0) {
    if (!s) return fail(AHOM_E_ARG, "null solver");
    if (s->phys != PHYS_THERMAL) return fail(AHOM_E_ARG, "an elasticity solver: use ahom_solver_set_reference");
    if (!(k0 > 0.0) || !std::isfinite(k0)) return fail(AHOM_E_MATERIAL, "reference needs 0 < k0 < inf");
    s->lam0 = s->mu0 = k0;
    s->ref_set = true;
    return AHOM_OK;
}

}  // extern "C"

namespace {
int upload_table(ahom_solver* s, int n_phase, const double* lame, const uint8_t* phase, int mem_flags) {
    double llo = 1e300, lhi = -1e300, mlo = 1e300, mhi = -1e300;
    for (int k = 0; k < n_phase; ++k) {
        const double l = lame[2 * k], mu = lame[2 * k + 1];
        llo = std::min(llo, l); lhi = std::max(lhi, l); mlo = std::min(mlo, mu); mhi = std::max(mhi, mu);
    }
    const int64_t m = s->pat->sf.m;
    dfree(s->d_lame_pts);
    if (!s->d_phase) HIPCHK(hipMalloc((void**)&s->d_phase, m));
    dfree(s->d_lame_tab);
    HIPCHK(hipMalloc((void**)&s->d_lame_tab, 2 * n_phase * sizeof(double)));
    HIPCHK(hipMemcpy(s->d_lame_tab, lame, 2 * n_phase * sizeof(double), hipMemcpyHostToDevice));
    if (mem_flags == AHOM_MEM_DEVICE) {
        HIPCHK(hipMemcpyAsync(s->d_phase, phase, m, hipMemcpyDeviceToDevice, s->stream));
    } else {
        std::vector<uint8_t> chk(phase, phase + m);
        for (int64_t i = 0; i < m; ++i)
            if (chk[i] >= n_phase) return fail(AHOM_E_ARG, "phase id out of range");
        HIPCHK(hipMemcpy(s->d_phase, phase, m, hipMemcpyHostToDevice));
    }
    {
        const Plan& P = s->pat->plan;
        dfree(s->d_lame_pts_t);
        if (!s->d_phase_t) HIPCHK(hipMalloc((void**)&s->d_phase_t, m));
        if (ahom_launch_transpose(s->d_phase, s->d_phase_t, P.ax[0].len, m / P.ax[0].len, 1, s->stream))
            return fail(AHOM_E_DEVICE, "transpose phase ids");
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    s->n_phase = n_phase;
    s->lam_lo = llo; s->lam_hi = lhi; s->mu_lo = mlo; s->mu_hi = mhi;
    s->has_material = true;
    if (!s->ref_set) { s->lam0 = 0.5 * (llo + lhi); s->mu0 = 0.5 * (mlo + mhi); }
    return AHOM_OK;
}

}  // namespace

extern "C" {

int ahom_solver_set_stiffness_field(ahom_solver* s, const double* lame_pts, int mem_flags) {
    if (!s || !lame_pts) return fail(AHOM_E_ARG, "null argument");
    if (s->phys != PHYS_ELASTIC) return fail(AHOM_E_ARG, "per-point fields are elastic only");
    const int64_t m = s->pat->sf.m;
    std::vector<double> h;
    const double* hp = lame_pts;
    if (mem_flags == AHOM_MEM_DEVICE) {
        h.resize(2 * m);
        HIPCHK(hipMemcpy(h.data(), lame_pts, 2 * m * sizeof(double), hipMemcpyDeviceToHost));
        hp = h.data();
    }
    double llo = 1e300, lhi = -1e300, mlo = 1e300, mhi = -1e300;
    for (int64_t i = 0; i < m; ++i) {
        const double l = hp[2 * i], mu = hp[2 * i + 1];
        if (!(mu > 0.0) || !(3.0 * l + 2.0 * mu > 0.0)) return fail(AHOM_E_MATERIAL, "point " + std::to_string(i) + ": need mu > 0 and 3 lambda + 2 mu > 0");
        llo = std::min(llo, l); lhi = std::max(lhi, l); mlo = std::min(mlo, mu); mhi = std::max(mhi, mu);
    }
    dfree(s->d_lame_pts);
    HIPCHK(hipMalloc((void**)&s->d_lame_pts, 2 * m * sizeof(double)));
    HIPCHK(hipMemcpy(s->d_lame_pts, hp, 2 * m * sizeof(double), hipMemcpyHostToDevice));
    {
        const Plan& P = s->pat->plan;
        dfree(s->d_lame_pts_t);
        HIPCHK(hipMalloc((void**)&s->d_lame_pts_t, 2 * m * sizeof(double)));
        if (ahom_launch_transpose(s->d_lame_pts, s->d_lame_pts_t, P.ax[0].len, m / P.ax[0].len, 16, s->stream))
            return fail(AHOM_E_DEVICE, "transpose stiffness field");
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    s->lam_lo = llo; s->lam_hi = lhi; s->mu_lo = mlo; s->mu_hi = mhi;
    s->has_material = true;
    if (!s->ref_set) { s->lam0 = 0.5 * (llo + lhi); s->mu0 = 0.5 * (mlo + mhi); }
    return AHOM_OK;
}

int ahom_solver_set_reference(ahom_solver* s, double lambda0, double mu0) {
    if (!s) return fail(AHOM_E_ARG, "null solver");
    if (s->phys != PHYS_ELASTIC) return fail(AHOM_E_ARG, "a conductivity solver: use ahom_solver_set_reference_conductivity");
    if (!(mu0 > 0.0) || !(lambda0 + 2.0 * mu0 > 0.0)) return fail(AHOM_E_MATERIAL, "reference needs mu0 > 0 and lambda0 + 2 mu0 > 0");
    s->lam0 = lambda0;
    s->mu0 = mu0;
    s->ref_set = true;
    return AHOM_OK;
}

}  // extern "C"

namespace {
// Algorithm 1 (or CG) for n_load macroscopic fields given as component
// vectors ebc[n_load * ncomp] of the solver's field layout; mean_out
// (nullable) receives the mean stress (flux) components the same way.
int solve_core(ahom_solver* s, int n_load, const double* ebc, const void* init, void* strain_out,
               int* iters, double* resid, double* mean_out, int mem_flags) {
    RoctxRange range(s->cg ? "ahom_solve (conjugate gradients)" : "ahom_solve (Basic Scheme)");
    if (!s->has_material) return fail(AHOM_E_MATERIAL, "no material set");
    if (init && s->cfg.stop_rule == AHOM_STOP_CAUCHY)
        return fail(AHOM_E_ARG, "the Cauchy stop rule measures against sqrt(m) |eps_bar|, not a guessed start: no init");
    if (s->cg) {
        if (init && s->cfg.guess_probe > 0) return fail(AHOM_E_ARG, "guess_probe is a Basic Scheme option (the CG start is the projected guess)");
        return solve_cg(s, n_load, ebc, init, strain_out, iters, resid, mean_out, mem_flags);
    }
    // guess probe: the plain start runs beside the guessed one as loads
    // n_load .. 2 n_load - 1 for the first guess_probe iterations
    const bool probe = init && s->cfg.guess_probe > 0;
    const int nl2 = probe ? 2 * n_load : n_load;
    int rc = s->ensure_capacity(nl2);
    if (rc) return rc;
    s->spec_toff = nullptr;
    s->spec_dout = s->spec_dneg = nullptr;
    s->red_sig_base = nullptr;
    s->cur_tol = s->cfg.tol;
    if ((rc = s->autotune(n_load))) return rc;
    const Plan& P = s->pat->plan;
    const int nc = s->ncomp;
    hipStream_t st = s->stream;
    const bool refine = s->prec == AHOM_FP32_MIXED && s->cfg.refine > 0.0;
    if (refine) s->cur_tol = std::max(s->cfg.tol, s->cfg.refine);
    // set up the FP64 companion ahead of the timed region when a restart is expected
    if (refine && s->cfg.tol < s->cur_tol && (rc = ensure_ref64(s, n_load))) return rc;
    std::vector<double> eb(ebc, ebc + (size_t)n_load * nc);
    if (probe) eb.insert(eb.end(), ebc, ebc + (size_t)n_load * nc);
    HIPCHK(hipMemcpyAsync(s->d_epsbar, eb.data(), eb.size() * sizeof(double), hipMemcpyHostToDevice, st));
    // denominator of the Cauchy measure: |eps(0)| = sqrt(m) |eps_bar|_F for the
    // plain start (kept with a user initial guess)
    std::vector<double> norm0(nl2);
    for (int l = 0; l < nl2; ++l) {
        double f = 0.0;
        for (int c = 0; c < nc; ++c) f += field_weight(s->phys, s->dim, c) * eb[(size_t)l * nc + c] * eb[(size_t)l * nc + c];
        norm0[l] = std::sqrt((double)P.m * f);
    }
    HIPCHK(hipMemcpyAsync(s->d_norm0, norm0.data(), norm0.size() * sizeof(double), hipMemcpyHostToDevice, st));
    if (ahom_launch_reset(s->d_st, nl2, st)) return fail(AHOM_E_DEVICE, "reset");
    if (ahom_launch_zero(s->prec, s->d_tbuf, (int64_t)nl2 * s->nt * P.S, st)) return fail(AHOM_E_DEVICE, "zero");
    s->last_start.assign(n_load, init ? 1 : 0);
    auto fill = [&](void* buf) -> int {
        FillArgs f{};
        f.buf = buf;
        f.eps_bar = s->d_epsbar;
        f.S = P.S;
        f.row = P.S / P.ax[0].slen;
        f.nfield = nc;
        return ahom_launch_fill(s->prec, f, n_load, st);
    };
    if (!init) {
        if (fill(s->d_buf0)) return fail(AHOM_E_DEVICE, "fill");
    } else {
        RealArgs fr = s->real_args(REAL_FROM_REAL);
        if (mem_flags == AHOM_MEM_DEVICE) {
            fr.real_io = const_cast<double*>(static_cast<const double*>(init));
        } else {
            if ((rc = s->ensure_real_staging())) return rc;
            const size_t bytes = (size_t)n_load * nc * P.m * sizeof(double);
            HIPCHK(hipMemcpyAsync(s->d_real, init, bytes, hipMemcpyHostToDevice, st));
            fr.real_io = s->d_real;
        }
        if (ahom_launch_real(s->prec, s->dim, REAL_FROM_REAL, fr, s->g_real.nwg, n_load, s->g_real.lds, st))
            return fail(AHOM_E_DEVICE, "launch from_real");
        // traction of eps(0): t(0) = -(C0 : eps_hat(0)) xi, so that the first
        // residual is sigma_hat(0) xi = t(1) - t(0) as on later iterations
        HIPCHK(hipMemcpyAsync(s->d_buf1, s->d_buf0, (size_t)n_load * nc * P.S * s->es(), hipMemcpyDeviceToDevice, st));
        for (int a = 1; a <= P.D - 2; ++a) {
            AxisArgs aa = s->axis_args(a);
            aa.st = nullptr;
            aa.buf0 = s->d_buf1;
            if (ahom_launch_axis(s->prec, -1, aa, s->g_axis[a].nwg, nc, n_load, s->g_axis[a].lds, st))
                return fail(AHOM_E_DEVICE, "launch init axis");
        }
        SpecArgs sa = s->spec_args();
        sa.buf0 = s->d_buf1;
        sa.buf1 = nullptr;
        sa.lam0_init = s->lam0;
        if (ahom_launch_spec_init(s->prec, s->dim, sa, s->g_spec.nwg, n_load, s->g_spec.lds, st))
            return fail(AHOM_E_DEVICE, "launch init traction");
        if (probe) {   // the plain starts of the probe
            FillArgs f{};
            f.buf = static_cast<char*>(s->d_buf0) + (size_t)n_load * nc * P.S * s->es();
            f.eps_bar = s->d_epsbar + (size_t)n_load * nc;
            f.S = P.S;
            f.row = P.S / P.ax[0].slen;
            f.nfield = nc;
            if (ahom_launch_fill(s->prec, f, n_load, st)) return fail(AHOM_E_DEVICE, "fill");
        }
    }
    HIPCHK(hipEventRecord(s->ev0, st));
    int enq = 0;
    if (probe) {
        // Both starts for guess_probe iterations in the same launches; per load
        // keep the start that met the tolerance (of the first FP32 stage with
        // restarts) first, or if neither has, the guessed start if
        // it is predicted to reach tol in at most 90 % of the plain start's
        // updates; for the plain start carry its state (fields, traction,
        // history) over.
        for (int i = 0; i < s->cfg.guess_probe; ++i) {
            if ((rc = s->enqueue_iteration(nl2))) return rc;
            ++enq;
        }
        const int kp = s->cfg.guess_probe;
        std::vector<double> hh((size_t)nl2 * s->hist_cap);
        HIPCHK(hipMemcpyAsync(s->h_st, s->d_st, nl2 * sizeof(LoadState), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hh.data(), s->d_hist, hh.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        // updates still needed from a start, predicted from its residuals over the
        // probe's second half: the last evaluated r(i2) and r(i1) with i1 near
        // i2 / 2 give the contraction per update rho, and log(r(i2) / tol) /
        // log(1 / rho) more updates reach tol
        auto predicted = [&](int load) -> double {
            const double* h = hh.data() + (size_t)load * s->hist_cap;
            int i2 = -1, i1 = -1;
            for (int i = std::min(kp, s->hist_cap) - 1; i >= 0; --i)
                if (h[i] > 0.0) { i2 = i; break; }
            for (int i = 0; i < i2; ++i)
                if (h[i] > 0.0 && 2 * i >= i2) { i1 = i; break; }
            if (i2 < 0) return 1e300;
            if (h[i2] <= s->cfg.tol) return i2;
            if (i1 < 0 || !(h[i2] < h[i1])) return 1e300;
            const double rate = std::log(h[i1] / h[i2]) / (double)(i2 - i1);
            return i2 + std::log(h[i2] / s->cfg.tol) / rate;
        };
        const size_t fbytes = (size_t)nc * P.S * s->es(), tbytes = (size_t)s->nt * P.S * s->es();
        for (int l = 0; l < n_load; ++l) {
            const LoadState& g = s->h_st[l];
            const LoadState& z = s->h_st[l + n_load];
            const bool gc = g.done && g.status == 0, zc = z.done && z.status == 0;
            bool keep_guess;
            if (gc && zc) keep_guess = g.iter <= z.iter;     // both met the (stage) tolerance: the earlier one
            else if (gc) keep_guess = true;
            else if (zc) keep_guess = false;
            else if (g.status == 2) keep_guess = false;
            else keep_guess = predicted(l) <= 0.9 * predicted(l + n_load);   // a guess must promise 10 % fewer updates
            s->last_start[l] = keep_guess ? 1 : 0;
            if (keep_guess) continue;
            char* b0 = static_cast<char*>(s->d_buf0);
            char* b1 = static_cast<char*>(s->d_buf1);
            char* tb = static_cast<char*>(s->d_tbuf);
            HIPCHK(hipMemcpyAsync(b0 + l * fbytes, b0 + (l + n_load) * fbytes, fbytes, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(b1 + l * fbytes, b1 + (l + n_load) * fbytes, fbytes, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(tb + l * tbytes, tb + (l + n_load) * tbytes, tbytes, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(s->d_hist + (size_t)l * s->hist_cap, s->d_hist + (size_t)(l + n_load) * s->hist_cap,
                                  s->hist_cap * sizeof(double), hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(s->d_chist + (size_t)l * s->hist_cap, s->d_chist + (size_t)(l + n_load) * s->hist_cap,
                                  s->hist_cap * sizeof(double), hipMemcpyDeviceToDevice, st));
            s->h_st[l] = z;
        }
        HIPCHK(hipMemcpyAsync(s->d_st, s->h_st, n_load * sizeof(LoadState), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    // iterate until every load case has stopped (device-side loop control);
    // the host reads the load states every check_period iterations
    auto run_stage = [&]() -> int {
        const int limit = s->cfg.max_iter + 1;
        int local = 0;
        bool all_done = false;
        while (!all_done) {
            const int k = std::min(s->cfg.check_period, std::max(1, limit - local));
            for (int i = 0; i < k; ++i) {
                int rc2 = s->enqueue_iteration(n_load);
                if (rc2) return rc2;
                ++local;
                ++enq;
            }
            HIPCHK(hipMemcpyAsync(s->h_st, s->d_st, n_load * sizeof(LoadState), hipMemcpyDeviceToHost, st));
            HIPCHK(hipEventRecord(s->ev1, st));
            HIPCHK(hipStreamSynchronize(st));
            all_done = true;
            for (int l = 0; l < n_load; ++l) all_done = all_done && s->h_st[l].done;
            if (local > limit + 2 * s->cfg.check_period) return fail(AHOM_E_DEVICE, "loop control did not terminate");
        }
        return AHOM_OK;
    };
    if ((rc = run_stage())) return rc;

    // FP32 defect-correction restarts (see ahom_config.refine).  With the FP64
    // iterate eps_b = F(eps_h) (one FP64 update of eps_h = FP64 base + FP32
    // state) and its traction step d = t(eps_b) - t(eps_h), the correction
    // e = eps - eps_b obeys e(k+1) = Gamma0-map of (t(e(k)) + d) with zero
    // mean, and the residual of eps_b + e(k) is t(e(k)) - t(e(k-1)), with
    // t(e(-1)) = -d.  The mean stress is that of eps_b plus that of e.
    int nrestart = 0;
    std::vector<double> hsig((size_t)n_load * nc), zeros((size_t)n_load * nc, 0.0), hrec(n_load);
    const double not_evaluated = -1.0;   // Cauchy measure of a restart's FP64 step: not recorded
    while (refine) {
        bool need = false, stop = false;
        for (int l = 0; l < n_load; ++l) {
            const LoadState& ls = s->h_st[l];
            if (ls.status != 0) stop = true;
            else if (ls.resid > s->cfg.tol) need = true;
        }
        if (stop || !need) break;
        if ((rc = ensure_ref64(s, n_load))) return rc;
        ahom_solver* r = s->ref64;
        HIPCHK(hipMemcpyAsync(r->d_epsbar, eb.data(), (size_t)n_load * nc * sizeof(double), hipMemcpyHostToDevice, st));
        GatherArgs g{};
        g.out = static_cast<double2*>(r->d_buf0);
        g.base = nrestart ? static_cast<const double2*>(r->d_buf1) : nullptr;
        g.in0 = static_cast<const float2*>(s->d_buf0);
        g.in1 = static_cast<const float2*>(s->d_buf1);
        g.st = s->d_st;
        g.per_load = (int64_t)nc * P.S;
        if (ahom_launch_refine_gather(g, n_load, st)) return fail(AHOM_E_DEVICE, "launch refine gather");
        if (ahom_launch_reset(r->d_st, n_load, st)) return fail(AHOM_E_DEVICE, "reset");
        if (ahom_launch_zero(AHOM_FP64, r->d_tbuf, (int64_t)n_load * r->nt * P.S, st)) return fail(AHOM_E_DEVICE, "zero");
        r->spec_dout = s->d_toff;
        r->spec_dneg = s->d_tbuf;
        for (int i = 0; i < 2; ++i)
            if ((rc = r->enqueue_iteration(n_load))) { r->spec_dout = r->spec_dneg = nullptr; return rc; }
        r->spec_dout = r->spec_dneg = nullptr;
        enq += 2;
        HIPCHK(hipMemcpyAsync(r->h_st, r->d_st, n_load * sizeof(LoadState), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        double rmax = 0.0;
        bool any = false;
        for (int l = 0; l < n_load; ++l) {
            const LoadState& lr = r->h_st[l];
            LoadState ls{};
            ls.iter = std::min(s->h_st[l].iter + 1, s->cfg.max_iter);
            ls.r0 = s->h_st[l].r0;
            ls.resid = lr.resid;
            for (int c = 0; c < nc; ++c) ls.mean[c] = hsig[(size_t)l * nc + c] = lr.mean[c];
            ls.final_buf = ls.iter & 1;
            if (!(lr.resid == lr.resid) || std::isinf(lr.resid)) { ls.done = 1; ls.status = 2; }
            else if (lr.resid <= s->cfg.tol) { ls.done = 1; ls.status = 0; }
            else if (ls.iter >= s->cfg.max_iter) { ls.done = 1; ls.status = 1; }
            else { rmax = std::max(rmax, lr.resid); any = true; }
            hrec[l] = lr.resid;
            if (ls.done && ls.iter < s->hist_cap) {
                HIPCHK(hipMemcpyAsync(s->d_hist + (size_t)l * s->hist_cap + ls.iter, &hrec[l], sizeof(double), hipMemcpyHostToDevice, st));
                HIPCHK(hipMemcpyAsync(s->d_chist + (size_t)l * s->hist_cap + ls.iter, &not_evaluated, sizeof(double),
                                      hipMemcpyHostToDevice, st));
            }
            s->h_st[l] = ls;
        }
        HIPCHK(hipMemcpyAsync(s->d_st, s->h_st, n_load * sizeof(LoadState), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(s->d_sigbase, hsig.data(), hsig.size() * sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(s->d_epsbar, zeros.data(), zeros.size() * sizeof(double), hipMemcpyHostToDevice, st));
        if (fill(s->d_buf0) || fill(s->d_buf1)) return fail(AHOM_E_DEVICE, "fill");
        HIPCHK(hipStreamSynchronize(st));
        ++nrestart;
        if (!any) break;
        s->spec_toff = s->d_toff;
        s->red_sig_base = s->d_sigbase;
        s->cur_tol = std::max(s->cfg.tol, s->cfg.refine * rmax);
        rc = run_stage();
        s->spec_toff = nullptr;
        s->red_sig_base = nullptr;
        if (rc) return rc;
    }
    s->cur_tol = s->cfg.tol;

    float ms = 0.f;
    HIPCHK(hipEventRecord(s->ev1, st));
    HIPCHK(hipEventSynchronize(s->ev1));
    HIPCHK(hipEventElapsedTime(&ms, s->ev0, s->ev1));
    s->last_ms = ms;
    s->last_enqueued = enq;
    s->last_nload = n_load;
    if (strain_out) {
        if (mem_flags != AHOM_MEM_DEVICE && (rc = s->ensure_real_staging())) return rc;
        double* dst = mem_flags == AHOM_MEM_DEVICE ? static_cast<double*>(strain_out) : s->d_real;
        RealArgs ra = s->real_args(REAL_TO_REAL);
        ra.real_io = dst;
        if (nrestart) {
            // strain = FP64 iterate + FP32 correction
            ahom_solver* r = s->ref64;
            RealArgs rb = r->real_args(REAL_TO_REAL);
            rb.real_io = dst;
            if (ahom_launch_real(AHOM_FP64, r->dim, REAL_TO_REAL, rb, r->g_real.nwg, n_load, r->g_real.lds, st))
                return fail(AHOM_E_DEVICE, "launch to_real (FP64 iterate)");
            ra.accumulate = 1;
        }
        if (ahom_launch_real(s->prec, s->dim, REAL_TO_REAL, ra, s->g_real.nwg, n_load, s->g_real.lds, st))
            return fail(AHOM_E_DEVICE, "launch to_real");
        if (mem_flags != AHOM_MEM_DEVICE)
            HIPCHK(hipMemcpyAsync(strain_out, s->d_real, (size_t)n_load * nc * P.m * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    s->last_restarts = nrestart;
    int ret = AHOM_OK;
    for (int l = 0; l < n_load; ++l) {
        const LoadState& ls = s->h_st[l];
        if (iters) iters[l] = ls.iter;
        if (resid) resid[l] = ls.resid;
        if (mean_out)
            for (int c = 0; c < nc; ++c) mean_out[(size_t)l * nc + c] = ls.mean[c];
        if (ls.status == 2) ret = AHOM_E_DIVERGED;
        else if ((ls.status == 1 || (s->cfg.stop_rule == AHOM_STOP_RESIDUAL && ls.resid > s->cfg.tol)) && ret == AHOM_OK)
            ret = AHOM_W_NOT_CONVERGED;
    }
    if (ret == AHOM_E_DIVERGED) g_err = "residual diverged";
    return ret;
}
}  // namespace

extern "C" {

int ahom_solve(ahom_solver* s, int n_load, const double* eps_bar, const void* init, void* strain_out,
               int* iters, double* resid, double* mean_stress, int mem_flags) {
    if (!s || !eps_bar || n_load < 1) return fail(AHOM_E_ARG, "bad solve arguments");
    if (s->phys != PHYS_ELASTIC) return fail(AHOM_E_ARG, "a conductivity solver: use ahom_solve_conductivity");
    const int nc = s->ncomp;
    const int* comp = s->dim == 3 ? kComp3 : kComp2;
    std::vector<double> ebc((size_t)n_load * nc), mc((size_t)n_load * nc);
    for (int l = 0; l < n_load; ++l)
        for (int c = 0; c < nc; ++c) ebc[(size_t)l * nc + c] = eps_bar[(size_t)l * 9 + comp[c]];
    const int ret = solve_core(s, n_load, ebc.data(), init, strain_out, iters, resid, mc.data(), mem_flags);
    if (ret < 0 && ret != AHOM_E_DIVERGED) return ret;
    if (mean_stress)
        for (int l = 0; l < n_load; ++l) {
            double* ms9 = mean_stress + (size_t)l * 9;
            for (int q = 0; q < 9; ++q) ms9[q] = 0.0;
            for (int c = 0; c < nc; ++c) {
                const int pos = comp[c];
                ms9[pos] = mc[(size_t)l * nc + c];
                ms9[(pos % 3) * 3 + pos / 3] = mc[(size_t)l * nc + c];
            }
        }
    return ret;
}

int ahom_solve_conductivity(ahom_solver* s, int n_load, const double* grad_bar, void* field_out, int* iters, double* resid,
                            double* mean_flux, int mem_flags) {
    if (!s || !grad_bar || n_load < 1) return fail(AHOM_E_ARG, "bad solve arguments");
    if (s->phys != PHYS_THERMAL) return fail(AHOM_E_ARG, "an elasticity solver: use ahom_solve");
    const int d = s->dim;
    std::vector<double> ebc((size_t)n_load * d), mc((size_t)n_load * d);
    for (int l = 0; l < n_load; ++l)
        for (int c = 0; c < d; ++c) ebc[(size_t)l * d + c] = grad_bar[(size_t)l * 3 + c];
    const int ret = solve_core(s, n_load, ebc.data(), nullptr, field_out, iters, resid, mc.data(), mem_flags);
    if (ret < 0 && ret != AHOM_E_DIVERGED) return ret;
    if (mean_flux)
        for (int l = 0; l < n_load; ++l)
            for (int c = 0; c < 3; ++c) mean_flux[(size_t)l * 3 + c] = c < d ? mc[(size_t)l * d + c] : 0.0;
    return ret;
}

int ahom_effective_conductivity(ahom_solver* s, double* Keff, int* iters) {
    if (!s || !Keff) return fail(AHOM_E_ARG, "null argument");
    const int d = s->dim;
    std::vector<double> g((size_t)d * 3, 0.0), q((size_t)d * 3);
    for (int l = 0; l < d; ++l) g[(size_t)l * 3 + l] = 1.0;
    const int rc = ahom_solve_conductivity(s, d, g.data(), nullptr, iters, nullptr, q.data(), AHOM_MEM_HOST);
    if (rc < 0) return rc;
    for (int col = 0; col < d; ++col)
        for (int row = 0; row < d; ++row) Keff[row * d + col] = q[(size_t)col * 3 + row];
    return rc;
}

int ahom_effective_stiffness(ahom_solver* s, double* Ceff, int* iters) {
    if (!s || !Ceff) return fail(AHOM_E_ARG, "null argument");
    const int d = s->dim;
    const int k = d == 3 ? 6 : 3;
    const int pr3[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};
    const int pr2[3][2] = {{0, 0}, {1, 1}, {0, 1}};
    std::vector<double> eb((size_t)k * 9, 0.0), ms((size_t)k * 9);
    const double r2 = std::sqrt(2.0);
    for (int l = 0; l < k; ++l) {
        const int i = d == 3 ? pr3[l][0] : pr2[l][0], j = d == 3 ? pr3[l][1] : pr2[l][1];
        const double v = i == j ? 1.0 : 1.0 / r2;
        eb[(size_t)l * 9 + i * 3 + j] = v;
        eb[(size_t)l * 9 + j * 3 + i] = v;
    }
    int rc = ahom_solve(s, k, eb.data(), nullptr, nullptr, iters, nullptr, ms.data(), AHOM_MEM_HOST);
    if (rc < 0) return rc;
    for (int col = 0; col < k; ++col)
        for (int row = 0; row < k; ++row) {
            const int i = d == 3 ? pr3[row][0] : pr2[row][0], j = d == 3 ? pr3[row][1] : pr2[row][1];
            Ceff[row * k + col] = ms[(size_t)col * 9 + i * 3 + j] * (i == j ? 1.0 : r2);
        }
    return rc;
}

int ahom_solver_pass_times(ahom_solver* s, int n_iter, double* ms, double* bytes, int cap, int* n_pass) {
    if (!s || !ms || !n_pass || n_iter < 1 || s->last_nload < 1) return fail(AHOM_E_ARG, "bad pass-timing arguments (solve first)");
    const Plan& P = s->pat->plan;
    const int nload = s->last_nload;
    const int np = 2 * (P.D - 2) + 3;
    if (cap < np) return fail(AHOM_E_ARG, "cap too small");
    hipStream_t st = s->stream;
    std::vector<hipEvent_t> ev(np + 1);
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    std::vector<double> acc(np, 0.0);
    if (ahom_launch_reset(s->d_st, nload, st)) return fail(AHOM_E_DEVICE, "reset");
    if (ahom_launch_zero(s->prec, s->d_tbuf, (int64_t)nload * s->nt * P.S, st)) return fail(AHOM_E_DEVICE, "zero");
    FillArgs f{};
    f.buf = s->d_buf0; f.eps_bar = s->d_epsbar; f.S = P.S; f.row = P.S / P.ax[0].slen; f.nfield = s->ncomp;
    if (ahom_launch_fill(s->prec, f, nload, st)) return fail(AHOM_E_DEVICE, "fill");
    ReduceArgs r{};
    r.phys = s->phys;
    r.st = s->d_st; r.sig_part = s->d_sig; r.res_part = s->d_res; r.hist = s->d_hist;
    r.n_real = s->n_real_wg(); r.n_spec = s->n_spec_wg(); r.hist_cap = s->hist_cap; r.m = P.m;
    r.tol = -1.0; r.max_iter = 1 << 30; r.resid_period = s->cfg.resid_period;
    for (int it = 0; it < n_iter; ++it) {
        int p = 0;
        HIPCHK(hipEventRecord(ev[p], st));
        if (s->launch_real_turn(nload, st)) return fail(AHOM_E_DEVICE, "real");
        HIPCHK(hipEventRecord(ev[++p], st));
        for (int a = 1; a <= P.D - 2; ++a) {
            if (s->launch_axis(a, -1, nload, st)) return fail(AHOM_E_DEVICE, "axis");
            HIPCHK(hipEventRecord(ev[++p], st));
        }
        if (s->launch_spec(nload, st)) return fail(AHOM_E_DEVICE, "spec");
        HIPCHK(hipEventRecord(ev[++p], st));
        for (int a = P.D - 2; a >= 1; --a) {
            if (s->launch_axis(a, +1, nload, st)) return fail(AHOM_E_DEVICE, "axis");
            HIPCHK(hipEventRecord(ev[++p], st));
        }
        if (ahom_launch_reduce(s->dim, r, nload, st)) return fail(AHOM_E_DEVICE, "reduce");
        HIPCHK(hipEventRecord(ev[++p], st));
        HIPCHK(hipEventSynchronize(ev[p]));
        for (int q = 0; q < np; ++q) {
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, ev[q], ev[q + 1]));
            acc[q] += t;
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    const double es = (double)s->es();
    const double field = (double)P.S * es;      // one stored field
    for (int q = 0; q < np; ++q) {
        ms[q] = acc[q] / n_iter;
        if (!bytes) continue;
        double b = 0.0;
        if (q == 0) b = 2.0 * s->ncomp * field + (double)P.m * (s->d_lame_pts ? 16.0 : 1.0);
        else if (q == np - 1) b = 0.0;
        else if (q == P.D - 1) b = 2.0 * s->ncomp * field + 2.0 * s->nt * field;
        else b = 2.0 * s->ncomp * field;
        bytes[q] = b * nload;
    }
    *n_pass = np;
    return AHOM_OK;
}

int ahom_solver_last_timing(const ahom_solver* s, double* ms, int* enq) {
    if (!s) return fail(AHOM_E_ARG, "null solver");
    if (ms) *ms = s->last_ms;
    if (enq) *enq = s->last_enqueued;
    return AHOM_OK;
}

int ahom_solver_last_starts(const ahom_solver* s, int* which, int cap) {
    if (!s || !which || cap < 1) return fail(AHOM_E_ARG, "bad arguments");
    const int n = std::min<int>(cap, (int)s->last_start.size());
    for (int l = 0; l < n; ++l) which[l] = s->last_start[l];
    return AHOM_OK;
}

int ahom_solver_last_restarts(const ahom_solver* s, int* n) {
    if (!s || !n) return fail(AHOM_E_ARG, "null argument");
    *n = s->last_restarts;
    return AHOM_OK;
}

int ahom_solver_history(const ahom_solver* s, int load, double* hist, int cap, int* count) {
    if (!s || !hist || !count || load < 0 || load >= s->last_nload) return fail(AHOM_E_ARG, "bad history arguments");
    const int n = std::min(cap, std::min(s->hist_cap, s->h_st[load].iter + 1));
    HIPCHK(hipMemcpy(hist, s->d_hist + (size_t)load * s->hist_cap, n * sizeof(double), hipMemcpyDeviceToHost));
    *count = n;
    return AHOM_OK;
}

int ahom_solver_cauchy_history(const ahom_solver* s, int load, double* hist, int cap, int* count) {
    if (!s || !hist || !count || load < 0 || load >= s->last_nload) return fail(AHOM_E_ARG, "bad history arguments");
    const int n = std::min(cap, std::min(s->hist_cap, s->h_st[load].iter + 1));
    HIPCHK(hipMemcpy(hist, s->d_chist + (size_t)load * s->hist_cap, n * sizeof(double), hipMemcpyDeviceToHost));
    *count = n;
    return AHOM_OK;
}

}  // extern "C"
