// Kernel argument blocks and launchers (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ahom_internal.h"

enum { REAL_TURN = 0, REAL_TO_REAL = 1, REAL_FROM_REAL = 2 };

// Physics of the cell problem.  Elasticity: the strain field, components
// (11,22,33,23,13,12) / (11,22,12), traction sigma_hat xi with d components.
// Conductivity: the gradient field, components (1,2,3) / (1,2), flux q = k e,
// the normal flux q_hat . xi (one component); the law's per-phase value k
// sits in the first slot of the (lambda, mu) table, the reference k0 in both
// reference constants.
enum { PHYS_ELASTIC = 0, PHYS_THERMAL = 1 };
template <int DIM, int PH> struct Fields {
    static constexpr int N = PH == PHYS_ELASTIC ? (DIM == 3 ? 6 : 3) : DIM;   // real components per point
    static constexpr int NP = (N + 1) / 2;                                     // packed complex transforms
    static constexpr int NT = PH == PHYS_ELASTIC ? DIM : 1;                    // traction components
};
// weight of component c in a full contraction u : v (symmetric off-diagonal
// strain components appear twice)
__host__ __device__ constexpr double field_weight(int ph, int dim, int c) {
    return (ph == PHYS_ELASTIC && c >= dim) ? 2.0 : 1.0;
}
enum { SPEC_TURN = 0, SPEC_INIT = 1 };

// Device-side state of one load case.  iter = n of the iterate being
// processed; done/status/final_buf are set by k_reduce.
struct LoadState {
    int iter;
    int done;
    int status;      // 0 converged, 1 max_iter, 2 diverged
    int final_buf;   // state buffer that holds eps(n) at stop
    double r0;
    double resid;
    double mean[6];
};

struct RealArgs {
    int phys;                 // PHYS_ELASTIC or PHYS_THERMAL
    const Plan* plan;
    void* buf0;
    void* buf1;
    const void* tw;           // Stockham roots in the working precision
    const double2* tw64;      // FP64 roots (four-step twiddles)
    LoadState* st;
    const uint8_t* phase;
    const double* lame_tab;   // (lambda, mu) per phase
    const double* lame_pts;   // or per point (nullptr if unused)
    const uint8_t* phase_t;   // the same, transposed to [column][axis-0 position]
    const double* lame_pts_t; //   (point n*I + c stored at c*L0 + n; fast kernels)
    double lam0, mu0;
    double* sig_part;         // [load][wg][ncomp]
    double* real_io;          // [load][ncomp][m] for TO_REAL / FROM_REAL
    const double* eps_bar;    // [load][ncomp]
    int NC, CS;
    int nload;                // fast path: load cases covered by the persistent grid
    int accumulate;           // TO_REAL: add to real_io instead of overwriting it
    int n_phase;              // entries of lame_tab (fast path stages them in LDS)
    // [load][tile] sums of eps : tau over the tile's points (nullable); with
    // lam0 = mu0 = 0 the law is tau = C : eps and these are eps : C : eps
    // (the conjugate-gradient scheme's <p, A p>)
    double* en_part;
};

struct AxisArgs {
    const Plan* plan;
    void* buf0;
    void* buf1;
    const void* tw;
    const double2* tw64;
    LoadState* st;            // nullptr: always use buf0
    int64_t load_stride, field_stride;
    int axis;
    int slen0_full;           // 1: axis 0 stored at full length (bare DFT)
    int NC, CS;
    int nload, nfield;        // fast path: work items covered by the persistent grid
};

struct SpecArgs {
    int phys;                 // PHYS_ELASTIC or PHYS_THERMAL
    const Plan* plan;
    void* buf0;
    void* buf1;
    void* tbuf;               // traction tau_hat xi of the previous iteration
    const void* tw;
    LoadState* st;
    const double* eps_bar;
    double mu0, beta;
    double lam0_init;          // lambda0 (used by SPEC_INIT)
    double* res_part;         // [load][wg]
    double* cau_part;         // [load][wg] Cauchy-measure partial sums (nullable)
    int NC, CS;
    int nload;                // fast path: load cases covered by the persistent grid
    int resid_period;         // evaluate the residual for iter = 0 (mod resid_period) and at max_iter
    int max_iter;
    // defect correction (FP32 refinement): the traction that enters Gamma0 is
    // t + toff (toff in the working precision, [load][NT][S]); when dout is
    // set, the traction step d = t(n) - t(n-1) is also stored as FP32 complex
    // in dout and its negative in dneg (same layout).
    const void* toff;
    void* dout;
    void* dneg;
    // conjugate-gradient traction recurrence (nullable): with alpha =
    // cg_alpha[load] the pass writes t <- t + alpha tau_hat xi and sums |t|^2
    // of the new t (the equilibrium residual of the updated iterate) instead
    // of t <- tau_hat xi with |t(n+1) - t(n)|^2
    const double* cg_alpha;
};

// traction traffic of iteration n: read (and evaluate r(n)) / write t(n + 1)
__host__ __device__ inline bool ahom_check_iter(int n, int period, int max_iter) {
    return period <= 1 || n % period == 0 || n >= max_iter;
}
__host__ __device__ inline bool ahom_write_traction(int n, int period, int max_iter) {
    return period <= 1 || ahom_check_iter(n + 1, period, max_iter);
}

struct ReduceArgs {
    int phys;                 // PHYS_ELASTIC or PHYS_THERMAL
    LoadState* st;
    const double* sig_part;
    const double* res_part;
    double* hist;
    int n_real, n_spec, hist_cap;
    int64_t m;
    double tol;
    int max_iter;
    int resid_period;
    const double* sig_base;   // [load][ncomp] added to the mean stress (nullptr: none)
    // Cauchy measure (nullable chist: not recorded): c(n) = sqrt(cau_scale *
    // sum of cau_part) / norm0[load], cau_scale = m / (2 mu0^2)
    const double* cau_part;
    double* chist;
    const double* norm0;
    double cau_scale;
    int stop_cauchy;          // 1: stop on c(n) <= tol instead of r(n) <= tol (needs chist)
};

struct FillArgs {
    void* buf;
    const double* eps_bar;
    int64_t S, row;
    int nfield;
};

struct ReorderArgs {
    const Plan* plan;
    const void* in;
    void* out;
    double scale;
    int dir;
};

int ahom_launch_real(int prec, int dim, int mode, const RealArgs& a, int nwg, int nload, size_t lds, hipStream_t s);
int ahom_launch_axis(int prec, int dir, const AxisArgs& a, int nwg, int nfield, int nload, size_t lds, hipStream_t s);
int ahom_launch_spec(int prec, int dim, const SpecArgs& a, int nwg, int nload, size_t lds, hipStream_t s);
int ahom_launch_spec_init(int prec, int dim, const SpecArgs& a, int nwg, int nload, size_t lds, hipStream_t s);
int ahom_launch_reduce(int dim, const ReduceArgs& a, int nload, hipStream_t s);
int ahom_launch_fill(int prec, const FillArgs& a, int nload, hipStream_t s);
int ahom_launch_reset(LoadState* st, int n, hipStream_t s);
int ahom_launch_zero(int prec, void* p, int64_t n_complex, hipStream_t s);
int ahom_launch_reorder(int prec, const ReorderArgs& a, int64_t m, hipStream_t s);
// out64[l] = (base64 ? base64[l] : 0) + (double) in32[l], per load l, where in32
// is the state buffer st32[l].final_buf of a working-precision-FP32 solver
struct GatherArgs {
    double2* out;
    const double2* base;
    const float2* in0;
    const float2* in1;
    const LoadState* st;
    int64_t per_load;         // complex elements per load
};
int ahom_launch_refine_gather(const GatherArgs& a, int nload, hipStream_t s);
// dst[c * L0 + n] = src[n * I + c] for elements of `bytes` bytes (1 or 16)
int ahom_launch_transpose(const void* src, void* dst, int64_t L0, int64_t I, int bytes, hipStream_t s);

// ---- conjugate gradients on the same passes (ahom_cg.hip).  Per load: the
// direction p in state buffer buf[iter & 1], the operator output -Gamma0 C p
// in buf[(iter + 1) & 1] (the passes run with the law C : eps and cg_alpha
// set), the iterate eps_bar + x in xbuf and the residual field r in rbuf;
// all in the state layout (half spectrum along axis 0).
struct CgScalars {
    double rr;        // <r, r>_C0 of the current residual field
    double alpha;     // step length of the current update (1 for the start)
    double beta;      // direction update after the current step
    double pcp;       // <p, C p> of the current direction
    double rr0;       // <r, r>_C0 of the start (inner solves of the mixed-precision scheme)
};

struct CgArgs {
    int phys;                 // PHYS_ELASTIC or PHYS_THERMAL
    LoadState* st;
    CgScalars* cg;
    double* alpha;            // [load] alpha, read by the spectral pass
    void* buf0;
    void* buf1;
    void* xbuf;
    void* rbuf;
    const double* sig_part;   // [load][n_real][ncomp] sums of C p
    const double* en_part;    // [load][n_real] sums of p : C p
    const double* res_part;   // [load][n_spec] |t|^2 of the updated iterate's traction
    double* rr_part;          // [load][nblk] sums of r : C0 : r (update kernel)
    double* hist;             // [load][hist_cap] residual history
    int n_real, n_spec, nblk, hist_cap;
    int64_t S;                // stored complex elements per field
    int64_t I;                // S / stored length of axis 0
    int64_t m;
    int L0;                   // transform length of axis 0 (Hermitian weights)
    double lam0, mu0;
    double tol;
    int max_iter;
    int start;                // 1: the start (r(0), p_0 = r_0), 0: an update
    int no_x;                 // 1: the iterate x is not formed (no field output asked)
    // > 0: an inner solve of the mixed-precision scheme: the recorded residual
    // is sqrt(<r, r>_C0 / <r(0), r(0)>_C0) and the stop is that ratio <= rr_stop
    double rr_stop;
};

int ahom_launch_cg_alpha(int dim, const CgArgs& a, int nload, hipStream_t s);
int ahom_launch_cg_update(int prec, int dim, const CgArgs& a, int nload, hipStream_t s);
int ahom_launch_cg_reduce(int dim, const CgArgs& a, int nload, hipStream_t s);
int ahom_launch_cg_direction(int prec, int dim, const CgArgs& a, int nload, hipStream_t s);
// workgroups per load of the update kernel (size of rr_part)
int ahom_cg_blocks(int64_t S);
// out[i] = (float) in[i] for n complex values
int ahom_launch_cg_demote(const double2* in, float2* out, int64_t n, hipStream_t s);
// x[i] -= d[i], i < n
int ahom_launch_cg_sub(double2* x, const double2* d, int64_t n, hipStream_t s);

// ---- batched solves: one persistent launch over many (pattern, load) items.
// A workgroup takes an item from the queue and runs Algorithm 1 for it to the
// end (all passes, its own loop control), so no grid-wide synchronisation is
// needed.  FP32 items with refine > 0 run the defect-correction restarts
// in place (FP64 companion buffers per item).
struct BatchItem {
    RealArgs ra;                       // working-precision passes; load index 0
    AxisArgs ax[AHOM_MAX_AXES];        // middle axes 1..D-2
    SpecArgs sa;                       // plain stage (eps_bar = the load)
    SpecArgs sa_corr;                  // correction stage (eps_bar = 0, toff set)
    RealArgs ra64;                     // FP64 companion (defect evaluation)
    AxisArgs ax64[AHOM_MAX_AXES];
    SpecArgs sa64;                     // dout / dneg -> toff / tbuf of the item
    int D;
    int64_t S, row, m;                 // stored complex per field, fill row, points
    int64_t t_real, t_spec, t_axis[AHOM_MAX_AXES];          // tiles per pass
    int64_t t_real64, t_spec64, t_axis64[AHOM_MAX_AXES];
    double* hist;                      // [hist_cap] residual history
    double* chist;                     // [hist_cap] Cauchy measure history
    int hist_cap;
    LoadState* st;                     // result state of the item
    int* restarts;
    int k;                             // workgroups that iterate the item together (>= 1)
    int* gcount;                       // group barrier arrivals (zeroed before each launch)
    double* gpart;                     // [2][k][8] partial sums of the group's workgroups
    double* sbase;                     // [8] FP32 restarts: mean stress of the FP64 base iterate
};

struct BatchArgs {
    const BatchItem* items;
    const int* order;                  // queue position -> item
    const int* qslot;                  // queue position -> slot of the item's group
    int n_queue;                       // queue positions (sum of the items' k)
    int* counter;                      // queue head (zeroed before each launch)
    double tol, refine;
    int max_iter, resid_period;
    int refine_on;                     // FP32 items: defect-correction restarts
    int phase;                         // BATCH_FP32 launches: 0 first stage, 1 correction stage
    long long group_wait;              // group barrier wait limit (100 MHz ticks)
};

// batch kernel kinds: the whole solve of FP64 items; the FP32 stages (first or
// correction); the FP64 step of an FP32 item's restart
enum { BATCH_SOLVE = 0, BATCH_FP32 = 1, BATCH_RESTART64 = 2 };

// queue head and group barrier counters to zero (plain kernel: safe inside a captured graph)
int ahom_launch_batch_reset(int* counter, int* gcount, int n_items, hipStream_t s);
// threads per workgroup of the FP32 stage kernel: its 235 VGPRs allow 8
// waves per CU, held as one workgroup so that its tiles get all of the LDS
constexpr int kBatchWg32 = 512;
// threads per workgroup of a batch kernel kind
int ahom_batch_wg_size(int kind);
int ahom_launch_batch(int kind, int dim, const BatchArgs& a, int nwg, size_t lds, hipStream_t s);
// static LDS bytes of the batch kernels (reduction scratch and item state) with wgs threads
size_t ahom_batch_static_lds(int dim, int wgs);
// resident workgroups per CU of a batch kernel kind with `lds` dynamic LDS bytes
int ahom_batch_occupancy(int kind, int dim, size_t lds);

// ---- power-of-two fast path (ahom_fast.hip)
enum { FAST_REAL = 0, FAST_AXIS = 1, FAST_SPEC = 2 };
struct FastGeom {
    int NC = 1, threads = 64;
    bool persistent = false;
    size_t lds = 0;
};
constexpr int AHOM_FAST_VARIANTS = 5;   // tile width x schedule (+ register-resident real pass), chosen by the autotuner
bool ahom_fast_geom(int prec, int kind, int dim, int L, int variant, FastGeom* g, int phys = PHYS_ELASTIC);
// total = tiles of the pass (all loads/fields); the grid is sized from the occupancy API
int ahom_launch_fast_real(int prec, int dim, int L, int variant, const RealArgs& a, int64_t total, int ncu, hipStream_t s);
int ahom_launch_fast_axis(int prec, int dir, int L, int variant, const AxisArgs& a, int64_t total, int ncu, hipStream_t s);
int ahom_launch_fast_spec(int prec, int dim, int L, int variant, const SpecArgs& a, int64_t total, int ncu, hipStream_t s);
