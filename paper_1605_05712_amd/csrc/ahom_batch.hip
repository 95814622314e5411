// Batched solves: Algorithm 1 (Sec. 3.2) on many patterns P(M_i) of uneven
// size in one persistent launch (optionally replayed from a HIP graph).
//
// Every member has its own Smith form, plan and twiddles; every
// (member, load) pair is an item with its own state buffers.  The plan and
// tile widths of each distinct Smith shape are picked by timing the
// candidates on the device (per-process cache).
#include <rocprofiler-sdk-roctx/roctx.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ahom.h"
#include "ahom_internal.h"
#include "ahom_kernels.h"

namespace {

int bfail(int code, const std::string& msg) {
    ahom_set_error(msg);
    return code;
}

#define BCHK(expr)                                                                                     \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return bfail(AHOM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// plan variants tried by the autotuner: (largest radix, LDS budget divisor)
struct Variant {
    int max_radix;
    int budget_div;
};
const Variant kVariants[] = {{8, 1}, {4, 1}, {8, 2}, {4, 2}};
constexpr int kNumVariants = 4;
// dynamic LDS per workgroup for the largest tiles (every batch kernel runs one
// workgroup per CU: 512 threads for the FP32 stages, 256 for the FP64
// kernels), less where the kernel's static LDS leaves less of the 160 KB
constexpr size_t kBudget = 128 * 1024;
constexpr int kMaxNC = 512;
constexpr int kGroupMax = 8;            // workgroups per item at most
constexpr int kGroupPart = 2 * kGroupMax * 8;   // doubles of an item's group partial sums

struct PassGeo {
    int NC = 1, CS = 1;
    int64_t tiles = 0;
    size_t lds = 0;
};

PassGeo pass_geo(int L, int64_t ncols, int nbuf, size_t es, size_t budget) {
    PassGeo g;
    g.CS = L + 1;
    const size_t twl = (size_t)L * es;   // LDS copy of the axis's twiddle table
    int64_t nc = (int64_t)((budget > twl ? budget - twl : 0) / ((size_t)nbuf * g.CS * es));
    nc = std::max<int64_t>(1, std::min<int64_t>({nc, ncols, (int64_t)kMaxNC}));
    g.NC = (int)nc;
    g.tiles = (ncols + nc - 1) / nc;
    g.lds = (size_t)nbuf * g.NC * g.CS * es + twl;
    return g;
}

struct Member {
    SmithForm sf{};
    Plan plan{};
    std::vector<double> tw;
    Plan* d_plan = nullptr;
    double2* d_tw64 = nullptr;
    float2* d_tw32 = nullptr;
    uint8_t* d_phase = nullptr;
    double* d_lame = nullptr;
    bool has_cell = false;          // transformed pattern P_L(M): cell matrix L (d*d, row-major)
    double cell[9] = {};
    double lam0 = 0, mu0 = 0;
    double lam_lo = 0, lam_hi = 0, mu_lo = 0, mu_hi = 0;
    bool has_material = false, ref_set = false;
    int variant = -1;
};

struct ShapeKey {
    int prec, d;
    int64_t e0, e1, e2;
    bool operator<(const ShapeKey& o) const { return std::tie(prec, d, e0, e1, e2) < std::tie(o.prec, o.d, o.e0, o.e1, o.e2); }
};
std::map<ShapeKey, int>& shape_cache() {
    static std::map<ShapeKey, int> c;
    return c;
}
std::mutex& shape_mutex() {
    static std::mutex m;
    return m;
}

template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

}  // namespace

struct ahom_batch {
    int d = 2, ncomp = 3, nt = 2, prec = 0;
    ahom_config cfg{};
    hipStream_t stream = nullptr;
    std::vector<Member> mem;
    int forced_variant = -1;          // autotuner trials: fixed plan variant
    // per-solve device state
    int nload = 0;
    char* arena = nullptr;            // every item buffer
    BatchItem* d_items = nullptr;
    int* d_order = nullptr;
    int* d_qslot = nullptr;
    int* d_gcount = nullptr;
    double* d_gpart = nullptr;
    double* d_sbase = nullptr;
    int n_queue = 0;
    int* d_counter = nullptr;
    LoadState* d_st = nullptr;
    LoadState* d_st_base = nullptr;   // final_buf = 1: where the FP64 base iterate is
    int* d_restarts = nullptr;
    double* d_hist = nullptr;
    double* d_epsbar = nullptr;
    double* d_zero = nullptr;
    std::vector<BatchItem> h_items;
    std::vector<LoadState> h_st;
    std::vector<int> h_restarts;
    // the first kernel kind of a solve (BATCH_SOLVE for FP64, BATCH_FP32) and
    // the FP64 restart step: dynamic LDS and workgroups of each
    int kind = BATCH_SOLVE;
    size_t lds = 0, lds64 = 0;
    int nwg = 1, nwg64 = 1;
    int graph_rounds = 2;             // restart rounds captured in the graph
    int hist_cap = 0;
    // graph of (queue reset, batch kernel) on a stream of its own
    hipStream_t gstream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double last_ms = 0.0;

    size_t es() const { return prec == AHOM_FP64 ? 16 : 8; }
    // dynamic LDS for the tiles of plan variant v in precision pr (at most
    // the CU's LDS less the kernel's static LDS)
    size_t tile_budget(int pr, int v) const {
        const size_t rest = 160 * 1024 - ahom_batch_static_lds(d, pr == AHOM_FP64 ? AHOM_WG : kBatchWg32);
        return std::min(kBudget, rest & ~(size_t)1023) / (size_t)kVariants[v].budget_div;
    }
    bool refine_on() const { return prec == AHOM_FP32_MIXED && cfg.refine > 0.0; }

    void free_items() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        dfree(arena); dfree(d_items); dfree(d_order); dfree(d_qslot); dfree(d_gcount); dfree(d_gpart); dfree(d_sbase);
        dfree(d_counter); dfree(d_st); dfree(d_st_base);
        dfree(d_restarts); dfree(d_hist); dfree(d_epsbar); dfree(d_zero);
        nload = 0;
    }

    ~ahom_batch() {
        free_items();
        for (auto& m : mem) {
            dfree(m.d_plan); dfree(m.d_tw64); dfree(m.d_tw32); dfree(m.d_phase); dfree(m.d_lame);
        }
        if (gstream) (void)hipStreamDestroy(gstream);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
    }

    int set_plan(Member& mb, int variant) {
        std::string err;
        int rc = ahom_build_plan_ex(mb.sf, 256, kVariants[variant].max_radix, &mb.plan, &err);
        if (rc) return bfail(rc, err);
        if (mb.has_cell && (rc = ahom_plan_set_cell(&mb.plan, mb.sf.d, mb.cell, &err))) return bfail(rc, err);
        ahom_build_twiddles(&mb.plan, &mb.tw);
        dfree(mb.d_plan); dfree(mb.d_tw64); dfree(mb.d_tw32);
        BCHK(hipMalloc((void**)&mb.d_plan, sizeof(Plan)));
        BCHK(hipMemcpy(mb.d_plan, &mb.plan, sizeof(Plan), hipMemcpyHostToDevice));
        const size_t n = std::max<size_t>(mb.tw.size() / 2, 1);
        BCHK(hipMalloc((void**)&mb.d_tw64, n * sizeof(double2)));
        BCHK(hipMalloc((void**)&mb.d_tw32, n * sizeof(float2)));
        std::vector<float> t32(mb.tw.size());
        for (size_t i = 0; i < mb.tw.size(); ++i) t32[i] = (float)mb.tw[i];
        if (!mb.tw.empty()) {
            BCHK(hipMemcpy(mb.d_tw64, mb.tw.data(), mb.tw.size() / 2 * sizeof(double2), hipMemcpyHostToDevice));
            BCHK(hipMemcpy(mb.d_tw32, t32.data(), t32.size() / 2 * sizeof(float2), hipMemcpyHostToDevice));
        }
        mb.variant = variant;
        return AHOM_OK;
    }

    // per-pass tiles of a member in element size es
    void geometry(const Member& mb, size_t esz, size_t budget, PassGeo* real, PassGeo* spec, PassGeo* axis) const {
        const Plan& P = mb.plan;
        // LDS buffers of a tile: the fields and a ping-pong buffer of the same size
        *real = pass_geo(P.ax[0].len, P.S / P.ax[0].slen, 2 * (d == 3 ? 3 : 2), esz, budget);
        *spec = pass_geo(P.ax[P.D - 1].len, P.S / P.ax[P.D - 1].len, 2 * ncomp, esz, budget);
        for (int a = 1; a <= P.D - 2; ++a) {
            int64_t O = 1, I = 1;
            for (int b = 0; b < a; ++b) O *= P.ax[b].slen;
            for (int b = a + 1; b < P.D; ++b) I *= P.ax[b].slen;
            axis[a] = pass_geo(P.ax[a].len, O * I, 2, esz, budget);
        }
    }

    int autotune();
    int build_items(int n_load);
    int run(bool use_graph);
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

int ahom_batch::build_items(int n_load) {
    free_items();
    const int nm = (int)mem.size();
    const int n_items = nm * n_load;
    hist_cap = cfg.max_iter + 1;
    const bool ref = refine_on();
    // arena layout per item
    std::vector<size_t> off(n_items + 1, 0);
    std::vector<int64_t> Sv(nm);
    for (int i = 0; i < nm; ++i) Sv[i] = mem[i].plan.S;
    for (int q = 0; q < n_items; ++q) {
        const int64_t S = Sv[q / n_load];
        size_t b = 2 * align256((size_t)ncomp * S * es()) + align256((size_t)nt * S * es()) + 2 * align256((size_t)hist_cap * 8);
        if (ref) b += align256((size_t)nt * S * 8) + 2 * align256((size_t)ncomp * S * 16) + align256((size_t)nt * S * 16);
        off[q + 1] = off[q] + b;
    }
    BCHK(hipMalloc((void**)&arena, std::max<size_t>(off[n_items], 256)));
    BCHK(hipMalloc((void**)&d_items, n_items * sizeof(BatchItem)));
    BCHK(hipMalloc((void**)&d_counter, 256));
    BCHK(hipMalloc((void**)&d_gcount, n_items * sizeof(int)));
    BCHK(hipMalloc((void**)&d_gpart, (size_t)n_items * kGroupPart * sizeof(double)));
    BCHK(hipMalloc((void**)&d_sbase, (size_t)n_items * 8 * sizeof(double)));
    BCHK(hipMalloc((void**)&d_st, n_items * sizeof(LoadState)));
    BCHK(hipMalloc((void**)&d_st_base, sizeof(LoadState)));
    BCHK(hipMalloc((void**)&d_restarts, n_items * sizeof(int)));
    BCHK(hipMalloc((void**)&d_epsbar, (size_t)n_load * ncomp * sizeof(double)));
    BCHK(hipMalloc((void**)&d_zero, (size_t)ncomp * sizeof(double)));
    {
        LoadState b{};
        b.final_buf = 1;
        BCHK(hipMemcpy(d_st_base, &b, sizeof(LoadState), hipMemcpyHostToDevice));
        std::vector<double> z(ncomp, 0.0);
        BCHK(hipMemcpy(d_zero, z.data(), z.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    h_items.assign(n_items, BatchItem{});
    size_t lds_main = 0, lds_r64 = 0;
    for (int q = 0; q < n_items; ++q) {
        const int i = q / n_load, l = q % n_load;
        const Member& mb = mem[i];
        const Plan& P = mb.plan;
        const int64_t S = P.S;
        const size_t budget = tile_budget(AHOM_FP64, mb.variant);
        const size_t budget_main = tile_budget(prec, mb.variant);
        char* p = arena + off[q];
        auto take = [&](size_t bytes) { char* r = p; p += align256(bytes); return (void*)r; };
        void* buf0 = take((size_t)ncomp * S * es());
        void* buf1 = take((size_t)ncomp * S * es());
        void* tbuf = take((size_t)nt * S * es());
        double* hist = (double*)take((size_t)hist_cap * 8);
        double* chist = (double*)take((size_t)hist_cap * 8);
        void *toff = nullptr, *b64_0 = nullptr, *b64_1 = nullptr, *tb64 = nullptr;
        if (ref) {
            toff = take((size_t)nt * S * 8);
            b64_0 = take((size_t)ncomp * S * 16);
            b64_1 = take((size_t)ncomp * S * 16);
            tb64 = take((size_t)nt * S * 16);
        }
        BatchItem& it = h_items[q];
        it.D = P.D;
        it.S = S;
        it.row = S / P.ax[0].slen;
        it.m = P.m;
        it.hist = hist;
        it.chist = chist;
        it.hist_cap = hist_cap;
        it.st = d_st + q;
        it.restarts = d_restarts + q;
        it.k = 1;
        it.gcount = d_gcount + q;
        it.gpart = d_gpart + (size_t)q * kGroupPart;
        it.sbase = d_sbase + (size_t)q * 8;
        const double beta = (mb.lam0 + mb.mu0) / (mb.lam0 + 2.0 * mb.mu0);
        auto fill_args = [&](int pr, void* b0, void* b1, void* tb, RealArgs* ra, AxisArgs* ax, SpecArgs* sa,
                             int64_t* t_real, int64_t* t_spec, int64_t* t_axis, size_t& lds_max, size_t bud) {
            const size_t esz = pr == AHOM_FP64 ? 16 : 8;
            PassGeo gr, gs, ga[AHOM_MAX_AXES];
            geometry(mb, esz, bud, &gr, &gs, ga);
            const void* tw = pr == AHOM_FP64 ? (const void*)mb.d_tw64 : (const void*)mb.d_tw32;
            *ra = RealArgs{};
            ra->plan = mb.d_plan; ra->buf0 = b0; ra->buf1 = b1; ra->tw = tw; ra->tw64 = mb.d_tw64;
            ra->st = it.st; ra->phase = mb.d_phase; ra->lame_tab = mb.d_lame;
            ra->lam0 = mb.lam0; ra->mu0 = mb.mu0; ra->eps_bar = d_epsbar + (size_t)l * ncomp;
            ra->NC = gr.NC; ra->CS = gr.CS; ra->nload = 1;
            *t_real = gr.tiles;
            lds_max = std::max(lds_max, gr.lds);
            for (int a = 1; a <= P.D - 2; ++a) {
                AxisArgs& x = ax[a];
                x = AxisArgs{};
                x.plan = mb.d_plan; x.buf0 = b0; x.buf1 = b1; x.tw = tw; x.tw64 = mb.d_tw64; x.st = it.st;
                x.load_stride = (int64_t)ncomp * S; x.field_stride = S; x.axis = a;
                x.NC = ga[a].NC; x.CS = ga[a].CS; x.nload = 1; x.nfield = ncomp;
                t_axis[a] = ga[a].tiles;
                lds_max = std::max(lds_max, ga[a].lds);
            }
            *sa = SpecArgs{};
            sa->plan = mb.d_plan; sa->buf0 = b0; sa->buf1 = b1; sa->tbuf = tb; sa->tw = tw; sa->st = it.st;
            sa->eps_bar = d_epsbar + (size_t)l * ncomp; sa->mu0 = mb.mu0; sa->beta = beta;
            sa->NC = gs.NC; sa->CS = gs.CS; sa->nload = 1;
            sa->resid_period = cfg.resid_period; sa->max_iter = cfg.max_iter;
            *t_spec = gs.tiles;
            lds_max = std::max(lds_max, gs.lds);
        };
        fill_args(prec, buf0, buf1, tbuf, &it.ra, it.ax, &it.sa, &it.t_real, &it.t_spec, it.t_axis, lds_main, budget_main);
        it.sa_corr = it.sa;
        if (ref) {
            it.sa_corr.eps_bar = d_zero;
            it.sa_corr.toff = toff;
            fill_args(AHOM_FP64, b64_0, b64_1, tb64, &it.ra64, it.ax64, &it.sa64, &it.t_real64, &it.t_spec64, it.t_axis64,
                      lds_r64, budget);
            it.sa64.resid_period = 1;
            it.sa64.max_iter = 1;
            it.sa64.dout = toff;
            it.sa64.dneg = tbuf;
        }
    }
    kind = prec == AHOM_FP64 ? BATCH_SOLVE : BATCH_FP32;
    lds = lds_main;
    lds64 = lds_r64;
    if (std::max(lds + ahom_batch_static_lds(d, ahom_batch_wg_size(kind)), lds64 + ahom_batch_static_lds(d, AHOM_WG)) >
        160 * 1024)
        return bfail(AHOM_E_UNSUPPORTED_SIZE, "batch tiles exceed the LDS");
    int ncu = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0) ncu = n;
    }
    const int occ = std::max(1, ahom_batch_occupancy(kind, d, lds));
    const int cap = std::max(1, occ * ncu);   // workgroups resident at once
    const int cap64 = std::max(1, std::max(1, ahom_batch_occupancy(BATCH_RESTART64, d, lds64)) * ncu);
    // Items much larger than a workgroup's fair share are iterated by a group
    // of k workgroups (tiles of every pass dealt round-robin, a group barrier
    // between passes).  k <= nwg keeps the queue deadlock-free: a group's queue
    // positions are consecutive, so at most the group at the queue head is
    // incomplete and the workgroups of the complete ones join it when done.
    {
        double total = 0.0;
        for (int q = 0; q < n_items; ++q) total += (double)Sv[q / n_load];
        const int kmax = std::min(kGroupMax, std::min(cap, cap64));
        // share factor: measured best 2 for the FP32 stage kernel on the
        // 512-member 2-D batch (1.5: +3 %, 3: +8 %, 1: +44 %) and 3 for the
        // FP64 kernel on the 393-member sweep (2: +8 %, 4: +6 %)
        const double fac = kind == BATCH_FP32 ? 2.0 : 3.0;
        for (int q = 0; q < n_items; ++q) {
            const double share = fac * (double)Sv[q / n_load] * cap / std::max(total, 1.0);
            h_items[q].k = std::max(1, std::min(kmax, (int)std::ceil(share)));
        }
    }
    BCHK(hipMemcpy(d_items, h_items.data(), n_items * sizeof(BatchItem), hipMemcpyHostToDevice));
    // largest members first (the queue hands them out in this order), one
    // queue position per workgroup of an item's group
    std::vector<int> order(n_items);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return Sv[a / n_load] > Sv[b / n_load]; });
    std::vector<int> qitem, qslot;
    for (int q : order)
        for (int sl = 0; sl < h_items[q].k; ++sl) { qitem.push_back(q); qslot.push_back(sl); }
    n_queue = (int)qitem.size();
    nwg = std::min(n_queue, cap);   // >= every item's k
    nwg64 = std::min(n_queue, cap64);
    BCHK(hipMalloc((void**)&d_order, n_queue * sizeof(int)));
    BCHK(hipMalloc((void**)&d_qslot, n_queue * sizeof(int)));
    BCHK(hipMemcpy(d_order, qitem.data(), n_queue * sizeof(int), hipMemcpyHostToDevice));
    BCHK(hipMemcpy(d_qslot, qslot.data(), n_queue * sizeof(int), hipMemcpyHostToDevice));
    h_st.assign(n_items, LoadState{});
    h_restarts.assign(n_items, 0);
    nload = n_load;
    return AHOM_OK;
}

int ahom_batch::run(bool use_graph) {
    BatchArgs a{};
    a.items = d_items;
    a.order = d_order;
    a.qslot = d_qslot;
    a.n_queue = n_queue;
    a.counter = d_counter;
    a.tol = cfg.tol;
    a.refine = cfg.refine;
    a.max_iter = cfg.max_iter;
    a.resid_period = cfg.resid_period;
    a.refine_on = refine_on() ? 1 : 0;
    // group barrier wait limit: 4 s; AHOM_BATCH_GROUP_WAIT (ticks of the
    // 100 MHz clock) lets a test force the time-out path from the host
    a.group_wait = 400000000LL;
    if (const char* w = getenv("AHOM_BATCH_GROUP_WAIT")) a.group_wait = std::max(0LL, atoll(w));
    hipStream_t s = use_graph ? gstream : stream;
    const int n_items = (int)h_items.size();
    // one launch of a kernel kind over the whole queue, after zeroing the
    // queue head and the group barrier counters
    auto launch = [&](hipStream_t st, int k, int phase) -> int {
        a.phase = phase;
        if (ahom_launch_batch_reset(d_counter, d_gcount, n_items, st)) return -1;
        return k == BATCH_RESTART64 ? ahom_launch_batch(k, d, a, nwg64, lds64, st) : ahom_launch_batch(k, d, a, nwg, lds, st);
    };
    // FP32 with restarts: the first stage, then rounds of (FP64 restart step,
    // correction stage); an item that needs no further restart skips a round
    auto launch_solve = [&](hipStream_t st, int rounds) -> int {
        if (launch(st, kind, 0)) return -1;
        for (int r = 0; r < rounds; ++r)
            if (launch(st, BATCH_RESTART64, 0) || launch(st, BATCH_FP32, 1)) return -1;
        return 0;
    };
    const bool ref = refine_on();
    auto pending = [&]() {
        int n = 0;
        for (const LoadState& x : h_st) n += ref && x.done && x.status == 0 && x.resid > cfg.tol;
        return n;
    };
    const int rounds = ref ? graph_rounds : 0;
    if (use_graph && !gexec) {
        BCHK(hipStreamBeginCapture(gstream, hipStreamCaptureModeThreadLocal));
        const int r1 = launch_solve(gstream, rounds);
        hipGraph_t g = nullptr;
        BCHK(hipStreamEndCapture(gstream, &g));
        graph = g;
        if (r1) return bfail(AHOM_E_DEVICE, "batch graph capture failed");
        BCHK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    }
    BCHK(hipEventRecord(ev0, s));
    if (use_graph) {
        BCHK(hipGraphLaunch(gexec, s));
    } else {
        if (launch_solve(s, rounds)) return bfail(AHOM_E_DEVICE, "launch batch kernels");
    }
    BCHK(hipEventRecord(ev1, s));
    BCHK(hipEventSynchronize(ev1));
    BCHK(hipMemcpy(h_st.data(), d_st, h_st.size() * sizeof(LoadState), hipMemcpyDeviceToHost));
    // items still short of tol after the planned rounds: more rounds, one at
    // a time (each adds at least one update to every such item, so max_iter
    // bounds them); the next graph capture plans for as many
    int extra = 0;
    while (pending() > 0) {
        if (launch(s, BATCH_RESTART64, 0) || launch(s, BATCH_FP32, 1)) return bfail(AHOM_E_DEVICE, "launch batch kernels");
        BCHK(hipEventRecord(ev1, s));
        BCHK(hipEventSynchronize(ev1));
        BCHK(hipMemcpy(h_st.data(), d_st, h_st.size() * sizeof(LoadState), hipMemcpyDeviceToHost));
        ++extra;
    }
    if (extra > 0) {
        graph_rounds += extra;
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
    }
    float ms = 0.f;
    BCHK(hipEventElapsedTime(&ms, ev0, ev1));
    last_ms = ms;
    BCHK(hipMemcpy(h_restarts.data(), d_restarts, h_restarts.size() * sizeof(int), hipMemcpyDeviceToHost));
    return AHOM_OK;
}

// Time every plan variant of each distinct Smith shape on a one-member batch
// of that shape and keep the fastest (per-process cache).
int ahom_batch::autotune() {
    for (auto& mb : mem) {
        if (forced_variant >= 0) {
            if (mb.variant != forced_variant) {
                int rc = set_plan(mb, forced_variant);
                if (rc) return rc;
            }
            continue;
        }
        ShapeKey key{prec, d, mb.sf.e[0], mb.sf.e[1], d == 3 ? mb.sf.e[2] : 0};
        int best = -1;
        {
            std::lock_guard<std::mutex> g(shape_mutex());
            auto f = shape_cache().find(key);
            if (f != shape_cache().end()) best = f->second;
        }
        if (best < 0) {
            // distinct candidates only (same plan and tiles -> same kernel work)
            std::vector<std::pair<double, int>> times;
            std::vector<std::vector<int>> seen;
            for (int v = 0; v < kNumVariants; ++v) {
                Member probe{};
                probe.sf = mb.sf;
                std::string err;
                if (ahom_build_plan_ex(probe.sf, 256, kVariants[v].max_radix, &probe.plan, &err)) continue;
                PassGeo gr, gs, ga[AHOM_MAX_AXES];
                geometry(probe, es(), tile_budget(prec, v), &gr, &gs, ga);
                std::vector<int> sig = {gr.NC, gs.NC};
                for (int a = 0; a < probe.plan.D; ++a)
                    for (int s2 = 0; s2 < probe.plan.ax[a].nstage; ++s2) sig.push_back(probe.plan.ax[a].radix[s2]);
                for (int a = 1; a <= probe.plan.D - 2; ++a) sig.push_back(ga[a].NC);
                if (std::find(seen.begin(), seen.end(), sig) != seen.end()) continue;
                seen.push_back(sig);
                // one-member trial batch of this shape: diag(e), two phases
                ahom_batch* t = new ahom_batch();
                t->d = d; t->ncomp = ncomp; t->nt = nt; t->prec = prec;
                t->cfg = cfg;
                t->cfg.tol = 0.0;
                t->cfg.max_iter = 6;
                t->cfg.refine = -1.0;
                t->stream = stream;
                t->forced_variant = v;
                t->mem.resize(1);
                Member& pm = t->mem[0];
                pm.sf = mb.sf;
                int rc = t->set_plan(pm, v);
                std::vector<uint8_t> ph((size_t)pm.plan.m);
                for (size_t k = 0; k < ph.size(); ++k) ph[k] = (uint8_t)((k * 2654435761u >> 7) & 1);
                const double lame[4] = {1.0, 1.0, 10.0, 10.0};
                if (!rc && hipMalloc((void**)&pm.d_phase, ph.size()) != hipSuccess) rc = AHOM_E_DEVICE;
                if (!rc && hipMalloc((void**)&pm.d_lame, sizeof(lame)) != hipSuccess) rc = AHOM_E_DEVICE;
                if (!rc && hipMemcpy(pm.d_phase, ph.data(), ph.size(), hipMemcpyHostToDevice) != hipSuccess) rc = AHOM_E_DEVICE;
                if (!rc && hipMemcpy(pm.d_lame, lame, sizeof(lame), hipMemcpyHostToDevice) != hipSuccess) rc = AHOM_E_DEVICE;
                pm.lam0 = 5.5; pm.mu0 = 5.5; pm.has_material = true;
                if (!rc && (hipEventCreate(&t->ev0) != hipSuccess || hipEventCreate(&t->ev1) != hipSuccess)) rc = AHOM_E_DEVICE;
                if (!rc) rc = t->build_items(1);
                if (!rc) {
                    std::vector<double> eb(ncomp, 0.0);
                    eb[0] = 1.0;
                    if (hipMemcpy(t->d_epsbar, eb.data(), eb.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) rc = AHOM_E_DEVICE;
                }
                double best_ms = 1e30;
                for (int r = 0; !rc && r < 3; ++r) {
                    rc = t->run(false);
                    if (!rc && r > 0) best_ms = std::min(best_ms, t->last_ms);
                }
                delete t;
                if (rc) return rc;
                times.push_back({best_ms, v});
            }
            best = 0;
            if (!times.empty()) best = std::min_element(times.begin(), times.end())->second;
            std::lock_guard<std::mutex> g(shape_mutex());
            shape_cache()[key] = best;
        }
        if (mb.variant != best) {
            int rc = set_plan(mb, best);
            if (rc) return rc;
        }
    }
    return AHOM_OK;
}

extern "C" {

static int batch_create(int d, int n_members, const int64_t* M, const double* L, const ahom_config* cfg,
                        ahom_batch** out) {
    if (!out || !M || !cfg || n_members < 1 || (d != 2 && d != 3)) return bfail(AHOM_E_ARG, "bad batch arguments");
    *out = nullptr;
    if (cfg->precision != AHOM_FP64 && cfg->precision != AHOM_FP32_MIXED) return bfail(AHOM_E_ARG, "bad precision");
    if (cfg->max_iter < 0 || !(cfg->tol >= 0.0)) return bfail(AHOM_E_ARG, "bad tol/max_iter");
    if (cfg->nyquist != AHOM_NYQUIST_HERMITIAN) return bfail(AHOM_E_ARG, "unsupported Nyquist rule");
    if (!(cfg->refine < 1.0)) return bfail(AHOM_E_ARG, "refine must be < 1");
    if (cfg->stop_rule != AHOM_STOP_RESIDUAL) return bfail(AHOM_E_ARG, "batches stop on the residual only");
    if (cfg->scheme != AHOM_SCHEME_BASIC) return bfail(AHOM_E_ARG, "batches run the Basic Scheme only");
    if (cfg->physics != AHOM_ELASTICITY) return bfail(AHOM_E_ARG, "batches solve elasticity only");
    ahom_batch* b = new (std::nothrow) ahom_batch();
    if (!b) return bfail(AHOM_E_NOMEM, "host allocation failed");
    b->d = d;
    b->ncomp = d == 3 ? 6 : 3;
    b->nt = d == 3 ? 3 : 2;
    b->prec = cfg->precision;
    b->cfg = *cfg;
    if (b->cfg.refine == 0.0) b->cfg.refine = 1e-3;
    if (b->cfg.resid_period < 1) b->cfg.resid_period = 1;
    b->stream = (hipStream_t)cfg->stream;
    b->mem.resize(n_members);
    for (int i = 0; i < n_members; ++i) {
        std::string err;
        Member& mb = b->mem[i];
        int rc = ahom_smith_form(d, M + (size_t)i * d * d, &mb.sf, &err);
        if (rc) { delete b; return bfail(rc, "member " + std::to_string(i) + ": " + err); }
        if (mb.sf.m < 2) { delete b; return bfail(AHOM_E_ARG, "member " + std::to_string(i) + ": trivial pattern"); }
        rc = ahom_build_plan_ex(mb.sf, 256, 8, &mb.plan, &err);   // validates the size; replaced by the tuned plan
        if (rc) { delete b; return bfail(rc, "member " + std::to_string(i) + ": " + err); }
        if (L) {
            mb.has_cell = true;
            for (int k = 0; k < d * d; ++k) mb.cell[k] = L[(size_t)i * d * d + k];
            rc = ahom_plan_set_cell(&mb.plan, d, mb.cell, &err);   // validates L
            if (rc) { delete b; return bfail(rc, "member " + std::to_string(i) + ": " + err); }
        }
    }
    if (hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess) {
        delete b;
        return bfail(AHOM_E_DEVICE, "stream/event create");
    }
    *out = b;
    return AHOM_OK;
}

int ahom_batch_create(int d, int n_members, const int64_t* M, const ahom_config* cfg, ahom_batch** out) {
    return batch_create(d, n_members, M, nullptr, cfg, out);
}

int ahom_batch_create_transformed(int d, int n_members, const int64_t* M, const double* L, const ahom_config* cfg,
                                  ahom_batch** out) {
    if (!L) return bfail(AHOM_E_ARG, "null cell matrices");
    return batch_create(d, n_members, M, L, cfg, out);
}

void ahom_batch_destroy(ahom_batch* b) { delete b; }

int ahom_batch_member_info(const ahom_batch* b, int member, int64_t* m, int64_t* e) {
    if (!b || member < 0 || member >= (int)b->mem.size()) return bfail(AHOM_E_ARG, "bad member");
    const SmithForm& sf = b->mem[member].sf;
    if (m) *m = sf.m;
    if (e)
        for (int s = 0; s < b->d; ++s) e[s] = sf.e[s];
    return AHOM_OK;
}

int ahom_batch_member_points(const ahom_batch* b, int member, int64_t* num) {
    if (!b || !num || member < 0 || member >= (int)b->mem.size()) return bfail(AHOM_E_ARG, "bad member");
    ahom_canonical_points(b->mem[member].sf, num);
    return AHOM_OK;
}

int ahom_batch_set_material(ahom_batch* b, int member, int n_phase, const double* lame, const uint8_t* phase) {
    if (!b || !lame || !phase || member < 0 || member >= (int)b->mem.size() || n_phase < 1 || n_phase > 256)
        return bfail(AHOM_E_ARG, "bad batch material arguments");
    Member& mb = b->mem[member];
    double llo = 1e300, lhi = -1e300, mlo = 1e300, mhi = -1e300;
    for (int k = 0; k < n_phase; ++k) {
        const double l = lame[2 * k], mu = lame[2 * k + 1];
        if (!(mu > 0.0) || !(3.0 * l + 2.0 * mu > 0.0))
            return bfail(AHOM_E_MATERIAL, "member " + std::to_string(member) + " phase " + std::to_string(k) + ": need mu > 0 and 3 lambda + 2 mu > 0");
        llo = std::min(llo, l); lhi = std::max(lhi, l); mlo = std::min(mlo, mu); mhi = std::max(mhi, mu);
    }
    const int64_t m = mb.sf.m;
    for (int64_t i = 0; i < m; ++i)
        if (phase[i] >= n_phase) return bfail(AHOM_E_ARG, "member " + std::to_string(member) + ": phase id out of range");
    dfree(mb.d_phase);
    dfree(mb.d_lame);
    BCHK(hipMalloc((void**)&mb.d_phase, m));
    BCHK(hipMemcpy(mb.d_phase, phase, m, hipMemcpyHostToDevice));
    BCHK(hipMalloc((void**)&mb.d_lame, 2 * n_phase * sizeof(double)));
    BCHK(hipMemcpy(mb.d_lame, lame, 2 * n_phase * sizeof(double), hipMemcpyHostToDevice));
    mb.lam_lo = llo; mb.lam_hi = lhi; mb.mu_lo = mlo; mb.mu_hi = mhi;
    if (!mb.ref_set) { mb.lam0 = 0.5 * (llo + lhi); mb.mu0 = 0.5 * (mlo + mhi); }
    mb.has_material = true;
    b->free_items();
    return AHOM_OK;
}

int ahom_batch_set_reference(ahom_batch* b, int member, double lambda0, double mu0) {
    if (!b || member < 0 || member >= (int)b->mem.size()) return bfail(AHOM_E_ARG, "bad member");
    if (!(mu0 > 0.0) || !(lambda0 + 2.0 * mu0 > 0.0)) return bfail(AHOM_E_MATERIAL, "reference needs mu0 > 0 and lambda0 + 2 mu0 > 0");
    Member& mb = b->mem[member];
    mb.lam0 = lambda0;
    mb.mu0 = mu0;
    mb.ref_set = true;
    b->free_items();
    return AHOM_OK;
}

int ahom_batch_solve(ahom_batch* b, int n_load, const double* eps_bar, int* iters, double* resid, double* mean_stress,
                     int* status, int use_graph) {
    roctxRangePushA("ahom_batch_solve");
    struct PopRange { ~PopRange() { roctxRangePop(); } } pop_range;
    if (!b || !eps_bar || n_load < 1) return bfail(AHOM_E_ARG, "bad batch solve arguments");
    for (size_t i = 0; i < b->mem.size(); ++i)
        if (!b->mem[i].has_material) return bfail(AHOM_E_MATERIAL, "member " + std::to_string(i) + ": no material set");
    int rc;
    if (n_load != b->nload || !b->d_items) {
        if ((rc = b->autotune())) return rc;
        if ((rc = b->build_items(n_load))) return rc;
    }
    const int nc = b->ncomp;
    static const int comp3[6] = {0, 4, 8, 5, 2, 1}, comp2[3] = {0, 4, 1};
    const int* comp = b->d == 3 ? comp3 : comp2;
    std::vector<double> eb((size_t)n_load * nc);
    for (int l = 0; l < n_load; ++l)
        for (int c = 0; c < nc; ++c) eb[(size_t)l * nc + c] = eps_bar[(size_t)l * 9 + comp[c]];
    BCHK(hipMemcpy(b->d_epsbar, eb.data(), eb.size() * sizeof(double), hipMemcpyHostToDevice));
    if ((rc = b->run(use_graph != 0))) return rc;
    int ret = AHOM_OK;
    const int nm = (int)b->mem.size();
    for (int q = 0; q < nm * n_load; ++q) {
        const LoadState& ls = b->h_st[q];
        if (iters) iters[q] = ls.iter;
        if (resid) resid[q] = ls.resid;
        if (status) status[q] = ls.status == 0 && ls.resid > b->cfg.tol ? 1 : ls.status;
        if (mean_stress) {
            double* ms9 = mean_stress + (size_t)q * 9;
            for (int k = 0; k < 9; ++k) ms9[k] = 0.0;
            for (int c = 0; c < nc; ++c) {
                const int pos = comp[c];
                ms9[pos] = ls.mean[c];
                ms9[(pos % 3) * 3 + pos / 3] = ls.mean[c];
            }
        }
        if (ls.status == 3) ret = AHOM_E_DEVICE;
        else if (ls.status == 2 && ret != AHOM_E_DEVICE) ret = AHOM_E_DIVERGED;
        else if ((ls.status == 1 || ls.resid > b->cfg.tol) && ret == AHOM_OK) ret = AHOM_W_NOT_CONVERGED;
    }
    if (ret == AHOM_E_DEVICE) ahom_set_error("a workgroup group of some batch item timed out at a pass barrier (status 3)");
    if (ret == AHOM_E_DIVERGED) ahom_set_error("residual diverged (some batch item)");
    return ret;
}

int ahom_batch_strain(ahom_batch* b, int member, int load, double* out) {
    if (!b || !out || member < 0 || member >= (int)b->mem.size() || load < 0 || load >= b->nload)
        return bfail(AHOM_E_ARG, "bad batch strain arguments (solve first)");
    const int q = member * b->nload + load;
    const Member& mb = b->mem[member];
    const int64_t m = mb.plan.m;
    double* d_out = nullptr;
    BCHK(hipMalloc((void**)&d_out, (size_t)b->ncomp * m * sizeof(double)));
    const BatchItem& it = b->h_items[q];
    int rc = AHOM_OK;
    const size_t lds = b->lds;
    RealArgs ra = it.ra;
    ra.real_io = d_out;
    ra.st = it.st;
    if (b->h_restarts[q] > 0) {
        RealArgs rb = it.ra64;
        rb.real_io = d_out;
        rb.st = b->d_st_base;
        if (ahom_launch_real(AHOM_FP64, b->d, REAL_TO_REAL, rb, (int)it.t_real64, 1, b->lds64, b->stream)) rc = AHOM_E_DEVICE;
        ra.accumulate = 1;
    }
    if (!rc && ahom_launch_real(b->prec, b->d, REAL_TO_REAL, ra, (int)it.t_real, 1, lds, b->stream)) rc = AHOM_E_DEVICE;
    if (!rc && hipMemcpy(out, d_out, (size_t)b->ncomp * m * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) rc = AHOM_E_DEVICE;
    (void)hipFree(d_out);
    if (rc) return bfail(rc, "batch strain read-back failed");
    return AHOM_OK;
}

int ahom_batch_history(const ahom_batch* b, int member, int load, double* hist, int cap, int* count) {
    if (!b || !hist || !count || member < 0 || member >= (int)b->mem.size() || load < 0 || load >= b->nload)
        return bfail(AHOM_E_ARG, "bad batch history arguments");
    const int q = member * b->nload + load;
    const int n = std::min(cap, std::min(b->hist_cap, b->h_st[q].iter + 1));
    BCHK(hipMemcpy(hist, b->h_items[q].hist, n * sizeof(double), hipMemcpyDeviceToHost));
    *count = n;
    return AHOM_OK;
}

int ahom_batch_cauchy_history(const ahom_batch* b, int member, int load, double* hist, int cap, int* count) {
    if (!b || !hist || !count || member < 0 || member >= (int)b->mem.size() || load < 0 || load >= b->nload)
        return bfail(AHOM_E_ARG, "bad batch history arguments");
    const int q = member * b->nload + load;
    const int n = std::min(cap, std::min(b->hist_cap, b->h_st[q].iter + 1));
    BCHK(hipMemcpy(hist, b->h_items[q].chist, n * sizeof(double), hipMemcpyDeviceToHost));
    *count = n;
    return AHOM_OK;
}

int ahom_batch_last_timing(const ahom_batch* b, double* ms, int* restarts) {
    if (!b) return bfail(AHOM_E_ARG, "null batch");
    if (ms) *ms = b->last_ms;
    if (restarts) *restarts = std::accumulate(b->h_restarts.begin(), b->h_restarts.end(), 0);
    return AHOM_OK;
}

int ahom_batch_member_variant(const ahom_batch* b, int member, int* variant) {
    if (!b || !variant || member < 0 || member >= (int)b->mem.size()) return bfail(AHOM_E_ARG, "bad member");
    *variant = b->mem[member].variant;
    return AHOM_OK;
}

}  // extern "C"
