// Host side of the gfx950 ground-state library.
//
// Every solve occupies one slot: a block of device memory holding its fields,
// scratch and partial sums, plus a SolveState. Slots
// of the same grid shape, precision and chunk length form a class; each
// kernel of the iteration is launched once for all running slots of a class
// (blockIdx.y = slot), on the class's own stream. A host-side scheduler admits
// requests by device-memory footprint, enqueues chunks of iterations between
// completion checks, hands mixed-precision solves from the float class to the
// double class, runs the final evaluation of finished solves and retires them.
// A slot's arithmetic does not depend on which other slots share its launches,
// so a solve gives the same bits alone and in a batch.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "gs_internal.h"
#include "control.h"
#include "../../include/gs.h"

namespace gs {

LaunchEvents& launch_events() {
    static thread_local LaunchEvents e;
    return e;
}

static thread_local std::string g_err;
static int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}
#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return fail(GS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// supported line lengths: 2^a in [16, 1024], 3 * 2^a in [24, 768], and
// 80, 160, 600, 1200, 2400 (factors of 5: 2400 = 2^5 3 5^2 and its halvings
// that are multiples of 8, the largest tile of a transposing pass); lengths
// above 1024 in 2D only
static bool size_supported(int n) {
    if (n == 80 || n == 160 || n == 600 || n == 1200 || n == 2400) return true;
    const int m = (n % 3 == 0) ? n / 3 : n;
    return n >= 16 && n <= 1024 && m >= 1 && (m & (m - 1)) == 0 && (n % 3 != 0 || n >= 24);
}

static int check_grid(const gs_grid* g) {
    if (!g) return fail(GS_EINVAL, "grid is NULL");
    if (g->dim != 2 && g->dim != 3) return fail(GS_EINVAL, "grid.dim must be 2 or 3");
    for (int a = 0; a < g->dim; ++a) {
        if (!size_supported(g->n[a]))
            return fail(GS_EINVAL, "grid.n[a] must be 2^a in [16, 1024], 3 * 2^a in [24, 768], "
                                   "or one of 80, 160, 600, 1200, 2400");
        if (g->dim == 3 && g->n[a] > LONG_LINE) return fail(GS_EINVAL, "lengths above 1024 are for 2D grids");
        if (!(g->L[a] > 0.0) || !std::isfinite(g->L[a])) return fail(GS_EINVAL, "grid.L[a] must be positive");
    }
    return GS_OK;
}

static long long npts(const gs_grid* g) {
    long long m = (long long)g->n[0] * g->n[1];
    if (g->dim == 3) m *= g->n[2];
    return m;
}

static int check_options(const gs_options* o) {
    if (!o) return fail(GS_EINVAL, "options is NULL");
    if (o->stop_kind < GS_STOP_ENERGY || o->stop_kind > GS_STOP_WAVEFN) return fail(GS_EINVAL, "options.stop_kind invalid");
    if (o->precond < GS_PC_COMBINED || o->precond > GS_PC_POTENTIAL) return fail(GS_EINVAL, "options.precond invalid");
    if (o->line_search != GS_LS_ALG2 && o->line_search != GS_LS_EXACT)
        return fail(GS_EINVAL, "options.line_search invalid");
    if (!(o->tol >= 0.0)) return fail(GS_EINVAL, "options.tol must be >= 0");
    if (o->max_iter < 0) return fail(GS_EINVAL, "options.max_iter must be >= 0");
    if (o->precision < GS_FP64 || o->precision > GS_MIXED) return fail(GS_EINVAL, "options.precision invalid");
    if (!(o->sigma > 0.0 && o->sigma < 1.0)) return fail(GS_EINVAL, "options.sigma must be in (0, 1)");
    if (!(o->theta_trial > 0.0)) return fail(GS_EINVAL, "options.theta_trial must be positive");
    if (o->max_backtrack < 0) return fail(GS_EINVAL, "options.max_backtrack must be >= 0");
    if (o->check_every < 1) return fail(GS_EINVAL, "options.check_every must be >= 1");
    if (o->cm_levels < 1 || o->cm_levels > 7) return fail(GS_EINVAL, "options.cm_levels must be in [1, 7]");
    if (o->dir_precision != GS_FP64 && o->dir_precision != GS_FP32)
        return fail(GS_EINVAL, "options.dir_precision must be GS_FP64 or GS_FP32");
    if (o->nyquist_odd != GS_NYQ_KEEP && o->nyquist_odd != GS_NYQ_ZERO)
        return fail(GS_EINVAL, "options.nyquist_odd must be GS_NYQ_KEEP or GS_NYQ_ZERO");
    return GS_OK;
}

// Best constant of the Gagliardo-Nirenberg inequality in 2D used by the
// existence theorem of Sec. 2.1: C_b = inf |grad u|^2 |u|^2 / |u|_4^4, which is
// half the mass of the positive radial solution Q of Q'' + Q'/r - Q + Q^3 = 0
// (Weinstein's characterisation of the sharp constant); |Q|_2^2 = 11.700896.
constexpr double GN_CB_2D = 5.850448;

// Hypotheses of the existence theorem of Sec. 2.1 for a harmonic trap (see
// gs_existence_check in gs.h).
static int existence(const gs_grid* g, const gs_trap* t, const gs_params* p) {
    if (!g || !p || (g->dim != 2 && g->dim != 3)) return fail(GS_EINVAL, "existence check: invalid argument");
    if (t && (t->V || t->q4 != 0.0)) return GS_OK;   // not a harmonic trap: the theorem says nothing
    double ga2[3];
    for (int a = 0; a < 3; ++a) {
        const double ga = t ? t->g[a] : 1.0;
        ga2[a] = ga * ga + 2.0 * (t ? t->q2 : 0.0);   // V = 1/2 sum (g_a^2 + 2 q2) x_a^2
    }
    for (int a = 0; a < g->dim; ++a)
        if (!(ga2[a] > 0.0)) return GS_WEXISTENCE;   // not a confining harmonic trap
    if (!(std::fabs(p->omega) < std::sqrt(std::min(ga2[0], ga2[1])))) return GS_WEXISTENCE;
    const double c0 = p->c0, c1 = p->c1;
    if (g->dim == 2) return (c0 > -GN_CB_2D && c0 + c1 > -GN_CB_2D) ? GS_OK : GS_WEXISTENCE;
    return ((c0 >= 0.0 && c1 >= 0.0) || (c1 <= 0.0 && c0 + c1 >= 0.0)) ? GS_OK : GS_WEXISTENCE;
}

// slots per class (bounded by the launch grid's y extent and the state arrays)
constexpr int CLASS_CAP = 4096;

// rows of per-block partial sums of the reducing passes (the preconditioner's
// last pass runs in the direction type RD)
template <typename RD> static RedGeom red_geom(const gs_grid* g) {
    RedGeom r;
    const long long M = npts(g);
    const int Nlast = g->n[g->dim - 1];
    r.nblk_mid = mid_blocks(Nlast, (int)(M / Nlast));
    r.nblk_pw = pw_blocks(M);
    r.nblk_dir = g->dim == 2 ? invT_pre_blocks<RD>(g->n[0], 1, g->n[1]) : invT_pre_blocks<RD>(g->n[0], g->n[2], g->n[1]);
    return r;
}

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// buffers of the state type (the others are of the direction type; scratch
// fields are sized for the state type, the wider of the two)
static bool state_buf(int b) { return b == B_PHI || b == B_HL || b >= B_T6A; }

// Device memory of one slot: 12 three-component fields (Phi, H_L Phi, r^n,
// r^{n-1}, Pr, P, H_L P^, u, four scratch), two six-component scratch fields,
// the P_V^{1/2} factors and the partial-sum rows.
template <typename RS, typename RD> static size_t slot_buffer_bytes(const gs_grid* g) {
    const long long M = npts(g);
    const RedGeom rg = red_geom<RD>(g);
    const size_t fs = al256((size_t)3 * M * sizeof(cpx<RS>)), fd = al256((size_t)3 * M * sizeof(cpx<RD>));
    size_t b = 0;
    for (int k = 0; k < B_X0; ++k) b += (k == B_T6A || k == B_T6B ? 2 : 1) * (state_buf(k) ? fs : fd);
    return b + al256((size_t)3 * M * sizeof(RD)) + al256((size_t)rg.nblk_pw * NS_MAX * sizeof(double)) +
           al256((size_t)rg.nblk_mid * RED_MID_STRIDE * sizeof(double)) +
           al256((size_t)rg.nblk_dir * RED_DIR_STRIDE * sizeof(double));
}
template <typename RS, typename RD> static size_t slot_bytes(const gs_grid* g) {
    return slot_buffer_bytes<RS, RD>(g) + sizeof(SolveState) + sizeof(Slot);
}

struct SlotMem {
    void* base = nullptr;
    size_t bytes = 0;
    void* buf[NBUF] = {};
    void* pv = nullptr;
    double* red_pw = nullptr;
    double* red_mid = nullptr;
    double* red_dir = nullptr;
    ~SlotMem() {
        if (base) (void)hipFree(base);
    }
};

template <typename RS, typename RD>
static int alloc_slot_mem(const gs_grid* g, hipStream_t s, std::unique_ptr<SlotMem>& out) {
    auto m = std::make_unique<SlotMem>();
    const long long M = npts(g);
    const size_t fs = al256((size_t)3 * M * sizeof(cpx<RS>)), fd = al256((size_t)3 * M * sizeof(cpx<RD>));
    m->bytes = slot_buffer_bytes<RS, RD>(g);
    if (hipMalloc(&m->base, m->bytes) != hipSuccess) {
        m->base = nullptr;
        (void)hipGetLastError();   // do not leave the failure to the next launch check
        return fail(GS_ENOMEM, "device allocation failed (slot)");
    }
    char* p = (char*)m->base;
    for (int b = 0; b < B_X0; ++b) {
        m->buf[b] = p;
        p += (b == B_T6A || b == B_T6B ? 2 : 1) * (state_buf(b) ? fs : fd);
    }
    m->pv = p;
    p += al256((size_t)3 * M * sizeof(RD));
    const RedGeom rg = red_geom<RD>(g);
    m->red_pw = (double*)p;
    p += al256((size_t)rg.nblk_pw * NS_MAX * sizeof(double));
    m->red_mid = (double*)p;
    p += al256((size_t)rg.nblk_mid * RED_MID_STRIDE * sizeof(double));
    m->red_dir = (double*)p;
    HIPCHK(hipMemsetAsync(m->base, 0, m->bytes, s));
    out = std::move(m);
    return GS_OK;
}

// ---------------------------------------------------------------------------
// per-kernel timer
// ---------------------------------------------------------------------------
// Every launch of one kernel kind of the iteration records its own start and
// end (dispatch timestamps, hipExtLaunchKernelGGL) into HIP events on the
// class's stream; elapsed times and the kernel's algorithmic bytes (each
// distinct array read or written once, times the slots that were still
// running at that iteration) are summed. Launches in which every slot had
// already finished (the tail of the last chunk) are left out.
enum KKind : int {
    KK_HL_FWD = 0, KK_HL_MID = 1, KK_HL_INV = 2, KK_PRE_FWD = 3, KK_PRE_MID = 4, KK_PRE_INV = 5,
    KK_EVAL = 6, KK_RESID = 7, KK_DIRRED = 8, KK_LSRED = 9, KK_HL_FWD2 = 10, KK_HL_INV2 = 11,
    KK_CTRL = 12, KK_COUNT = 13
};
struct TimerTotals {
    int kind = -1;
    double ms = 0.0, bytes = 0.0;
    long long launches = 0;
};
struct Timer {
    int kind = -1;
    struct Rec { int k, chain; double bytes_per_slot; };
    std::vector<hipEvent_t> ev;
    std::vector<Rec> rec;
    int iter_in_chunk = 0;
    int chain = 0;
    ~Timer() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

// `bytes`: algorithmic bytes of the launch for all its slots; `ns` slots.
template <typename F>
static hipError_t timed_ns(Timer* tm, int kind, double bytes, int ns, hipStream_t s, F&& f) {
    if (!tm || tm->kind != kind) return f();
    const size_t i = tm->rec.size();
    while (tm->ev.size() < 2 * (i + 1)) {
        hipEvent_t e;
        hipError_t er = hipEventCreate(&e);
        if (er != hipSuccess) return er;
        tm->ev.push_back(e);
    }
    // the launch itself records its start and end into the two events
    LaunchEvents& le = launch_events();
    le.start = tm->ev[2 * i];
    le.stop = tm->ev[2 * i + 1];
    hipError_t e = f();
    const bool consumed = le.start == nullptr;
    le.start = le.stop = nullptr;
    if (e == hipSuccess && !consumed) e = hipErrorInvalidValue;
    tm->rec.push_back({tm->iter_in_chunk, tm->chain, bytes / (ns > 0 ? ns : 1)});
    return e;
}

// After a chunk has completed, with adv[i] the steps slot i accepted in it and
// fin[i] whether it finished: iteration k ran in full for the slots with
// adv > k; for a slot that finished at iteration adv, the refresh (chain 0),
// the residual pass (chain 1) and the preconditioner with its control step
// (chain 2) of that iteration also ran.
static hipError_t timer_collect(Timer& tm, TimerTotals& tot, const std::vector<int>& adv,
                                const std::vector<char>& fin) {
    for (size_t i = 0; i < tm.rec.size(); ++i) {
        const Timer::Rec& r = tm.rec[i];
        int active = 0;
        for (size_t q = 0; q < adv.size(); ++q)
            active += adv[q] > r.k || (fin[q] && adv[q] == r.k && r.chain <= 2);
        if (!active) continue;
        float ms = 0.0f;
        hipError_t e = hipEventElapsedTime(&ms, tm.ev[2 * i], tm.ev[2 * i + 1]);
        if (e != hipSuccess) return e;
        tot.ms += ms;
        tot.bytes += r.bytes_per_slot * active;
        tot.launches++;
    }
    tm.rec.clear();
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// problem description
// ---------------------------------------------------------------------------
static int make_phys(const gs_grid* g, const gs_trap* t, const gs_params* p, Phys* ph, int nyq_zero = 0) {
    std::memset(ph, 0, sizeof(*ph));
    ph->dim = g->dim;
    ph->nyq_zero = nyq_zero;
    ph->n[0] = g->n[0];
    ph->n[1] = g->n[1];
    ph->n[2] = g->dim == 3 ? g->n[2] : 1;
    ph->cell = 1.0;
    for (int a = 0; a < 3; ++a) {
        ph->L[a] = a < g->dim ? g->L[a] : 1.0;
        ph->h[a] = a < g->dim ? 2.0 * g->L[a] / g->n[a] : 1.0;
        if (a < g->dim) ph->cell *= ph->h[a];
    }
    ph->M = npts(g);
    if (p) {
        if (!std::isfinite(p->omega) || !std::isfinite(p->gamma) || !std::isfinite(p->c0) || !std::isfinite(p->c1))
            return fail(GS_EINVAL, "params must be finite");
        ph->omega = p->omega;
        ph->gamma = p->gamma;
        ph->c0 = p->c0;
        ph->c1 = p->c1;
    }
    if (t) {
        for (int a = 0; a < 3; ++a) ph->hg[a] = a < g->dim ? 0.5 * t->g[a] * t->g[a] : 0.0;
        ph->q2 = t->q2;
        ph->q4 = t->q4;
        if (!std::isfinite(t->q2) || !std::isfinite(t->q4)) return fail(GS_EINVAL, "trap must be finite");
        for (int a = 0; a < g->dim; ++a)
            if (!std::isfinite(t->g[a])) return fail(GS_EINVAL, "trap must be finite");
        if (t->V)
            for (long long i = 0; i < ph->M; ++i)
                if (!std::isfinite(t->V[i])) return fail(GS_EINVAL, "trap.V must be finite");
    } else {
        ph->hg[0] = ph->hg[1] = 0.5;
        ph->hg[2] = g->dim == 3 ? 0.5 : 0.0;
    }
    return GS_OK;
}

static void init_state(SolveState* h, const gs_options* o, int phase) {
    std::memset(h, 0, sizeof(*h));
    h->status = GS_OK;
    h->stop_kind = o->stop_kind;
    h->tol = o->tol;
    h->max_iter = o->max_iter;
    h->max_backtrack = o->max_backtrack;
    h->theta_trial = o->theta_trial;
    h->sigma = o->sigma;
    h->switch_resid = o->switch_resid;
    h->phase_max_iter = o->fp32_max_iter;
    h->stall_window = o->stall_window;
    h->precond = o->precond;
    h->exact_ls = o->line_search == GS_LS_EXACT;
    h->wchange = INFINITY;
    h->phase = phase;
    h->best_resid = INFINITY;
    h->inv_norm = 1.0;
    h->c = 1.0;
}

static void fill_result(const SolveState* h, gs_result* r, int iters_fp32, double wall) {
    if (!r) return;
    std::memset(r, 0, sizeof(*r));
    if (h) {
        r->E = h->E;
        r->mu = h->mu;
        for (int c = 0; c < 3; ++c) {
            r->mu_comp[c] = h->mu_comp[c];
            r->norm_comp[c] = h->norm_comp[c];
        }
        r->e_kin = h->e_kin;
        r->e_pot = h->e_pot;
        r->e_rot = h->e_rot;
        r->e_spin = h->e_spin;
        r->e_soc = h->e_soc;
        r->virial = h->virial;
        r->resid_inf = h->resid_inf;
        r->dE_last = h->dE_last;
        r->iters = h->iter;
        r->backtracks = h->backtracks;
        r->resets = h->resets;
        r->status = h->status;
        r->dphi_inf = h->wchange;
    } else {
        r->dphi_inf = INFINITY;
    }
    r->iters_fp32 = iters_fp32;
    r->wall_s = wall;
    r->iters_coarse = 0;
}

// ---------------------------------------------------------------------------
// operator chains over a launch set of slots
// ---------------------------------------------------------------------------
template <typename RS, typename RD>
struct Geo {
    int dim = 2, n[3] = {1, 1, 1};
    long long M = 0;
    RedGeom g{};
    const cpx<RS>* tws[3] = {};   // twiddles of the state-type transforms
    const cpx<RD>* twd[3] = {};   // and of the direction-type ones
    int rot_any = 0;
};
struct Sub {
    const Slot* tab;
    int ns;
};

// ---------------------------------------------------------------------------
// schedules of the FFT passes and their autotuner
// ---------------------------------------------------------------------------
// The passes of one PCG iteration (the preconditioner's and the H_L P^ chain's)
// each have NCAND candidate launch schedules that compute the same bits (see
// gs_internal.h). A Sched names the candidate of every pass; the fixed table
// is all zeros. The autotuner of a class times the valid candidates of every
// pass on the class's own launches during the first chunk of iterations run
// with a given number of running solves (bucketed by powers of two), then
// keeps the fastest for that bucket (see Tuner).
enum PassId : int {
    P_PRE_FWD = 0, P_PRE_FWD2, P_PRE_MID, P_PRE_INV2, P_PRE_INV,   // preconditioner, 2D: FWD, MID, INV
    P_HL_FWD, P_HL_FWD2, P_HL_MID, P_HL_INV2, P_HL_INV,            // H_L P^ (with Phi's spectrum)
    NPASS
};
static const char* const PASS_NAME[NPASS] = {"pre_fwd", "pre_fwd2", "pre_mid", "pre_inv2", "pre_inv",
                                             "hl_fwd", "hl_fwd2", "hl_mid", "hl_inv2", "hl_inv"};
struct Sched {
    int c[NPASS] = {};
};
// launch records of a tuning chunk: pass, candidate and iteration of each
// timed launch, with its start and end events
struct TuneRun {
    bool on = false;
    int bucket = 0, it = 0;
    struct Rec { int pass, cand, it; };
    std::vector<Rec> rec;
    std::vector<hipEvent_t> ev;
    ~TuneRun() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};
template <typename F>
static hipError_t tuned(TuneRun* tr, int pass, int cand, F&& f) {
    if (!tr || !tr->on) return f();
    const size_t i = tr->rec.size();
    while (tr->ev.size() < 2 * (i + 1)) {
        hipEvent_t e;
        hipError_t er = hipEventCreate(&e);
        if (er != hipSuccess) return er;
        tr->ev.push_back(e);
    }
    LaunchEvents& le = launch_events();
    le.start = tr->ev[2 * i];
    le.stop = tr->ev[2 * i + 1];
    hipError_t e = f();
    const bool consumed = le.start == nullptr;
    le.start = le.stop = nullptr;
    if (e == hipSuccess && !consumed) e = hipErrorInvalidValue;
    tr->rec.push_back({pass, cand, tr->it});
    return e;
}

// out = H_L in  (H_L = -1/2 Lap + V - Omega L_z - gamma S), transforms in type R,
// with the prologue `pro` applied to `in` first (see launch_fwdT; the operand
// of the other type RX is aux1 for PRO_DIR). dual (with
// PRO_DIR): aux1 (Phi) is transformed with in, and the middle pass reduces the
// kinetic coefficients of both for the next iterate's alpha_l. sc: schedules
// (nullptr: the fixed table).
template <typename R, typename RX>
static hipError_t chain_HL(int dim, const int n[3], long long M, int rot, const cpx<R>* const tw[3], Sub L, int pro,
                           int dual, int in, int out, int aux0, int aux1, int use_invnP, hipStream_t s, Timer* tm,
                           const Sched* sc = nullptr, TuneRun* tr = nullptr) {
    const int Nx = n[0], Ny = n[1], Nz = n[2];
    const double F = 3.0 * M * sizeof(cpx<R>) * L.ns, Fx = 3.0 * M * sizeof(cpx<RX>) * L.ns;
    const double b_fwd = dual ? 5 * F + Fx : (pro == PRO_DIR ? 4 * F + Fx : 2 * F);
    const double b_mid = (rot ? 2 : 1) * F + (dual ? 2 : 1) * F, b_inv = (rot ? 4 : 3) * F;
    const int midop = dual ? MID_HLX : MID_HL;
    const int outB = rot ? B_T1 : B_NONE;
    static const Sched fixed;
    const Sched& S = sc ? *sc : fixed;
    const int cF = S.c[P_HL_FWD], cF2 = S.c[P_HL_FWD2], cM = S.c[P_HL_MID], cI2 = S.c[P_HL_INV2], cI = S.c[P_HL_INV];
    hipError_t e;
    if (dim == 2) {
        if ((e = timed_ns(tm, KK_HL_FWD, b_fwd, L.ns, s, [&] { return tuned(tr, P_HL_FWD, cF, [&] {
                 return launch_fwdT<R, RX>(Nx, pro, dual, L.tab, L.ns, in, B_T6A, aux0, aux1, 1, Ny, 3, tw[0], cF, s); }); }))) return e;
        if (Ny > LONG_LINE) {
            // split middle pass: y transforms T6A -> T6B, the operator into
            // T0 (and T1), inverse y transforms in place (with the rotation
            // term from the x-transformed input in T6A)
            if ((e = launch_lfft<R>(Ny, 0, L.tab, L.ns, B_T6A, B_T6B, dual ? 6 : 3, Nx, B_NONE, B_NONE, B_NONE, tw[1], s)))
                return e;
            if ((e = timed_ns(tm, KK_HL_MID, b_mid, L.ns, s, [&] {
                     return launch_lspec<R>(midop, L.tab, L.ns, B_T6B, B_T0, outB, Ny, Nx, rot, s); }))) return e;
            if ((e = launch_lfft<R>(Ny, 1, L.tab, L.ns, B_T0, B_T0, 3, Nx, rot ? B_T6A : B_NONE, rot ? B_T1 : B_NONE,
                                    rot ? B_T1 : B_NONE, tw[1], s))) return e;
        } else if ((e = timed_ns(tm, KK_HL_MID, b_mid, L.ns, s, [&] { return tuned(tr, P_HL_MID, cM, [&] {
                 return launch_mid<R>(Ny, midop, L.tab, L.ns, B_T6A, B_T0, outB, Nx, rot, tw[1], cM, s); }); }))) return e;
        return timed_ns(tm, KK_HL_INV, b_inv, L.ns, s, [&] { return tuned(tr, P_HL_INV, cI, [&] {
            return launch_invT<R>(Nx, EPI_HL, L.tab, L.ns, B_T0, B_T1, out, B_NONE, in, 1, Ny, 1.0, use_invnP, rot, tw[0], cI, s); }); });
    }
    const int nc = dual ? 6 : 3;
    if ((e = timed_ns(tm, KK_HL_FWD, b_fwd, L.ns, s, [&] { return tuned(tr, P_HL_FWD, cF, [&] {
             return launch_fwdT<R, RX>(Nx, pro, dual, L.tab, L.ns, in, B_T6A, aux0, aux1, Nz, Ny, 3, tw[0], cF, s); }); }))) return e;
    if ((e = timed_ns(tm, KK_HL_FWD2, 2 * (nc / 3) * F, L.ns, s, [&] { return tuned(tr, P_HL_FWD2, cF2, [&] {
             return launch_fwdT<R, RX>(Ny, PRO_PLAIN, 0, L.tab, L.ns, B_T6A, B_T6B, B_NONE, B_NONE, Nx, Nz, nc, tw[1], cF2, s); }); }))) return e;
    if ((e = timed_ns(tm, KK_HL_MID, b_mid, L.ns, s, [&] { return tuned(tr, P_HL_MID, cM, [&] {
             return launch_mid<R>(Nz, midop, L.tab, L.ns, B_T6B, B_T0, outB, Ny * Nx, rot, tw[2], cM, s); }); }))) return e;
    if ((e = timed_ns(tm, KK_HL_INV2, (rot ? 5 : 2) * F, L.ns, s, [&] { return tuned(tr, P_HL_INV2, cI2, [&] {
             return launch_invT<R>(Ny, rot ? EPI_ROTX : EPI_SCALE, L.tab, L.ns, B_T0, B_T1, B_T2, rot ? B_T3 : B_NONE,
                                   B_T6A, Nx, Nz, 1.0, 0, rot, tw[1], cI2, s); }); }))) return e;
    return timed_ns(tm, KK_HL_INV, b_inv, L.ns, s, [&] { return tuned(tr, P_HL_INV, cI, [&] {
        return launch_invT<R>(Nx, EPI_HL, L.tab, L.ns, B_T2, B_T3, out, B_NONE, in, Nz, Ny, 1.0, use_invnP, rot, tw[0], cI, s); }); });
}

// out = P_V^{1/2} P_Delta P_V^{1/2} r in the direction type RD (the first factor
// is already applied: input in u); dir = 1 fuses the partial sums of the
// direction scalars into the last pass
template <typename RS, typename RD>
static hipError_t chain_pre(const Geo<RS, RD>& G, Sub L, int dir, int out, hipStream_t s, Timer* tm,
                            const Sched* sc = nullptr, TuneRun* tr = nullptr) {
    const int Nx = G.n[0], Ny = G.n[1], Nz = G.n[2];
    const double F = 3.0 * G.M * sizeof(cpx<RD>) * L.ns, Fr = 3.0 * G.M * sizeof(RD) * L.ns;
    const double Fs = 3.0 * G.M * sizeof(cpx<RS>) * L.ns;
    const double b_inv = (dir ? 5 * F + Fs : 2 * F) + Fr;
    static const Sched fixed;
    const Sched& S = sc ? *sc : fixed;
    const int cF = S.c[P_PRE_FWD], cF2 = S.c[P_PRE_FWD2], cM = S.c[P_PRE_MID], cI2 = S.c[P_PRE_INV2], cI = S.c[P_PRE_INV];
    hipError_t e;
    if (G.dim == 2) {
        if ((e = timed_ns(tm, KK_PRE_FWD, 2 * F, L.ns, s, [&] { return tuned(tr, P_PRE_FWD, cF, [&] {
                 return launch_fwdT<RD, RD>(Nx, PRO_PLAIN, 0, L.tab, L.ns, B_U, B_T6A, B_NONE, B_NONE, 1, Ny, 3, G.twd[0], cF, s); }); }))) return e;
        if (Ny > LONG_LINE) {
            if ((e = launch_lfft<RD>(Ny, 0, L.tab, L.ns, B_T6A, B_T6B, 3, Nx, B_NONE, B_NONE, B_NONE, G.twd[1], s)))
                return e;
            if ((e = timed_ns(tm, KK_PRE_MID, 2 * F, L.ns, s, [&] {
                     return launch_lspec<RD>(MID_PRE, L.tab, L.ns, B_T6B, B_T0, B_NONE, Ny, Nx, 0, s); }))) return e;
            if ((e = launch_lfft<RD>(Ny, 1, L.tab, L.ns, B_T0, B_T0, 3, Nx, B_NONE, B_NONE, B_NONE, G.twd[1], s)))
                return e;
        } else if ((e = timed_ns(tm, KK_PRE_MID, 2 * F, L.ns, s, [&] { return tuned(tr, P_PRE_MID, cM, [&] {
                 return launch_mid<RD>(Ny, MID_PRE, L.tab, L.ns, B_T6A, B_T0, B_NONE, Nx, 0, G.twd[1], cM, s); }); }))) return e;
        return timed_ns(tm, KK_PRE_INV, b_inv, L.ns, s, [&] { return tuned(tr, P_PRE_INV, cI, [&] {
            return launch_invT_pre<RD, RS>(Nx, L.tab, L.ns, B_T0, out, 1, Ny, dir, G.twd[0], cI, s); }); });
    }
    if ((e = timed_ns(tm, KK_PRE_FWD, 2 * F, L.ns, s, [&] { return tuned(tr, P_PRE_FWD, cF, [&] {
             return launch_fwdT<RD, RD>(Nx, PRO_PLAIN, 0, L.tab, L.ns, B_U, B_T6A, B_NONE, B_NONE, Nz, Ny, 3, G.twd[0], cF, s); }); }))) return e;
    if ((e = tuned(tr, P_PRE_FWD2, cF2, [&] {
             return launch_fwdT<RD, RD>(Ny, PRO_PLAIN, 0, L.tab, L.ns, B_T6A, B_T6B, B_NONE, B_NONE, Nx, Nz, 3, G.twd[1], cF2, s); }))) return e;
    if ((e = timed_ns(tm, KK_PRE_MID, 2 * F, L.ns, s, [&] { return tuned(tr, P_PRE_MID, cM, [&] {
             return launch_mid<RD>(Nz, MID_PRE, L.tab, L.ns, B_T6B, B_T0, B_NONE, Ny * Nx, 0, G.twd[2], cM, s); }); }))) return e;
    if ((e = tuned(tr, P_PRE_INV2, cI2, [&] {
             return launch_invT<RD>(Ny, EPI_SCALE, L.tab, L.ns, B_T0, B_NONE, B_T1, B_NONE, B_NONE, Nx, Nz, 1.0, 0, 0, G.twd[1], cI2, s); }))) return e;
    return timed_ns(tm, KK_PRE_INV, b_inv, L.ns, s, [&] { return tuned(tr, P_PRE_INV, cI, [&] {
        return launch_invT_pre<RD, RS>(Nx, L.tab, L.ns, B_T1, out, Nz, Ny, dir, G.twd[0], cI, s); }); });
}

// Candidates of pass p that are valid for grid n (RD: direction type, in which
// the passes of the iteration run).
template <typename RD> static std::vector<int> valid_cands(int dim, const int n[3], int p) {
    std::vector<int> v;
    const int Nx = n[0], Ny = n[1], Nz = n[2], Nl = dim == 2 ? Ny : Nz;
    for (int c = 0; c < NCAND; ++c) {
        bool ok = false;
        switch (p) {
        case P_PRE_FWD: case P_HL_FWD: ok = fwdT_cand_ok<RD>(Nx, c, Ny); break;
        case P_PRE_FWD2: case P_HL_FWD2: ok = dim == 3 && fwdT_cand_ok<RD>(Ny, c, Nz); break;
        case P_PRE_MID: case P_HL_MID: ok = mid_cand_ok(Nl, c); break;
        case P_PRE_INV2: case P_HL_INV2: ok = dim == 3 && invT_cand_ok<RD>(Ny, c, Nz); break;
        case P_PRE_INV: ok = invT_pre_cand_ok<RD>(Nx, c); break;
        case P_HL_INV: ok = invT_cand_ok<RD>(Nx, c, Ny); break;
        }
        if (ok) v.push_back(c);
    }
    return v;
}
// lines per block and threads per block of candidate c of pass p
template <typename RD> static Cand cand_of(int dim, const int n[3], int p, int c) {
    const int Nx = n[0], Ny = n[1], Nz = n[2], Nl = dim == 2 ? Ny : Nz;
    switch (p) {
    case P_PRE_FWD: case P_HL_FWD: return fwdT_cand_of<RD>(Nx, c);
    case P_PRE_FWD2: case P_HL_FWD2: return fwdT_cand_of<RD>(Ny, c);
    case P_PRE_MID: case P_HL_MID: return mid_cand_of(Nl, c);
    case P_PRE_INV2: case P_HL_INV2: return invT_cand_of<RD>(Ny, c);
    case P_PRE_INV: return invT_pre_cand_of<RD>(Nx, c);
    default: return invT_cand_of<RD>(Nx, c);
    }
}

// Per class: the chosen candidates per bucket of running solves, and the
// timings behind them.
constexpr int NBUCKET = 8;   // running solves 1, 2-3, 4-7, ..., >= 128
static int bucket_of(int nrun) {
    int b = 0;
    while (b + 1 < NBUCKET && (2 << b) <= nrun) ++b;
    return b;
}
struct Tuner {
    bool decided[NBUCKET] = {};
    int chunks[NBUCKET] = {};          // tuning chunks spent on the bucket
    Sched best[NBUCKET];
    double ms[NBUCKET][NPASS][NCAND] = {};   // summed launch times (first launch of each left out)
    int n[NBUCKET][NPASS][NCAND] = {};       // launches counted
    int seen[NBUCKET][NPASS][NCAND] = {};    // launches timed
    TuneRun run;
};

// bytes of partial-sum rows a control step reads
static double fin_bytes(const RedGeom& g, int what, int ns) {
    double rows = 0.0;
    switch (what) {
    case FIN_EVAL: rows = (double)g.nblk_pw * NS_EVAL + (double)g.nblk_mid * 4; break;
    case FIN_DIR: rows = (double)g.nblk_pw * NS_RES + (double)g.nblk_dir * NS_DIR; break;
    case FIN_LS: rows = (double)g.nblk_pw * NS_LS + (double)g.nblk_mid * NS_KIN; break;
    default: rows = (double)g.nblk_pw * NS_RES; break;
    }
    return rows * sizeof(double) * ns;
}
static hipError_t fin(const RedGeom& g, Sub L, int what, hipStream_t s, Timer* tm) {
    return timed_ns(tm, KK_CTRL, fin_bytes(g, what, L.ns), L.ns, s, [&] { return launch_fin(L.tab, L.ns, g, what, s); });
}

// Fresh evaluation of the current iterate, in the state type: apply a pending
// update to Phi (with the largest change, criterion (3.9)), H_L Phi from
// scratch, energy parts, mu, alpha_l.
template <typename RS, typename RD>
static hipError_t refresh(const Geo<RS, RD>& G, Sub L, hipStream_t s, Timer* tm) {
    const double Fs = 3.0 * G.M * sizeof(cpx<RS>) * L.ns;
    hipError_t e;
    if ((e = launch_apply<RS, RD>(L.tab, L.ns, G.g, s))) return e;
    if ((e = chain_HL<RS, RD>(G.dim, G.n, G.M, G.rot_any, G.tws, L, PRO_PLAIN, 0, B_PHI, B_HL, B_NONE, B_NONE, 0, s, tm))) return e;
    if ((e = timed_ns(tm, KK_EVAL, 2 * Fs, L.ns, s, [&] { return launch_eval<RS>(L.tab, L.ns, G.g, s); }))) return e;
    return fin(G.g, L, FIN_EVAL, s, tm);
}

// normalisation of Phi (applied as a pending rescale by the next pass)
template <typename RS, typename RD>
static hipError_t normalize(const Geo<RS, RD>& G, Sub L, hipStream_t s) {
    hipError_t e;
    if ((e = launch_normalize<RS>(L.tab, L.ns, G.g, s))) return e;
    return fin(G.g, L, FIN_NORM, s, nullptr);
}

// residual norm of the current iterate (after a refresh)
template <typename RS, typename RD>
static hipError_t resid_final(const Geo<RS, RD>& G, Sub L, hipStream_t s) {
    hipError_t e;
    if ((e = launch_resid<RS, RD>(L.tab, L.ns, G.g, 1, s))) return e;
    return fin(G.g, L, FIN_RFINAL, s, nullptr);
}

// One PCG iteration (Algorithm 1 with Algorithm 2), entirely on the device:
//   0. (first iteration of a chunk) fresh H_L Phi, E, mu, alpha_l
//   1. pending update Phi <- (c Phi + s P^)/|.|, H_L Phi by the same combination;
//      r = H(Phi)Phi - mu Phi, P_V^{1/2} factors
//   2. preconditioned residual (3 or 5 FFT passes) with the sums of the
//      direction scalars fused into its last pass; control: stopping tests,
//      PRP beta, projection and descent test
//   3. P^n = D - Re<D,Phi> Phi, H_L P^ (3 or 5 FFT passes; Phi transformed
//      alongside for the kinetic coefficients)
//   4. energy along the retraction; control: step size, backtracking, and the
//      scalars (mu, E, alpha_l) of the next iterate
// Steps 2 and 3 run in the direction type RD, the rest in the state type RS;
// every reduction and scalar is double.
template <typename RS, typename RD>
static hipError_t iterate(const Geo<RS, RD>& G, Sub L, int do_refresh, hipStream_t s, Timer* tm,
                          const Sched* sc = nullptr, TuneRun* tr = nullptr) {
    const double Fs = 3.0 * G.M * sizeof(cpx<RS>) * L.ns, Fd = 3.0 * G.M * sizeof(cpx<RD>) * L.ns;
    const double Frd = 3.0 * G.M * sizeof(RD) * L.ns;
    hipError_t e;
    if (do_refresh) {
        if (tm) tm->chain = 0;
        if ((e = refresh<RS, RD>(G, L, s, tm))) return e;
    }
    if (tm) tm->chain = 1;
    if ((e = timed_ns(tm, KK_RESID, 4 * Fs + 4 * Fd + Frd, L.ns, s, [&] { return launch_resid<RS, RD>(L.tab, L.ns, G.g, 0, s); }))) return e;
    if (tm) tm->chain = 2;
    if ((e = chain_pre<RS, RD>(G, L, 1, B_PR, s, tm, sc, tr))) return e;
    if ((e = fin(G.g, L, FIN_DIR, s, tm))) return e;
    if (tm) tm->chain = 3;
    if ((e = chain_HL<RD, RS>(G.dim, G.n, G.M, G.rot_any, G.twd, L, PRO_DIR, 1, B_P, B_HLP, B_PR, B_PHI, 1, s, tm, sc,
                              tr))) return e;
    if ((e = timed_ns(tm, KK_LSRED, 2 * Fs + 2 * Fd, L.ns, s, [&] { return launch_lsred<RS, RD>(L.tab, L.ns, G.g, s); }))) return e;
    return fin(G.g, L, FIN_LS, s, tm);
}

// ---------------------------------------------------------------------------
// requests, classes, context
// ---------------------------------------------------------------------------
enum JobStage : int { JS_QUEUED = 0, JS_RUNNING, JS_FINAL, JS_DONE };

struct Job {
    uint64_t ticket = 0;
    gs_grid grid{};
    gs_options opt{};
    Phys ph{};
    double* Vdev = nullptr;
    const cpx<double>* psi0 = nullptr;
    cpx<double>* out = nullptr;
    size_t reserve = 0;
    int stage = JS_QUEUED;
    bool admitted = false;   // reservation held
    bool cancel = false;
    int slot = -1;           // slot in the current class (preset for a hand-over)
    bool handover = false;   // queued in the double class after the float phase
    SolveState mig{};        // state handed over from the float phase
    hipEvent_t ev = nullptr; // the guess or hand-over is complete (recorded on another stream)
    bool wait_ev = false;
    int iters_fp32 = 0;
    // cascadic multigrid: levels coarse to fine; the current level's grid is `grid`
    int level = 0, nlevels = 1;
    gs_grid fine{};
    gs_trap trap{};
    gs_params prm{};
    cpx<double>* cm_buf[2] = {nullptr, nullptr};   // level result / interpolated guess (finest size)
    cpx<double>* user_out = nullptr;
    int iters_coarse = 0;
    bool warn_existence = false;   // the parameters fail the hypotheses of the existence theorem
    int rc = GS_OK;
    gs_result res{};
    std::string err;
    std::chrono::steady_clock::time_point t0;
    ~Job() {
        if (Vdev) (void)hipFree(Vdev);
        for (auto* b : cm_buf)
            if (b) (void)hipFree(b);
        if (ev) (void)hipEventDestroy(ev);
    }
};

template <typename RS, typename RD>
struct Class {
    gs_grid grid{};
    int check_every = 0;
    long long M = 0;
    RedGeom g{};
    const cpx<RS>* tws[3] = {};
    const cpx<RD>* twd[3] = {};
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    SolveState* d_st = nullptr;
    SolveState* h_st = nullptr;     // pinned mirror
    Slot* d_tab = nullptr;
    Slot* h_tab = nullptr;          // pinned
    std::vector<std::unique_ptr<SlotMem>> mem;   // by slot id
    std::vector<Job*> owner;                      // by slot id
    std::vector<int> run, fin, iter0;
    std::deque<Job*> queue;
    bool inflight = false;
    uint64_t seq = 0;
    Timer tm;
    Tuner tun;
    std::vector<int> valid[NPASS];   // valid schedule candidates of each pass (the autotuner's set)
    ~Class() {
        if (stream) (void)hipStreamSynchronize(stream);
        mem.clear();
        if (d_st) (void)hipFree(d_st);
        if (d_tab) (void)hipFree(d_tab);
        if (h_st) (void)hipHostFree(h_st);
        if (h_tab) (void)hipHostFree(h_tab);
        if (ev) (void)hipEventDestroy(ev);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

// single-slot plan of the operator-level entry points (one precision)
template <typename R>
struct OpPlan {
    gs_grid grid{};
    long long M = 0;
    RedGeom g{};
    const cpx<R>* tw[3] = {};
    std::unique_ptr<SlotMem> mem;
    SolveState* d_st = nullptr;
    SolveState* h_st = nullptr;
    Slot* d_tab = nullptr;
    Slot* h_tab = nullptr;
    ~OpPlan() {
        mem.reset();
        if (d_st) (void)hipFree(d_st);
        if (d_tab) (void)hipFree(d_tab);
        if (h_st) (void)hipHostFree(h_st);
        if (h_tab) (void)hipHostFree(h_tab);
    }
};

using ClassKey = std::tuple<int, int, int, int, int>;   // dim, n0, n1, n2, check_every
using GridKey = std::tuple<int, int, int, int>;

struct Ctx {
    int device = 0;
    std::map<ClassKey, std::unique_ptr<Class<double, double>>> c64;
    std::map<ClassKey, std::unique_ptr<Class<float, float>>> c32;
    std::map<ClassKey, std::unique_ptr<Class<double, float>>> cmx;   // double phase of mixed solves
    std::map<GridKey, std::unique_ptr<OpPlan<double>>> o64;
    std::map<GridKey, std::unique_ptr<OpPlan<float>>> o32;
    std::map<std::pair<int, int>, void*> twiddles;   // (N, sizeof(R)) -> table
    std::map<uint64_t, std::unique_ptr<Job>> jobs;
    uint64_t next_ticket = 1, next_seq = 1;
    uint64_t moves = 0;   // requests queued into another class (hand-overs, multigrid levels)
    size_t budget = 0, reserved = 0, allocated = 0;
    TimerTotals timer;
    int autotune = 1;   // 1: tune the FFT pass schedules per class and bucket; 0: the fixed table
    std::string report;
    ~Ctx() {
        (void)hipSetDevice(device);
        c64.clear();
        c32.clear();
        cmx.clear();
        o64.clear();
        o32.clear();
        jobs.clear();
        for (auto& kv : twiddles) (void)hipFree(kv.second);
    }
};

template <typename RS, typename RD> struct ClassMap;
template <> struct ClassMap<double, double> { static auto& get(Ctx& cx) { return cx.c64; } };
template <> struct ClassMap<float, float> { static auto& get(Ctx& cx) { return cx.c32; } };
template <> struct ClassMap<double, float> { static auto& get(Ctx& cx) { return cx.cmx; } };
// f(class) over every class (float state first); stops at the first nonzero return
template <typename F> static int each_class(Ctx& cx, F&& f) {
    int rc;
    for (auto& kv : cx.c32)
        if ((rc = f(*kv.second))) return rc;
    for (auto& kv : cx.cmx)
        if ((rc = f(*kv.second))) return rc;
    for (auto& kv : cx.c64)
        if ((rc = f(*kv.second))) return rc;
    return 0;
}
template <typename R> static auto& opplans(Ctx& cx);
template <> auto& opplans<double>(Ctx& cx) { return cx.o64; }
template <> auto& opplans<float>(Ctx& cx) { return cx.o32; }

// Host image of the twiddle table of length N in type R: exp(-2 pi i m / N),
// m < N, each entry rounded once from long double; a float table is followed
// by the same table in double (the float passes form twiddle powers from it).
template <typename R> static std::vector<unsigned char> twiddle_image(int N) {
    const bool dbl_too = sizeof(R) == 4;
    std::vector<unsigned char> img(sizeof(cpx<R>) * N + (dbl_too ? sizeof(cpx<double>) * N : 0));
    cpx<R>* h = reinterpret_cast<cpx<R>*>(img.data());
    cpx<double>* hd = reinterpret_cast<cpx<double>*>(img.data() + sizeof(cpx<R>) * N);
    for (int m = 0; m < N; ++m) {
        const long double ang = 2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)N;
        h[m] = cpx<R>{(R)cosl(ang), (R)(-sinl(ang))};
        if (dbl_too) hd[m] = cpx<double>{(double)cosl(ang), (double)(-sinl(ang))};
    }
    return img;
}

template <typename R>
static int get_twiddle(Ctx& cx, int N, const cpx<R>** out) {
    auto key = std::make_pair(N, (int)sizeof(R));
    auto it = cx.twiddles.find(key);
    if (it != cx.twiddles.end()) {
        *out = (const cpx<R>*)it->second;
        return GS_OK;
    }
    const std::vector<unsigned char> img = twiddle_image<R>(N);
    void* d = nullptr;
    if (hipMalloc(&d, img.size()) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GS_ENOMEM, "twiddle table allocation failed");
    }
    HIPCHK(hipMemcpy(d, img.data(), img.size(), hipMemcpyHostToDevice));
    cx.twiddles[key] = d;
    *out = (const cpx<R>*)d;
    return GS_OK;
}

static GridKey grid_key(const gs_grid* g) {
    return std::make_tuple(g->dim, g->n[0], g->n[1], g->dim == 3 ? g->n[2] : 1);
}

template <typename RS, typename RD>
static int get_class(Ctx& cx, const gs_grid* g, int check_every, Class<RS, RD>** out) {
    auto key = std::make_tuple(g->dim, g->n[0], g->n[1], g->dim == 3 ? g->n[2] : 1, check_every);
    auto& mp = ClassMap<RS, RD>::get(cx);
    auto it = mp.find(key);
    if (it != mp.end()) {
        *out = it->second.get();
        return GS_OK;
    }
    auto c = std::make_unique<Class<RS, RD>>();
    c->grid = *g;
    if (g->dim == 2) c->grid.n[2] = 1;
    c->check_every = check_every;
    c->M = npts(g);
    c->g = red_geom<RD>(g);
    for (int a = 0; a < g->dim; ++a) {
        int rc = get_twiddle<RS>(cx, g->n[a], &c->tws[a]);
        if (!rc) rc = get_twiddle<RD>(cx, g->n[a], &c->twd[a]);
        if (rc) return rc;
    }
    // non-blocking: the class's work never waits for the null stream
    HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&c->ev, hipEventDisableTiming));
    if (hipMalloc((void**)&c->d_st, sizeof(SolveState) * CLASS_CAP) != hipSuccess ||
        hipMalloc((void**)&c->d_tab, sizeof(Slot) * CLASS_CAP) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GS_ENOMEM, "device allocation failed (class tables)");
    }
    if (hipHostMalloc((void**)&c->h_st, sizeof(SolveState) * CLASS_CAP, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->h_tab, sizeof(Slot) * CLASS_CAP, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GS_ENOMEM, "pinned allocation failed (class tables)");
    }
    std::memset(c->h_st, 0, sizeof(SolveState) * CLASS_CAP);
    const int nn[3] = {g->n[0], g->n[1], g->dim == 3 ? g->n[2] : 1};
    for (int p = 0; p < NPASS; ++p) c->valid[p] = valid_cands<RD>(g->dim, nn, p);
    *out = c.get();
    mp[key] = std::move(c);
    return GS_OK;
}

static Slot entry_of(SlotMem& m, SolveState* st, const Phys& ph) {
    Slot e;
    std::memset(&e, 0, sizeof(e));
    for (int b = 0; b < NBUF; ++b) e.buf[b] = m.buf[b];
    e.pv = m.pv;
    e.st = st;
    e.red_mid = m.red_mid;
    e.red_pw = m.red_pw;
    e.red_dir = m.red_dir;
    e.p = ph;
    return e;
}

template <typename RS, typename RD>
static Geo<RS, RD> geo_of(const gs_grid& g, long long M, RedGeom rg, const cpx<RS>* const tws[3],
                          const cpx<RD>* const twd[3], int rot_any) {
    Geo<RS, RD> G;
    G.dim = g.dim;
    G.n[0] = g.n[0];
    G.n[1] = g.n[1];
    G.n[2] = g.dim == 3 ? g.n[2] : 1;
    G.M = M;
    G.g = rg;
    for (int a = 0; a < 3; ++a) {
        G.tws[a] = tws[a];
        G.twd[a] = twd[a];
    }
    G.rot_any = rot_any;
    return G;
}

// Release the device memory of idle slots (any class) until `need` more bytes
// fit in the budget.
template <typename RS, typename RD>
static void trim_class(Class<RS, RD>& c, Ctx& cx, size_t need) {
    for (size_t k = 0; k < c.mem.size() && cx.allocated + need > cx.budget; ++k) {
        if (c.mem[k] && !c.owner[k]) {
            cx.allocated -= c.mem[k]->bytes;
            c.mem[k].reset();
        }
    }
}
static void trim(Ctx& cx, size_t need) {
    (void)hipDeviceSynchronize();   // pending work may still read a released slot
    each_class(cx, [&](auto& c) { trim_class(c, cx, need); return 0; });
}

constexpr int SLOT_WAIT = 1;

// Free slot of the class for job j (allocated if needed; a new slot is zeroed
// on stream s, which must precede every later use of the slot). GS_OK,
// SLOT_WAIT (no memory now) or an error.
template <typename RS, typename RD>
static int acquire_slot(Ctx& cx, Class<RS, RD>& c, Job* j, hipStream_t s, int* out) {
    int id = -1;
    for (size_t k = 0; k < c.mem.size(); ++k)
        if (c.mem[k] && !c.owner[k]) { id = (int)k; break; }
    if (id < 0) {
        for (size_t k = 0; k < c.mem.size(); ++k)
            if (!c.mem[k] && !c.owner[k]) { id = (int)k; break; }
        if (id < 0) {
            if ((int)c.mem.size() >= CLASS_CAP) return SLOT_WAIT;
            id = (int)c.mem.size();
            c.mem.emplace_back();
            c.owner.push_back(nullptr);
        }
        const size_t need = slot_buffer_bytes<RS, RD>(&c.grid);
        if (cx.allocated + need > cx.budget) trim(cx, need);
        if (cx.allocated + need > cx.budget) return SLOT_WAIT;
        int rc = alloc_slot_mem<RS, RD>(&c.grid, s, c.mem[id]);
        if (rc) return rc;
        cx.allocated += need;
    }
    c.owner[id] = j;
    *out = id;
    return GS_OK;
}

static void finish_job(Ctx& cx, Job* j, int rc, const SolveState* h, const std::string& msg) {
    const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - j->t0).count();
    if (rc == GS_OK && j->warn_existence) rc = GS_WEXISTENCE;
    fill_result(h, &j->res, j->iters_fp32, wall);
    j->res.iters_coarse = j->iters_coarse;
    j->res.status = rc;
    j->rc = rc;
    if (rc < 0) j->err = msg;
    j->stage = JS_DONE;
    j->slot = -1;
    if (j->admitted) {
        cx.reserved -= j->reserve;
        j->admitted = false;
    }
}

// Float phase of a mixed solve finished with a switch request: hand Phi (made
// double on the float stream) and the state (beta reset, phase FP64) to the
// double-state class of the same grid (with the search direction in RD).
template <typename RD>
static int hand_over_to(Ctx& cx, Class<float, float>& c, int k, Job* j) {
    Class<double, RD>* d = nullptr;
    int rc = get_class<double, RD>(cx, &j->grid, c.check_every, &d);
    if (rc) return rc;
    int kd = -1;
    rc = acquire_slot<double, RD>(cx, *d, j, c.stream, &kd);
    if (rc == SLOT_WAIT) return fail(GS_ENOMEM, "no device memory for the double phase");
    if (rc) return rc;
    HIPCHK(launch_convert_f2d(static_cast<cpx<float>*>(c.mem[k]->buf[B_PHI]),
                              static_cast<cpx<double>*>(d->mem[kd]->buf[B_PHI]), 3 * c.M, c.stream));
    if (!j->ev) HIPCHK(hipEventCreateWithFlags(&j->ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(j->ev, c.stream));
    j->wait_ev = true;
    SolveState h = c.h_st[k];
    j->iters_fp32 = h.iter;
    h.done = 0;
    h.switch_req = 0;
    h.phase = PH_FP64;
    h.have_prev = 0;
    h.pending_step = 0;
    h.final_pending = 0;
    h.iter_phase = 0;
    h.status = GS_OK;
    h.wchange = INFINITY;
    j->mig = h;
    j->slot = kd;
    j->handover = true;
    j->stage = JS_QUEUED;
    d->queue.push_front(j);
    cx.moves++;
    return GS_OK;
}
static int hand_over(Ctx& cx, Class<float, float>& c, int k, Job* j) {
    return j->opt.dir_precision == GS_FP32 ? hand_over_to<float>(cx, c, k, j) : hand_over_to<double>(cx, c, k, j);
}

// Initial guess of job j into slot k's Phi (the Gaussian guess is built in
// double, then rounded when the state is float).
template <typename RS, typename RD>
static int load_guess(Class<RS, RD>& c, int k, Job* j) {
    SlotMem& m = *c.mem[k];
    const long long n3 = 3 * c.M;
    if constexpr (std::is_same<RS, double>::value) {
        cpx<double>* phi = static_cast<cpx<double>*>(m.buf[B_PHI]);
        if (j->psi0) HIPCHK(hipMemcpyAsync(phi, j->psi0, sizeof(cpx<double>) * n3, hipMemcpyDeviceToDevice, c.stream));
        else HIPCHK(launch_gaussian(phi, j->ph, c.stream));
    } else {
        const cpx<double>* src = j->psi0;
        if (!src) {
            cpx<double>* tmp = static_cast<cpx<double>*>(m.buf[B_T6A]);   // 2 float fields = 1 double field
            HIPCHK(launch_gaussian(tmp, j->ph, c.stream));
            src = tmp;
        }
        HIPCHK(launch_convert_d2f(src, static_cast<cpx<float>*>(m.buf[B_PHI]), n3, c.stream));
    }
    return GS_OK;
}

template <typename RS, typename RD>
static int copy_out(Class<RS, RD>& c, int k, Job* j) {
    const long long n3 = 3 * c.M;
    if constexpr (std::is_same<RS, double>::value)
        HIPCHK(hipMemcpyAsync(j->out, c.mem[k]->buf[B_PHI], sizeof(cpx<double>) * n3, hipMemcpyDeviceToDevice, c.stream));
    else
        HIPCHK(launch_convert_f2d(static_cast<cpx<float>*>(c.mem[k]->buf[B_PHI]), j->out, n3, c.stream));
    return GS_OK;
}

template <typename R> static int fft_impl(Ctx& cx, const gs_grid* g, int sign, const cpx<R>* in, cpx<R>* out,
                                          hipStream_t s);

// Fourier interpolation gc -> gf (same box): forward transform on gc,
// zero-padding of the spectrum, inverse transform on gf. tmp: [3][gc] scratch.
static int interp_impl(Ctx& cx, const gs_grid* gc, const cpx<double>* in, const gs_grid* gf, cpx<double>* out,
                       cpx<double>* tmp, hipStream_t s) {
    int rc;
    if ((rc = fft_impl<double>(cx, gc, -1, in, tmp, s))) return rc;     // coarse spectrum in tmp
    const int nc[3] = {gc->n[0], gc->n[1], gc->dim == 3 ? gc->n[2] : 1};
    const int nf[3] = {gf->n[0], gf->n[1], gf->dim == 3 ? gf->n[2] : 1};
    HIPCHK(launch_spec_pad(tmp, out, gc->dim, nc, nf, s));                // fine spectrum in out
    // in place: the first pass of the transform only reads, the last only writes
    return fft_impl<double>(cx, gf, +1, out, out, s);
}

static gs_grid level_grid(const gs_grid& fine, int nlevels, int level) {
    gs_grid g = fine;
    const int sh = nlevels - 1 - level;
    for (int a = 0; a < fine.dim; ++a) g.n[a] = fine.n[a] >> sh;
    if (fine.dim == 2) g.n[2] = 1;
    return g;
}

// Queue request j in the class that runs its first precision phase on its
// current grid: double state for FP64 solves, float state otherwise; the
// direction precision of an FP64 solve follows its dir_precision option.
static int enqueue(Ctx& cx, Job* j, bool front) {
    int rc;
    if (j->opt.precision == GS_FP64 && j->opt.dir_precision == GS_FP32) {
        Class<double, float>* c;
        if ((rc = get_class<double, float>(cx, &j->grid, j->opt.check_every, &c))) return rc;
        front ? c->queue.push_front(j) : c->queue.push_back(j);
    } else if (j->opt.precision == GS_FP64) {
        Class<double, double>* c;
        if ((rc = get_class<double, double>(cx, &j->grid, j->opt.check_every, &c))) return rc;
        front ? c->queue.push_front(j) : c->queue.push_back(j);
    } else {
        Class<float, float>* c;
        if ((rc = get_class<float, float>(cx, &j->grid, j->opt.check_every, &c))) return rc;
        front ? c->queue.push_front(j) : c->queue.push_back(j);
    }
    return GS_OK;
}

// Cascadic multigrid: the level just finished wrote its result to cm_buf[0];
// interpolate it to the next grid (into cm_buf[1], the next level's guess) on
// stream s and queue the request in the next grid's class.
static int next_level(Ctx& cx, Job* j, hipStream_t s) {
    const gs_grid gc = j->grid;
    const gs_grid gf = level_grid(j->fine, j->nlevels, j->level + 1);
    int rc;
    // cm_buf[0] (coarse result) is free after the forward transform: it holds
    // the padded spectrum; cm_buf[1] is scratch, then the result
    if ((rc = fft_impl<double>(cx, &gc, -1, j->cm_buf[0], j->cm_buf[1], s))) return rc;
    const int nc[3] = {gc.n[0], gc.n[1], gc.dim == 3 ? gc.n[2] : 1};
    const int nf[3] = {gf.n[0], gf.n[1], gf.dim == 3 ? gf.n[2] : 1};
    HIPCHK(launch_spec_pad(j->cm_buf[1], j->cm_buf[0], gc.dim, nc, nf, s));
    if ((rc = fft_impl<double>(cx, &gf, +1, j->cm_buf[0], j->cm_buf[1], s))) return rc;
    if (!j->ev) HIPCHK(hipEventCreateWithFlags(&j->ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(j->ev, s));
    j->wait_ev = true;
    j->level++;
    j->grid = gf;
    if ((rc = make_phys(&gf, &j->trap, &j->prm, &j->ph, j->opt.nyquist_odd == GS_NYQ_ZERO))) return rc;
    j->psi0 = j->cm_buf[1];
    j->out = j->level + 1 == j->nlevels ? j->user_out : j->cm_buf[0];
    j->iters_fp32 = 0;
    j->stage = JS_QUEUED;
    j->slot = -1;
    j->handover = false;
    if ((rc = enqueue(cx, j, true))) return rc;
    cx.moves++;
    return GS_OK;
}

// Timings of a tuning chunk that has completed (adv[i]: steps slot i accepted
// in it): launches at iterations that every slot of the chunk ran are added
// per pass and candidate, leaving out each candidate's first launch (code load,
// cold caches). A bucket is decided once every valid candidate of every pass
// has two counted launches, or after three tuning chunks with what was seen.
template <typename RS, typename RD>
static hipError_t tune_collect(Class<RS, RD>& c, const std::vector<int>& adv) {
    TuneRun& run = c.tun.run;
    const int b = run.bucket;
    int full = INT32_MAX;
    for (int a : adv) full = std::min(full, a);
    for (size_t i = 0; i < run.rec.size(); ++i) {
        const TuneRun::Rec& r = run.rec[i];
        if (r.it >= full) continue;
        float ms = 0.0f;
        hipError_t e = hipEventElapsedTime(&ms, run.ev[2 * i], run.ev[2 * i + 1]);
        if (e != hipSuccess) return e;
        if (c.tun.seen[b][r.pass][r.cand]++ == 0) continue;
        c.tun.ms[b][r.pass][r.cand] += ms;
        c.tun.n[b][r.pass][r.cand]++;
    }
    run.rec.clear();
    run.on = false;
    bool all = true;
    for (int p = 0; p < NPASS; ++p)
        for (int cd : c.valid[p]) all = all && c.tun.n[b][p][cd] >= 2;
    if (all || c.tun.chunks[b] >= 3) {
        for (int p = 0; p < NPASS; ++p) {
            int best = 0;
            double tb = 0.0;
            for (int cd : c.valid[p]) {
                if (c.tun.n[b][p][cd] == 0) continue;
                const double t = c.tun.ms[b][p][cd] / c.tun.n[b][p][cd];
                if (tb == 0.0 || t < tb) { tb = t; best = cd; }
            }
            c.tun.best[b].c[p] = best;
        }
        c.tun.decided[b] = true;
    }
    return hipSuccess;
}

// Chunk boundary of a class whose previous chunk (if any) has completed:
// retire finished solves, start final evaluations, hand over float phases,
// admit queued requests, then enqueue the next chunk.
template <typename RS, typename RD>
static int boundary(Ctx& cx, Class<RS, RD>& c) {
    constexpr bool is64 = std::is_same<RS, double>::value;
    int rc;
    // 1. final evaluations enqueued at the previous boundary have completed
    for (int k : c.fin) {
        Job* j = c.owner[k];
        const SolveState& h = c.h_st[k];
        c.owner[k] = nullptr;
        if (!is64) j->iters_fp32 = h.iter;
        if (h.nonfinite) finish_job(cx, j, GS_ENONFINITE, &h, "non-finite value in the final evaluation");
        else if (j->level + 1 < j->nlevels && !j->cancel) {
            j->iters_coarse += h.iter;
            if ((rc = next_level(cx, j, c.stream))) finish_job(cx, j, rc, &h, g_err);
        } else finish_job(cx, j, h.status, &h, "");
    }
    c.fin.clear();
    // 2. slots of the chunk that has completed
    if (!c.run.empty() && (c.tm.kind >= 0 || c.tun.run.on)) {
        std::vector<int> adv;
        std::vector<char> fin;
        for (size_t i = 0; i < c.run.size(); ++i) {
            const SolveState& h = c.h_st[c.run[i]];
            adv.push_back(h.iter - c.iter0[i]);
            fin.push_back(h.done ? 1 : 0);
        }
        if (c.tm.kind >= 0) HIPCHK(timer_collect(c.tm, cx.timer, adv, fin));
        if (c.tun.run.on) HIPCHK(tune_collect(c, adv));
    }
    std::vector<int> cont;
    for (size_t i = 0; i < c.run.size(); ++i) {
        const int k = c.run[i];
        Job* j = c.owner[k];
        SolveState& h = c.h_st[k];
        if (j->cancel) {
            finish_job(cx, j, GS_ECANCELED, &h, "request cancelled");
            c.owner[k] = nullptr;
            continue;
        }
        if (!h.done) {
            if (h.iter == c.iter0[i]) {   // every iteration accepts a step or ends the solve
                finish_job(cx, j, GS_EDEVICE, &h, "solver made no progress (device state not updated)");
                c.owner[k] = nullptr;
                continue;
            }
            cont.push_back(k);
            continue;
        }
        if (h.nonfinite) {
            if (!is64) j->iters_fp32 = h.iter;
            finish_job(cx, j, GS_ENONFINITE, &h, "non-finite value in the iteration (check the input and parameters)");
            c.owner[k] = nullptr;
            continue;
        }
        if constexpr (!is64) {
            if (h.switch_req && j->opt.precision == GS_MIXED) {
                rc = hand_over(cx, c, k, j);
                if (rc) finish_job(cx, j, rc, &h, g_err);
                c.owner[k] = nullptr;
                continue;
            }
        }
        h.done = 0;   // the final evaluation runs while done == 0
        j->stage = JS_FINAL;
        c.fin.push_back(k);
    }
    // 3. admissions. Requests that already hold their reservation (hand-overs
    //    and later multigrid levels) are always admitted; new requests in
    //    arrival order while their footprint fits in the budget.
    std::vector<int> fresh;
    std::deque<Job*> waiting;
    bool blocked = false;
    while (!c.queue.empty()) {
        Job* j = c.queue.front();
        c.queue.pop_front();
        if (j->cancel) {
            // a handed-over slot may still be the target of the hand-over copy on
            // another stream: order the slot's next use on this stream after it
            if (j->wait_ev) {
                HIPCHK(hipStreamWaitEvent(c.stream, j->ev, 0));
                j->wait_ev = false;
            }
            if (j->slot >= 0) c.owner[j->slot] = nullptr;
            finish_job(cx, j, GS_ECANCELED, nullptr, "request cancelled");
            continue;
        }
        int k = j->slot;
        if (!j->handover) {
            if (!j->admitted && (blocked || cx.reserved + j->reserve > cx.budget)) {
                blocked = true;   // wait for memory; later new requests wait behind it
                waiting.push_back(j);
                continue;
            }
            rc = acquire_slot<RS, RD>(cx, c, j, c.stream, &k);
            if (rc == SLOT_WAIT) {
                blocked = blocked || !j->admitted;
                waiting.push_back(j);
                continue;
            }
            if (rc) {
                finish_job(cx, j, rc, nullptr, g_err);
                continue;
            }
            if (!j->admitted) {
                cx.reserved += j->reserve;
                j->admitted = true;
            }
            j->slot = k;
        }
        if (j->wait_ev) {
            HIPCHK(hipStreamWaitEvent(c.stream, j->ev, 0));
            j->wait_ev = false;
        }
        if (j->handover) {
            c.h_st[k] = j->mig;
            j->handover = false;
        } else {
            init_state(&c.h_st[k], &j->opt, j->opt.precision == GS_MIXED ? PH_FP32 : PH_FP64);
            if ((rc = load_guess<RS, RD>(c, k, j))) return rc;
        }
        HIPCHK(hipMemsetAsync(c.mem[k]->buf[B_P], 0, sizeof(cpx<RD>) * 3 * c.M, c.stream));
        fresh.push_back(k);
        j->stage = JS_RUNNING;
    }
    c.queue = std::move(waiting);
    // 4. launch table: [fresh..., continuing...] run the chunk, then the slots
    //    under final evaluation
    c.run = fresh;
    c.run.insert(c.run.end(), cont.begin(), cont.end());
    if (c.run.empty() && c.fin.empty()) {
        c.inflight = false;
        return GS_OK;
    }
    int nt = 0, rot_any = 0, maxk = 0;
    c.iter0.clear();
    for (int k : c.run) c.iter0.push_back(c.h_st[k].iter);
    auto put = [&](int k) {
        const Phys& ph = c.owner[k]->ph;
        c.h_tab[nt++] = entry_of(*c.mem[k], c.d_st + k, ph);
        rot_any |= ph.omega != 0.0;
        maxk = std::max(maxk, k + 1);
    };
    for (int k : c.run) put(k);
    for (int k : c.fin) put(k);
    const int nrun = (int)c.run.size(), nfin = (int)c.fin.size(), nnew = (int)fresh.size();
    hipStream_t s = c.stream;
    HIPCHK(hipMemcpyAsync(c.d_st, c.h_st, sizeof(SolveState) * maxk, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c.d_tab, c.h_tab, sizeof(Slot) * nt, hipMemcpyHostToDevice, s));
    const Geo<RS, RD> G = geo_of<RS, RD>(c.grid, c.M, c.g, c.tws, c.twd, rot_any);
    if (nfin) {
        const Sub Lf{c.d_tab + nrun, nfin};
        HIPCHK((refresh<RS, RD>(G, Lf, s, nullptr)));
        HIPCHK((resid_final<RS, RD>(G, Lf, s)));
        for (int k : c.fin)
            if ((rc = copy_out<RS, RD>(c, k, c.owner[k]))) return rc;
    }
    if (nnew) HIPCHK((normalize<RS, RD>(G, Sub{c.d_tab, nnew}, s)));
    if (nrun) {
        c.tm.kind = cx.timer.kind;
        Timer* tm = c.tm.kind >= 0 ? &c.tm : nullptr;
        const Sub Lr{c.d_tab, nrun};
        // schedules: the bucket's decision, or a tuning chunk that cycles
        // through every pass's valid candidates (not while the kernel timer,
        // which takes the launches' events, is on)
        const int b = bucket_of(nrun);
        TuneRun* tr = nullptr;
        if (cx.autotune && !c.tun.decided[b] && !tm) {
            tr = &c.tun.run;
            tr->on = true;
            tr->bucket = b;
            tr->rec.clear();
            c.tun.chunks[b]++;
        }
        for (int it = 0; it < c.check_every; ++it) {
            if (tm) tm->iter_in_chunk = it;
            Sched sc;
            if (tr) {
                tr->it = it;
                for (int p = 0; p < NPASS; ++p)
                    if (!c.valid[p].empty()) sc.c[p] = c.valid[p][it % c.valid[p].size()];
            } else if (cx.autotune && c.tun.decided[b]) {
                sc = c.tun.best[b];
            }
            HIPCHK((iterate<RS, RD>(G, Lr, it == 0, s, tm, &sc, tr)));
        }
    }
    HIPCHK(hipMemcpyAsync(c.h_st, c.d_st, sizeof(SolveState) * maxk, hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(c.ev, s));
    c.inflight = true;
    c.seq = cx.next_seq++;
    return GS_OK;
}

template <typename RS, typename RD>
static int visit(Ctx& cx, Class<RS, RD>& c, bool& did) {
    if (c.inflight) {
        hipError_t q = hipEventQuery(c.ev);
        if (q == hipErrorNotReady) return GS_OK;
        if (q != hipSuccess) return fail(GS_EDEVICE, std::string("chunk completion: ") + hipGetErrorString(q));
        c.inflight = false;
    } else if (c.queue.empty() && c.run.empty() && c.fin.empty()) {
        return GS_OK;
    }
    int rc = boundary<RS, RD>(cx, c);
    if (rc) return rc;
    did = did || c.inflight;
    return GS_OK;
}

// Advance every class whose chunk has completed. block: if nothing could be
// advanced, wait for the chunk enqueued first and try again.
static int progress(Ctx& cx, bool block) {
    for (;;) {
        bool did = false;
        int rc;
        const uint64_t moves0 = cx.moves;
        if ((rc = each_class(cx, [&](auto& c) { return visit(cx, c, did); }))) return rc;
        if (cx.moves != moves0) continue;   // a request entered a class already visited
        if (!block || did) return GS_OK;
        hipEvent_t e = nullptr;
        uint64_t best = UINT64_MAX;
        each_class(cx, [&](auto& c) {
            if (c.inflight && c.seq < best) { best = c.seq; e = c.ev; }
            return 0;
        });
        if (!e) return GS_OK;   // nothing in flight
        HIPCHK(hipEventSynchronize(e));
    }
}

// Slot bytes of every precision phase of a solve of grid g.
static size_t footprint(const gs_grid* g, const gs_options* o) {
    size_t b = 0;
    if (o->precision != GS_FP64) b += slot_bytes<float, float>(g);
    if (o->precision != GS_FP32)
        b += o->dir_precision == GS_FP32 ? slot_bytes<double, float>(g) : slot_bytes<double, double>(g);
    return b;
}

static int submit_job(Ctx& cx, const gs_request* q, uint64_t* ticket) {
    int rc;
    if (!q) return fail(GS_EINVAL, "request is NULL");
    if ((rc = check_grid(&q->grid))) return rc;
    if ((rc = check_options(&q->options))) return rc;
    if (!q->d_psi_out) return fail(GS_EINVAL, "request.d_psi_out is NULL");
    auto j = std::make_unique<Job>();
    j->fine = q->grid;
    if (j->fine.dim == 2) j->fine.n[2] = 1;
    j->opt = q->options;
    j->nlevels = q->options.cm_levels;
    j->trap = q->trap;
    j->trap.V = nullptr;
    j->prm = q->params;
    if (j->nlevels > 1) {
        if (q->trap.V) return fail(GS_EINVAL, "a sampled trap V cannot be used with cm_levels > 1");
        for (int a = 0; a < j->fine.dim; ++a)
            if ((j->fine.n[a] >> (j->nlevels - 1)) < 16)
                return fail(GS_EINVAL, "cm_levels too large: the coarsest grid needs n[a] >= 16");
    }
    j->grid = level_grid(j->fine, j->nlevels, 0);
    const int nyq = q->options.nyquist_odd == GS_NYQ_ZERO;
    if ((rc = make_phys(&j->fine, &q->trap, &q->params, &j->ph, nyq))) return rc;   // validates the full-size V
    if ((rc = make_phys(&j->grid, &q->trap, &q->params, &j->ph, nyq))) return rc;
    j->warn_existence = existence(&j->fine, &q->trap, &q->params) == GS_WEXISTENCE;
    const long long M = npts(&j->fine);
    j->reserve = 0;
    j->reserve = footprint(&j->fine, &q->options);
    if (q->trap.V) j->reserve += sizeof(double) * M;
    if (j->nlevels > 1) j->reserve += 2 * sizeof(cpx<double>) * 3 * M;
    if (j->reserve > cx.budget) return fail(GS_ENOMEM, "request needs more device memory than the budget");
    if (j->nlevels > 1)
        for (auto*& b : j->cm_buf)
            if (hipMalloc((void**)&b, sizeof(cpx<double>) * 3 * M) != hipSuccess) {
                b = nullptr;
                (void)hipGetLastError();
                return fail(GS_ENOMEM, "device allocation failed (multigrid buffers)");
            }
    if (q->trap.V) {
        if (hipMalloc((void**)&j->Vdev, sizeof(double) * M) != hipSuccess) {
            j->Vdev = nullptr;
            (void)hipGetLastError();
            return fail(GS_ENOMEM, "device allocation failed (V)");
        }
        HIPCHK(hipMemcpy(j->Vdev, q->trap.V, sizeof(double) * M, hipMemcpyHostToDevice));
        j->ph.V = j->Vdev;
    }
    j->psi0 = (const cpx<double>*)q->d_psi0;
    j->user_out = (cpx<double>*)q->d_psi_out;
    j->out = j->nlevels > 1 ? j->cm_buf[0] : j->user_out;
    j->t0 = std::chrono::steady_clock::now();
    if ((rc = enqueue(cx, j.get(), false))) return rc;
    j->ticket = cx.next_ticket++;
    *ticket = j->ticket;
    cx.jobs[j->ticket] = std::move(j);
    return GS_OK;
}

// Result of a completed request; the ticket is released.
static int take_result(Ctx& cx, uint64_t ticket, gs_result* res) {
    auto it = cx.jobs.find(ticket);
    Job* j = it->second.get();
    if (res) *res = j->res;
    const int rc = j->rc;
    if (rc < 0) g_err = j->err;
    cx.jobs.erase(it);
    return rc;
}

static int wait_job(Ctx& cx, uint64_t ticket, gs_result* res) {
    auto it = cx.jobs.find(ticket);
    if (it == cx.jobs.end()) return fail(GS_EINVAL, "unknown ticket");
    Job* j = it->second.get();
    while (j->stage != JS_DONE) {
        int rc = progress(cx, true);
        if (rc) return rc;
        bool any = false;
        each_class(cx, [&](auto& c) { any = any || c.inflight; return 0; });
        if (!any && j->stage != JS_DONE) return fail(GS_EDEVICE, "request is not progressing");
    }
    return take_result(cx, ticket, res);
}

static int solve_device_impl(Ctx& cx, const gs_grid* g, const gs_trap* t, const gs_params* p, const gs_options* o,
                             const void* d_psi0, void* d_out, gs_result* res) {
    if (!p) return fail(GS_EINVAL, "params is NULL");
    gs_request q;
    std::memset(&q, 0, sizeof(q));
    if (g) q.grid = *g;
    else return fail(GS_EINVAL, "grid is NULL");
    if (t) q.trap = *t;
    else {
        q.trap.g[0] = q.trap.g[1] = q.trap.g[2] = 1.0;
    }
    q.params = *p;
    if (!o) return fail(GS_EINVAL, "options is NULL");
    q.options = *o;
    q.d_psi0 = d_psi0;
    q.d_psi_out = d_out;
    uint64_t ticket = 0;
    int rc = submit_job(cx, &q, &ticket);
    if (rc) return rc;
    return wait_job(cx, ticket, res);
}

// ---------------------------------------------------------------------------
// operator-level entry points (one slot of their own per grid and precision)
// ---------------------------------------------------------------------------
template <typename R>
static int get_opplan(Ctx& cx, const gs_grid* g, OpPlan<R>** out, hipStream_t s) {
    auto key = grid_key(g);
    auto& mp = opplans<R>(cx);
    auto it = mp.find(key);
    if (it != mp.end()) {
        *out = it->second.get();
        return GS_OK;
    }
    auto op = std::make_unique<OpPlan<R>>();
    op->grid = *g;
    if (g->dim == 2) op->grid.n[2] = 1;
    op->M = npts(g);
    op->g = red_geom<R>(g);
    int rc;
    for (int a = 0; a < g->dim; ++a)
        if ((rc = get_twiddle<R>(cx, g->n[a], &op->tw[a]))) return rc;
    if ((rc = alloc_slot_mem<R, R>(g, s, op->mem))) return rc;
    if (hipMalloc((void**)&op->d_st, sizeof(SolveState)) != hipSuccess ||
        hipMalloc((void**)&op->d_tab, sizeof(Slot)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GS_ENOMEM, "device allocation failed (operator plan)");
    }
    if (hipHostMalloc((void**)&op->h_st, sizeof(SolveState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&op->h_tab, sizeof(Slot), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GS_ENOMEM, "pinned allocation failed (operator plan)");
    }
    *out = op.get();
    mp[key] = std::move(op);
    return GS_OK;
}

// Upload the slot descriptor (caller buffers as X0, X1) and a state for a
// single evaluation. The stream is drained first: the pinned staging of the
// previous call may still be in use by its copies.
template <typename R>
static int op_setup(OpPlan<R>& op, const Phys& ph, const void* x0, void* x1, hipStream_t s) {
    HIPCHK(hipStreamSynchronize(s));
    gs_options o;
    gs_default_options(&o);
    o.max_iter = 1 << 30;
    init_state(op.h_st, &o, PH_FP64);
    *op.h_tab = entry_of(*op.mem, op.d_st, ph);
    op.h_tab->buf[B_X0] = const_cast<void*>(x0);
    op.h_tab->buf[B_X1] = x1;
    HIPCHK(hipMemcpyAsync(op.d_st, op.h_st, sizeof(SolveState), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(op.d_tab, op.h_tab, sizeof(Slot), hipMemcpyHostToDevice, s));
    return GS_OK;
}

// The passes of a forward (sign -1) or inverse (sign +1) transform of the
// three components of X0 into X1 (scratch T0, T1) of the one-slot table T.
template <typename R>
static int fft_passes(const gs_grid* g, int sign, const Slot* T, const cpx<R>* const tw[3], hipStream_t s) {
    const int Nx = g->n[0], Ny = g->n[1], Nz = g->dim == 3 ? g->n[2] : 1;
    const double invM = 1.0 / ((double)Nx * Ny * Nz);
    if (sign < 0) {
        if (g->dim == 2) {
            HIPCHK((launch_fwdT<R, R>(Nx, PRO_PLAIN, 0, T, 1, B_X0, B_T0, B_NONE, B_NONE, 1, Ny, 3, tw[0], 0, s)));
            HIPCHK((launch_fwdT<R, R>(Ny, PRO_PLAIN, 0, T, 1, B_T0, B_X1, B_NONE, B_NONE, 1, Nx, 3, tw[1], 0, s)));
        } else {
            HIPCHK((launch_fwdT<R, R>(Nx, PRO_PLAIN, 0, T, 1, B_X0, B_T0, B_NONE, B_NONE, Nz, Ny, 3, tw[0], 0, s)));
            HIPCHK((launch_fwdT<R, R>(Ny, PRO_PLAIN, 0, T, 1, B_T0, B_T1, B_NONE, B_NONE, Nx, Nz, 3, tw[1], 0, s)));
            HIPCHK((launch_fwdT<R, R>(Nz, PRO_PLAIN, 0, T, 1, B_T1, B_X1, B_NONE, B_NONE, Ny, Nx, 3, tw[2], 0, s)));
        }
    } else {
        if (g->dim == 2) {
            HIPCHK(launch_invT<R>(Ny, EPI_SCALE, T, 1, B_X0, B_NONE, B_T0, B_NONE, B_NONE, 1, Nx, 1.0, 0, 0, tw[1], 0, s));
            HIPCHK(launch_invT<R>(Nx, EPI_SCALE, T, 1, B_T0, B_NONE, B_X1, B_NONE, B_NONE, 1, Ny, invM, 0, 0, tw[0], 0, s));
        } else {
            HIPCHK(launch_invT<R>(Nz, EPI_SCALE, T, 1, B_X0, B_NONE, B_T0, B_NONE, B_NONE, Ny, Nx, 1.0, 0, 0, tw[2], 0, s));
            HIPCHK(launch_invT<R>(Ny, EPI_SCALE, T, 1, B_T0, B_NONE, B_T1, B_NONE, B_NONE, Nx, Nz, 1.0, 0, 0, tw[1], 0, s));
            HIPCHK(launch_invT<R>(Nx, EPI_SCALE, T, 1, B_T1, B_NONE, B_X1, B_NONE, B_NONE, Nz, Ny, invM, 0, 0, tw[0], 0, s));
        }
    }
    return GS_OK;
}

template <typename R>
static int fft_impl(Ctx& cx, const gs_grid* g, int sign, const cpx<R>* in, cpx<R>* out, hipStream_t s) {
    OpPlan<R>* op;
    int rc;
    if ((rc = get_opplan<R>(cx, g, &op, s))) return rc;
    Phys ph;
    if ((rc = make_phys(g, nullptr, nullptr, &ph))) return rc;
    if ((rc = op_setup<R>(*op, ph, in, out, s))) return rc;
    return fft_passes<R>(g, sign, op->d_tab, op->tw, s);
}

// ---------------------------------------------------------------------------
// the transform without allocation (gs_fft_noalloc)
// ---------------------------------------------------------------------------
// Every buffer of a call lives in `scratch`, one file-scope device array per
// GPU: the one-slot descriptor table and its solver state (header), the
// twiddle tables of every supported line length in both precisions (written
// once per device by gs_create), and the two scratch fields of a 3D transform
// of up to NA_MAX_POINTS points per component. Host code addresses the array
// only through the device pointer that hipGetSymbolAddress returned for the
// device (na_base). Calls on one GPU share the array: calls that overlap in
// time (different streams or host threads) race.
constexpr long long NA_MAX_POINTS = 1LL << 18;
constexpr size_t NA_HDR = 4096;            // descriptor at 0, solver state at 1024
constexpr int NA_LENGTHS[] = {16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 80, 160, 600, 1200, 2400};
constexpr int NA_NLEN = (int)(sizeof(NA_LENGTHS) / sizeof(NA_LENGTHS[0]));
constexpr size_t na_tw_bytes() {
    size_t b = 0;
    for (int k = 0; k < NA_NLEN; ++k)   // double table; float table with its double copy
        b += (size_t)NA_LENGTHS[k] * (sizeof(cpx<double>) + sizeof(cpx<float>) + sizeof(cpx<double>));
    return (b + 255) & ~(size_t)255;
}
constexpr size_t NA_FIELD = (size_t)3 * NA_MAX_POINTS * sizeof(cpx<double>);
constexpr size_t NA_TW_OFF = NA_HDR, NA_T0_OFF = NA_TW_OFF + na_tw_bytes(), NA_T1_OFF = NA_T0_OFF + NA_FIELD;
constexpr size_t NA_BYTES = NA_T1_OFF + NA_FIELD;
static_assert(sizeof(Slot) <= 1024 && sizeof(SolveState) <= NA_HDR - 1024, "header layout");

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

// offset of the twiddle table of length N and element size rsize in scratch
static size_t na_tw_offset(int N, size_t rsize) {
    size_t off = NA_TW_OFF;
    for (int k = 0; k < NA_NLEN; ++k) {
        const size_t n = (size_t)NA_LENGTHS[k];
        if (NA_LENGTHS[k] == N) return rsize == sizeof(double) ? off : off + n * sizeof(cpx<double>);
        off += n * (sizeof(cpx<double>) + sizeof(cpx<float>) + sizeof(cpx<double>));
    }
    return 0;
}

constexpr int NA_MAX_DEV = 64;
static std::mutex na_mutex;
static unsigned char* na_base[NA_MAX_DEV] = {};

// Once per device, with the device current: the device address of scratch and
// the twiddle tables (the same images as the allocating path's tables).
static int na_init(int device) {
    if (device < 0 || device >= NA_MAX_DEV) return fail(GS_EINVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(na_mutex);
    if (na_base[device]) return GS_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return fail(GS_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    unsigned char* base = static_cast<unsigned char*>(ptr);
    for (int k = 0; k < NA_NLEN; ++k) {
        const int N = NA_LENGTHS[k];
        const std::vector<unsigned char> d = twiddle_image<double>(N), f = twiddle_image<float>(N);
        HIPCHK(hipMemcpy(base + na_tw_offset(N, sizeof(double)), d.data(), d.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(base + na_tw_offset(N, sizeof(float)), f.data(), f.size(), hipMemcpyHostToDevice));
    }
    na_base[device] = base;
    return GS_OK;
}

// writes the one-slot descriptor and a zeroed solver state (done = 0) on the
// call's stream, so that no host staging buffer is involved
__global__ void k_na_setup(Slot e, Slot* dst, SolveState* st) {
    if (threadIdx.x == 0) {
        *dst = e;
        SolveState z;
        memset(&z, 0, sizeof z);
        *st = z;
    }
}

template <typename R>
static int fft_noalloc_impl(int device, const gs_grid* g, int sign, const cpx<R>* in, cpx<R>* out, hipStream_t s) {
    unsigned char* base;
    {
        std::lock_guard<std::mutex> lk(na_mutex);
        base = (device >= 0 && device < NA_MAX_DEV) ? na_base[device] : nullptr;
    }
    if (!base) return fail(GS_EDEVICE, "scratch of this device not set up (gs_create)");
    Phys ph;
    int rc;
    if ((rc = make_phys(g, nullptr, nullptr, &ph))) return rc;
    Slot e;
    std::memset(&e, 0, sizeof e);
    e.buf[B_X0] = const_cast<cpx<R>*>(in);
    e.buf[B_X1] = out;
    e.buf[B_T0] = base + NA_T0_OFF;
    e.buf[B_T1] = base + NA_T1_OFF;
    e.st = reinterpret_cast<SolveState*>(base + 1024);
    e.p = ph;
    Slot* T = reinterpret_cast<Slot*>(base);
    GS_LAUNCH(k_na_setup, dim3(1), dim3(64), 0, s, e, T, e.st);
    HIPCHK(hipGetLastError());
    const cpx<R>* tw[3] = {};
    for (int a = 0; a < g->dim; ++a) tw[a] = reinterpret_cast<const cpx<R>*>(base + na_tw_offset(g->n[a], sizeof(R)));
    return fft_passes<R>(g, sign, T, tw, s);
}

// user potential of an operator-level call: a device copy owned by the plan's context
static int op_potential(Ctx& cx, const gs_trap* t, Phys& ph, double** Vdev) {
    *Vdev = nullptr;
    if (!t || !t->V) return GS_OK;
    if (hipMalloc((void**)Vdev, sizeof(double) * ph.M) != hipSuccess) {
        *Vdev = nullptr;
        (void)hipGetLastError();
        return fail(GS_ENOMEM, "device allocation failed (V)");
    }
    HIPCHK(hipMemcpy(*Vdev, t->V, sizeof(double) * ph.M, hipMemcpyHostToDevice));
    ph.V = *Vdev;
    (void)cx;
    return GS_OK;
}

template <typename R>
static int ham_impl(Ctx& cx, const gs_grid* g, const gs_trap* t, const gs_params* p, const cpx<R>* psi,
                    cpx<R>* hpsi, gs_result* res, hipStream_t s) {
    OpPlan<R>* op;
    int rc;
    if ((rc = get_opplan<R>(cx, g, &op, s))) return rc;
    Phys ph;
    if ((rc = make_phys(g, t, p, &ph))) return rc;
    double* Vdev = nullptr;
    if ((rc = op_potential(cx, t, ph, &Vdev))) return rc;
    rc = op_setup<R>(*op, ph, psi, hpsi, s);
    const Sub L{op->d_tab, 1};
    const Geo<R, R> G = geo_of<R, R>(op->grid, op->M, op->g, op->tw, op->tw, ph.omega != 0.0);
    hipError_t e = hipSuccess;
    if (!rc) e = hipMemcpyAsync(op->mem->buf[B_PHI], psi, sizeof(cpx<R>) * 3 * op->M, hipMemcpyDeviceToDevice, s);
    if (!rc && !e) e = refresh<R, R>(G, L, s, nullptr);
    if (!rc && !e) e = resid_final<R, R>(G, L, s);
    if (!rc && !e) e = launch_hphi<R>(L.tab, 1, G.g, s);
    if (!rc && !e && (res || Vdev)) {
        e = hipMemcpyAsync(op->h_st, op->d_st, sizeof(SolveState), hipMemcpyDeviceToHost, s);
        if (!e) e = hipStreamSynchronize(s);
        if (!e && res) {
            fill_result(op->h_st, res, 0, 0.0);
            res->status = GS_OK;
        }
    }
    if (Vdev) (void)hipFree(Vdev);
    if (rc) return rc;
    if (e) return fail(GS_EDEVICE, hipGetErrorString(e));
    return GS_OK;
}

template <typename R>
static int pre_impl(Ctx& cx, const gs_grid* g, const gs_trap* t, const gs_params* p, const cpx<R>* psi,
                    const cpx<R>* r, cpx<R>* out, hipStream_t s) {
    OpPlan<R>* op;
    int rc;
    if ((rc = get_opplan<R>(cx, g, &op, s))) return rc;
    Phys ph;
    if ((rc = make_phys(g, t, p, &ph))) return rc;
    double* Vdev = nullptr;
    if ((rc = op_potential(cx, t, ph, &Vdev))) return rc;
    rc = op_setup<R>(*op, ph, r, out, s);
    const Sub L{op->d_tab, 1};
    const Geo<R, R> G = geo_of<R, R>(op->grid, op->M, op->g, op->tw, op->tw, ph.omega != 0.0);
    hipError_t e = hipSuccess;
    if (!rc) e = hipMemcpyAsync(op->mem->buf[B_PHI], psi, sizeof(cpx<R>) * 3 * op->M, hipMemcpyDeviceToDevice, s);
    if (!rc && !e) e = refresh<R, R>(G, L, s, nullptr);
    if (!rc && !e) e = launch_pvin<R>(L.tab, 1, G.g, s);
    if (!rc && !e) e = chain_pre<R, R>(G, L, 0, B_X1, s, nullptr);
    if (!rc && !e && Vdev) e = hipStreamSynchronize(s);
    if (Vdev) (void)hipFree(Vdev);
    if (rc) return rc;
    if (e) return fail(GS_EDEVICE, hipGetErrorString(e));
    return GS_OK;
}

// JSON description of the autotuner's decisions and timings in every class.
template <typename RS, typename RD>
static void report_class(const Class<RS, RD>& c, std::string& out, bool& first) {
    char buf[256];
    for (int b = 0; b < NBUCKET; ++b) {
        if (!c.tun.chunks[b]) continue;
        const int lo = 1 << b, hi = b + 1 < NBUCKET ? (2 << b) - 1 : 4096;
        std::snprintf(buf, sizeof buf, "%s{\"grid\":[%d,%d,%d],\"state\":\"%s\",\"dir\":\"%s\",\"running\":[%d,%d],"
                      "\"tuning_chunks\":%d,\"decided\":%s,\"passes\":{",
                      first ? "" : ",", c.grid.n[0], c.grid.n[1], c.grid.dim == 3 ? c.grid.n[2] : 1,
                      sizeof(RS) == 8 ? "fp64" : "fp32", sizeof(RD) == 8 ? "fp64" : "fp32", lo, hi, c.tun.chunks[b],
                      c.tun.decided[b] ? "true" : "false");
        out += buf;
        first = false;
        bool fp = true;
        const int nn[3] = {c.grid.n[0], c.grid.n[1], c.grid.dim == 3 ? c.grid.n[2] : 1};
        for (int p = 0; p < NPASS; ++p) {
            if (c.valid[p].empty()) continue;
            const Cand ch = cand_of<RD>(c.grid.dim, nn, p, c.tun.best[b].c[p]);
            std::snprintf(buf, sizeof buf, "%s\"%s\":{\"chosen\":\"%dx%d\",\"us\":{", fp ? "" : ",", PASS_NAME[p],
                          ch.tile, ch.nt);
            out += buf;
            fp = false;
            bool fc = true;
            for (int cd : c.valid[p]) {
                const Cand k = cand_of<RD>(c.grid.dim, nn, p, cd);
                const int n = c.tun.n[b][p][cd];
                std::snprintf(buf, sizeof buf, "%s\"%dx%d\":%.3f", fc ? "" : ",", k.tile, k.nt,
                              n ? 1e3 * c.tun.ms[b][p][cd] / n : -1.0);
                out += buf;
                fc = false;
            }
            out += "}}";
        }
        out += "}}";
    }
}

}  // namespace gs

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace gs;

struct gs_ctx {
    Ctx impl;
};

extern "C" {

const char* gs_last_error(void) { return g_err.c_str(); }

void gs_default_options(gs_options* o) {
    if (!o) return;
    o->stop_kind = GS_STOP_ENERGY;
    o->tol = 1e-12;
    o->max_iter = 100000;
    o->precision = GS_FP64;
    o->switch_resid = 1e-6;
    o->fp32_max_iter = 20000;
    o->stall_window = 50;
    o->theta_trial = 0.1;
    o->sigma = 0.5;
    o->max_backtrack = 40;
    o->check_every = 32;
    o->cm_levels = 1;
    o->dir_precision = GS_FP64;
    o->precond = GS_PC_COMBINED;
    o->line_search = GS_LS_ALG2;
    o->nyquist_odd = GS_NYQ_KEEP;
}

int gs_existence_check(const gs_grid* g, const gs_trap* t, const gs_params* p) { return existence(g, t, p); }

size_t gs_footprint_bytes(const gs_grid* g, const gs_options* o) {
    if (check_grid(g) != GS_OK || check_options(o) != GS_OK) return 0;
    return footprint(g, o);
}

int gs_create(gs_ctx** out, int device) {
    if (!out) return fail(GS_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(GS_EDEVICE, "no HIP device");
    if (device < 0 || device >= ndev) return fail(GS_EINVAL, "device index out of range");
    if (hipSetDevice(device) != hipSuccess) return fail(GS_EDEVICE, "hipSetDevice failed");
    auto c = std::make_unique<gs_ctx>();
    Ctx& cx = c->impl;
    cx.device = device;
    size_t freeb = 0, total = 0;
    if (hipMemGetInfo(&freeb, &total) != hipSuccess) return fail(GS_EDEVICE, "hipMemGetInfo failed");
    cx.budget = (size_t)(0.9 * (double)freeb);
    int rc = na_init(device);
    if (rc) return rc;
    *out = c.release();
    return GS_OK;
}

void gs_destroy(gs_ctx* ctx) { delete ctx; }

int gs_set_hbm_budget(gs_ctx* ctx, size_t bytes) {
    if (!ctx) return fail(GS_EINVAL, "ctx is NULL");
    Ctx& cx = ctx->impl;
    if (hipSetDevice(cx.device) != hipSuccess) return fail(GS_EDEVICE, "hipSetDevice failed");
    if (bytes == 0) {
        size_t freeb = 0, total = 0;
        if (hipMemGetInfo(&freeb, &total) != hipSuccess) return fail(GS_EDEVICE, "hipMemGetInfo failed");
        bytes = (size_t)(0.9 * (double)(freeb + cx.allocated));
    }
    cx.budget = bytes;
    if (cx.allocated > cx.budget) trim(cx, 0);
    return GS_OK;
}

int gs_memory_stats(gs_ctx* ctx, size_t* budget, size_t* reserved, size_t* allocated) {
    if (!ctx) return fail(GS_EINVAL, "ctx is NULL");
    if (budget) *budget = ctx->impl.budget;
    if (reserved) *reserved = ctx->impl.reserved;
    if (allocated) *allocated = ctx->impl.allocated;
    return GS_OK;
}

int gs_solve(gs_ctx* ctx, const gs_grid* g, const gs_trap* t, const gs_params* p, const gs_options* o,
             const double* psi0, double* psi_out, gs_result* res) {
    if (!ctx) return fail(GS_EINVAL, "ctx is NULL");
    if (!psi_out) return fail(GS_EINVAL, "psi_out is NULL");
    int rc = check_grid(g);
    if (rc) return rc;
    Ctx& cx = ctx->impl;
    if (hipSetDevice(cx.device) != hipSuccess) return fail(GS_EDEVICE, "hipSetDevice failed");
    const size_t bytes = sizeof(cpx<double>) * 3 * npts(g);
    void *din = nullptr, *dout = nullptr;
    if (hipMalloc(&dout, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GS_ENOMEM, "device allocation failed (psi)");
    }
    if (psi0 && hipMalloc(&din, bytes) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(dout);
        return fail(GS_ENOMEM, "device allocation failed (psi0)");
    }
    if (psi0 && hipMemcpy(din, psi0, bytes, hipMemcpyHostToDevice) != hipSuccess) rc = fail(GS_EDEVICE, "copy of psi0 failed");
    if (!rc) rc = solve_device_impl(cx, g, t, p, o, din, dout, res);
    if (rc >= 0 && hipMemcpy(psi_out, dout, bytes, hipMemcpyDeviceToHost) != hipSuccess) rc = fail(GS_EDEVICE, "copy of psi failed");
    if (din) (void)hipFree(din);
    (void)hipFree(dout);
    return rc;
}

int gs_solve_device(gs_ctx* ctx, const gs_grid* g, const gs_trap* t, const gs_params* p, const gs_options* o,
                    const void* d_psi0, void* d_psi_out, gs_result* res, void* stream) {
    if (!ctx) return fail(GS_EINVAL, "ctx is NULL");
    if (!d_psi_out) return fail(GS_EINVAL, "d_psi_out is NULL");
    Ctx& cx = ctx->impl;
    if (hipSetDevice(cx.device) != hipSuccess) return fail(GS_EDEVICE, "hipSetDevice failed");
    // the guess may come from work queued on the caller's stream
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return fail(GS_EDEVICE, "hipStreamSynchronize failed");
    return solve_device_impl(cx, g, t, p, o, d_psi0, d_psi_out, res);
}

int gs_submit(gs_ctx* ctx, const gs_request* req, uint64_t* ticket) {
    if (!ctx || !ticket) return fail(GS_EINVAL, "NULL argument");
    Ctx& cx = ctx->impl;
    if (hipSetDevice(cx.device) != hipSuccess) return fail(GS_EDEVICE, "hipSetDevice failed");
    int rc = submit_job(cx, req, ticket);
    if (rc) return rc;
    return progress(cx, false);
}

int gs_progress(gs_ctx* ctx, int block) {
    if (!ctx) return fail(GS_EINVAL, "ctx is NULL");
    Ctx& cx = ctx->impl;
    if (hipSetDevice(cx.device) != hipSuccess) return fail(GS_EDEVICE, "hipSetDevice failed");
    int rc = progress(cx, block != 0);
    if (rc) return rc;
    int n = 0;
    for (auto& kv : cx.jobs) n += kv.second->stage != JS_DONE;
    return n;
}

int gs_poll(gs_ctx* ctx, uint64_t ticket, gs_result* res) {
    if (!ctx) return fail(GS_EINVAL, "ctx is NULL");
    Ctx& cx = ctx->impl;
    auto it = cx.jobs.find(ticket);
    if (it == cx.jobs.end()) return fail(GS_EINVAL, "unknown ticket");
    if (it->second->stage != JS_DONE) {
        if (hipSetDevice(cx.device) != hipSuccess) return fail(GS_EDEVICE, "hipSetDevice failed");
        int rc = progress(cx, false);
        if (rc) return rc;
        if (it->second->stage != JS_DONE) return GS_PENDING;
    }
    return take_result(cx, ticket, res);
}

int gs_wait(gs_ctx* ctx, uint64_t ticket, gs_result* res) {
    if (!ctx) return fail(GS_EINVAL, "ctx is NULL");
    Ctx& cx = ctx->impl;
    if (hipSetDevice(cx.device) != hipSuccess) return fail(GS_EDEVICE, "hipSetDevice failed");
    return wait_job(cx, ticket, res);
}

int gs_cancel(gs_ctx* ctx, uint64_t ticket) {
    if (!ctx) return fail(GS_EINVAL, "ctx is NULL");
    auto it = ctx->impl.jobs.find(ticket);
    if (it == ctx->impl.jobs.end()) return fail(GS_EINVAL, "unknown ticket");
    it->second->cancel = true;
    return GS_OK;
}

int gs_batch_solve(gs_ctx* ctx, int nreq, const gs_request* reqs, gs_result* res) {
    if (!ctx) return fail(GS_EINVAL, "ctx is NULL");
    if (nreq < 0 || (nreq > 0 && !reqs)) return fail(GS_EINVAL, "invalid request array");
    Ctx& cx = ctx->impl;
    if (hipSetDevice(cx.device) != hipSuccess) return fail(GS_EDEVICE, "hipSetDevice failed");
    std::vector<uint64_t> tickets;
    tickets.reserve(nreq);
    for (int i = 0; i < nreq; ++i) {
        uint64_t t = 0;
        int rc = submit_job(cx, &reqs[i], &t);
        if (rc) {
            const std::string msg = "request " + std::to_string(i) + ": " + g_err;
            for (uint64_t u : tickets) {   // nothing has been launched yet
                Job* j = cx.jobs[u].get();
                each_class(cx, [&](auto& c) {
                    c.queue.erase(std::remove(c.queue.begin(), c.queue.end(), j), c.queue.end());
                    return 0;
                });
                cx.jobs.erase(u);
            }
            return fail(rc, msg);
        }
        tickets.push_back(t);
    }
    int first_err = GS_OK;
    for (int i = 0; i < nreq; ++i) {
        gs_result r;
        int rc = wait_job(cx, tickets[i], &r);
        if (rc < 0 && cx.jobs.count(tickets[i])) return rc;   // device failure: the context is unusable
        if (res) res[i] = r;
        if (rc < 0 && first_err == GS_OK) first_err = rc;
    }
    (void)first_err;
    return GS_OK;
}

int gs_interpolate(gs_ctx* ctx, const gs_grid* gc, const void* d_in, const gs_grid* gf, void* d_out, void* stream) {
    if (!ctx || !d_in || !d_out) return fail(GS_EINVAL, "NULL argument");
    int rc;
    if ((rc = check_grid(gc)) || (rc = check_grid(gf))) return rc;
    if (gc->dim != gf->dim) return fail(GS_EINVAL, "grids of different dimension");
    for (int a = 0; a < gc->dim; ++a)
        if (gf->n[a] < gc->n[a] || gf->L[a] != gc->L[a])
            return fail(GS_EINVAL, "the fine grid must have at least as many points per axis on the same box");
    Ctx& cx = ctx->impl;
    if (hipSetDevice(cx.device) != hipSuccess) return fail(GS_EDEVICE, "hipSetDevice failed");
    cpx<double>* tmp = nullptr;
    if (hipMalloc((void**)&tmp, sizeof(cpx<double>) * 3 * npts(gc)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GS_ENOMEM, "device allocation failed (interpolation scratch)");
    }
    hipStream_t s = (hipStream_t)stream;
    rc = interp_impl(cx, gc, (const cpx<double>*)d_in, gf, (cpx<double>*)d_out, tmp, s);
    if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = fail(GS_EDEVICE, "hipStreamSynchronize failed");
    (void)hipFree(tmp);
    return rc;
}

int gs_set_autotune(gs_ctx* ctx, int on) {
    if (!ctx) return fail(GS_EINVAL, "ctx is NULL");
    if (on != 0 && on != 1) return fail(GS_EINVAL, "autotune must be 0 or 1");
    ctx->impl.autotune = on;
    return GS_OK;
}

const char* gs_autotune_report(gs_ctx* ctx) {
    if (!ctx) {
        fail(GS_EINVAL, "ctx is NULL");
        return nullptr;
    }
    Ctx& cx = ctx->impl;
    std::string out = "[";
    bool first = true;
    each_class(cx, [&](auto& c) {
        report_class(c, out, first);
        return 0;
    });
    out += "]";
    cx.report = out;
    return cx.report.c_str();
}

int gs_kernel_timer_start(gs_ctx* ctx, int kind) {
    if (!ctx) return fail(GS_EINVAL, "ctx is NULL");
    if (kind < -1 || kind >= KK_COUNT) return fail(GS_EINVAL, "unknown kernel kind");
    TimerTotals& t = ctx->impl.timer;
    t.kind = kind;
    t.ms = 0.0;
    t.bytes = 0.0;
    t.launches = 0;
    return GS_OK;
}

int gs_kernel_timer_read(gs_ctx* ctx, double* total_ms, double* total_bytes, long long* launches) {
    if (!ctx) return fail(GS_EINVAL, "ctx is NULL");
    const TimerTotals& t = ctx->impl.timer;
    if (total_ms) *total_ms = t.ms;
    if (total_bytes) *total_bytes = t.bytes;
    if (launches) *launches = t.launches;
    return GS_OK;
}

int gs_fft(gs_ctx* ctx, const gs_grid* g, int precision, int sign, const void* d_in, void* d_out, void* stream) {
    if (!ctx || !d_in || !d_out) return fail(GS_EINVAL, "NULL argument");
    int rc = check_grid(g);
    if (rc) return rc;
    if (sign != -1 && sign != 1) return fail(GS_EINVAL, "sign must be -1 or +1");
    if (hipSetDevice(ctx->impl.device) != hipSuccess) return fail(GS_EDEVICE, "hipSetDevice failed");
    if (precision == GS_FP64)
        return fft_impl<double>(ctx->impl, g, sign, (const cpx<double>*)d_in, (cpx<double>*)d_out, (hipStream_t)stream);
    if (precision == GS_FP32)
        return fft_impl<float>(ctx->impl, g, sign, (const cpx<float>*)d_in, (cpx<float>*)d_out, (hipStream_t)stream);
    return fail(GS_EINVAL, "precision must be GS_FP64 or GS_FP32");
}

int gs_fft_noalloc(gs_ctx* ctx, const gs_grid* g, int precision, int sign, const void* d_in, void* d_out,
                   void* stream) {
    if (!ctx || !d_in || !d_out) return fail(GS_EINVAL, "NULL argument");
    int rc = check_grid(g);
    if (rc) return rc;
    if (npts(g) > NA_MAX_POINTS) return fail(GS_EINVAL, "gs_fft_noalloc: more than 2^18 points per component");
    if (sign != -1 && sign != 1) return fail(GS_EINVAL, "sign must be -1 or +1");
    if (precision != GS_FP64 && precision != GS_FP32) return fail(GS_EINVAL, "precision must be GS_FP64 or GS_FP32");
    if (hipSetDevice(ctx->impl.device) != hipSuccess) return fail(GS_EDEVICE, "hipSetDevice failed");
    if (precision == GS_FP64)
        return fft_noalloc_impl<double>(ctx->impl.device, g, sign, (const cpx<double>*)d_in, (cpx<double>*)d_out,
                                        (hipStream_t)stream);
    return fft_noalloc_impl<float>(ctx->impl.device, g, sign, (const cpx<float>*)d_in, (cpx<float>*)d_out,
                                   (hipStream_t)stream);
}

int gs_hamiltonian(gs_ctx* ctx, const gs_grid* g, const gs_trap* t, const gs_params* p, int precision,
                   const void* d_psi, void* d_hpsi, gs_result* res, void* stream) {
    if (!ctx || !d_psi || !d_hpsi || !p) return fail(GS_EINVAL, "NULL argument");
    int rc = check_grid(g);
    if (rc) return rc;
    if (hipSetDevice(ctx->impl.device) != hipSuccess) return fail(GS_EDEVICE, "hipSetDevice failed");
    if (precision == GS_FP64)
        return ham_impl<double>(ctx->impl, g, t, p, (const cpx<double>*)d_psi, (cpx<double>*)d_hpsi, res, (hipStream_t)stream);
    if (precision == GS_FP32)
        return ham_impl<float>(ctx->impl, g, t, p, (const cpx<float>*)d_psi, (cpx<float>*)d_hpsi, res, (hipStream_t)stream);
    return fail(GS_EINVAL, "precision must be GS_FP64 or GS_FP32");
}

int gs_precondition(gs_ctx* ctx, const gs_grid* g, const gs_trap* t, const gs_params* p, int precision,
                    const void* d_psi, const void* d_r, void* d_out, void* stream) {
    if (!ctx || !d_psi || !d_r || !d_out || !p) return fail(GS_EINVAL, "NULL argument");
    int rc = check_grid(g);
    if (rc) return rc;
    if (hipSetDevice(ctx->impl.device) != hipSuccess) return fail(GS_EDEVICE, "hipSetDevice failed");
    if (precision == GS_FP64)
        return pre_impl<double>(ctx->impl, g, t, p, (const cpx<double>*)d_psi, (const cpx<double>*)d_r,
                                (cpx<double>*)d_out, (hipStream_t)stream);
    if (precision == GS_FP32)
        return pre_impl<float>(ctx->impl, g, t, p, (const cpx<float>*)d_psi, (const cpx<float>*)d_r,
                               (cpx<float>*)d_out, (hipStream_t)stream);
    return fail(GS_EINVAL, "precision must be GS_FP64 or GS_FP32");
}

}  // extern "C"
