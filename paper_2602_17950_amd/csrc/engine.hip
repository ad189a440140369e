// Host side of the gfx950 ground-state library: per-grid plans (device
// buffers and twiddle tables), the kernel sequence of one PCG iteration, the
// solve driver (chunks of iterations between completion checks, FP32 -> FP64
// switch) and the C ABI of include/gs.h.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "gs_internal.h"
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

static bool pow2_in_range(int n) { return n >= 16 && n <= 1024 && (n & (n - 1)) == 0; }

static int check_grid(const gs_grid* g) {
    if (!g) return fail(GS_EINVAL, "grid is NULL");
    if (g->dim != 2 && g->dim != 3) return fail(GS_EINVAL, "grid.dim must be 2 or 3");
    for (int a = 0; a < g->dim; ++a) {
        if (!pow2_in_range(g->n[a])) return fail(GS_EINVAL, "grid.n[a] must be a power of two in [16, 1024]");
        if (!(g->L[a] > 0.0) || !std::isfinite(g->L[a])) return fail(GS_EINVAL, "grid.L[a] must be positive");
    }
    return GS_OK;
}

static long long npts(const gs_grid* g) {
    long long m = (long long)g->n[0] * g->n[1];
    if (g->dim == 3) m *= g->n[2];
    return m;
}

// Scratch of the FFT chains: two six-component buffers (P^ and Phi transformed
// together) and four single fields.
constexpr int SCRATCH_FIELDS = 8;

// rows of per-block partial sums: the pointwise grid and the preconditioner's
// last pass (3 * Nz * Ny / TILE blocks with TILE >= 2)
static long long pw_rows(const gs_grid* g) {
    const long long M = npts(g);
    const long long pre = 3LL * M / g->n[0] / 2;
    return std::max<long long>(pw_blocks(M), pre);
}
static long long mid_rows(const gs_grid* g) {
    const int Nlast = g->n[g->dim - 1];
    return mid_blocks(Nlast, (int)(npts(g) / Nlast));
}

template <typename R> static size_t plan_bytes(const gs_grid* g) {
    const long long M = npts(g);
    const size_t field = (size_t)3 * M * sizeof(cpx<R>);
    return field * (8 + SCRATCH_FIELDS) + (size_t)3 * M * sizeof(R) +
           (size_t)(pw_rows(g) * NS_MAX + mid_rows(g) * RED_MID_STRIDE) * sizeof(double);
}

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
template <typename R>
struct Plan {
    int dim = 0, n[3] = {1, 1, 1};
    long long M = 0;
    std::vector<void*> allocs;
    Fields<R> f{};
    cpx<R>* t6[2] = {};   // [6][M] each
    cpx<R>* t[4] = {};    // [3][M] each
    const cpx<R>* tw[3] = {};
    double* red_mid = nullptr;
    double* red_pw = nullptr;
    int nblk_mid = 0;
    ~Plan() {
        for (void* p : allocs) (void)hipFree(p);
    }
};

// Optional per-kernel timer: every launch of one kernel kind of the iteration
// records its own start and end (dispatch timestamps, hipExtLaunchKernelGGL)
// into HIP events on the solve's stream; the elapsed times and the kernel's
// algorithmic bytes (each distinct array read or written once) are summed. Launches that return at once because the solve has finished (the
// tail of the last chunk) are left out.
enum KKind : int {
    KK_HL_FWD = 0, KK_HL_MID = 1, KK_HL_INV = 2, KK_PRE_FWD = 3, KK_PRE_MID = 4, KK_PRE_INV = 5,
    KK_EVAL = 6, KK_RESID = 7, KK_DIRRED = 8, KK_LSRED = 9, KK_HL_FWD2 = 10, KK_HL_INV2 = 11,
    KK_COUNT = 12
};
struct Timer {
    int kind = -1;
    struct Rec { int k, chain; double bytes; };
    std::vector<hipEvent_t> ev;
    std::vector<Rec> rec;
    int iter_in_chunk = 0;
    int chain = 0;
    double ms = 0.0, bytes = 0.0;
    long long launches = 0;
    ~Timer() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

template <typename F>
static hipError_t timed(Timer* tm, int kind, double bytes, hipStream_t s, F&& f) {
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
    tm->rec.push_back({tm->iter_in_chunk, tm->chain, bytes});
    return e;
}

// After a chunk has completed: n_full iterations ran to the end; when the solve
// finished in the chunk, the refresh (chain 0) and the residual pass (chain 1)
// of iteration n_full also ran.
static hipError_t timer_collect(Timer* tm, int n_full, bool done) {
    if (!tm) return hipSuccess;
    for (size_t i = 0; i < tm->rec.size(); ++i) {
        const Timer::Rec& r = tm->rec[i];
        if (!(r.k < n_full || (done && r.k == n_full && r.chain <= 1))) continue;
        float ms = 0.0f;
        hipError_t e = hipEventElapsedTime(&ms, tm->ev[2 * i], tm->ev[2 * i + 1]);
        if (e != hipSuccess) return e;
        tm->ms += ms;
        tm->bytes += r.bytes;
        tm->launches++;
    }
    tm->rec.clear();
    return hipSuccess;
}

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::map<std::tuple<int, int, int, int>, std::unique_ptr<Plan<double>>> p64;
    std::map<std::tuple<int, int, int, int>, std::unique_ptr<Plan<float>>> p32;
    std::map<std::pair<int, int>, void*> twiddles;   // (N, sizeof(R)) -> table
    SolveState* st = nullptr;       // device
    SolveState* st_host = nullptr;  // pinned host mirror
    unsigned* counters = nullptr;
    double* Vdev = nullptr;
    size_t Vbytes = 0;
    std::vector<void*> allocs;
    Timer timer;
    ~Ctx() {
        (void)hipSetDevice(device);
        p64.clear();
        p32.clear();
        for (auto& kv : twiddles) (void)hipFree(kv.second);
        for (void* p : allocs) (void)hipFree(p);
        if (Vdev) (void)hipFree(Vdev);
        if (st_host) (void)hipHostFree(st_host);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

template <typename R>
static int get_twiddle(Ctx& cx, int N, const cpx<R>** out) {
    auto key = std::make_pair(N, (int)sizeof(R));
    auto it = cx.twiddles.find(key);
    if (it != cx.twiddles.end()) {
        *out = (const cpx<R>*)it->second;
        return GS_OK;
    }
    std::vector<cpx<R>> h(N);
    for (int m = 0; m < N; ++m) {
        const long double ang = 2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)N;
        h[m] = cpx<R>{(R)cosl(ang), (R)(-sinl(ang))};
    }
    void* d = nullptr;
    if (hipMalloc(&d, sizeof(cpx<R>) * N) != hipSuccess) return fail(GS_ENOMEM, "twiddle table allocation failed");
    HIPCHK(hipMemcpy(d, h.data(), sizeof(cpx<R>) * N, hipMemcpyHostToDevice));
    cx.twiddles[key] = d;
    *out = (const cpx<R>*)d;
    return GS_OK;
}

template <typename R> static auto& plans(Ctx& cx);
template <> auto& plans<double>(Ctx& cx) { return cx.p64; }
template <> auto& plans<float>(Ctx& cx) { return cx.p32; }

template <typename R>
static int get_plan(Ctx& cx, const gs_grid* g, Plan<R>** out) {
    auto key = std::make_tuple(g->dim, g->n[0], g->n[1], g->dim == 3 ? g->n[2] : 1);
    auto& mp = plans<R>(cx);
    auto it = mp.find(key);
    if (it != mp.end()) {
        *out = it->second.get();
        return GS_OK;
    }
    auto pl = std::make_unique<Plan<R>>();
    pl->dim = g->dim;
    pl->n[0] = g->n[0];
    pl->n[1] = g->n[1];
    pl->n[2] = g->dim == 3 ? g->n[2] : 1;
    pl->M = npts(g);
    const size_t field = (size_t)3 * pl->M * sizeof(cpx<R>);
    auto alloc = [&](size_t bytes, void** p) -> bool {
        if (hipMalloc(p, bytes) != hipSuccess) return false;
        pl->allocs.push_back(*p);
        return hipMemset(*p, 0, bytes) == hipSuccess;
    };
    void* p = nullptr;
    cpx<R>** fl[] = {&pl->f.phi, &pl->f.hl, &pl->f.r[0], &pl->f.r[1], &pl->f.pr, &pl->f.P, &pl->f.hlp, &pl->f.u};
    for (auto* q : fl) {
        if (!alloc(field, &p)) return fail(GS_ENOMEM, "device allocation failed (fields)");
        *q = (cpx<R>*)p;
    }
    if (!alloc((size_t)3 * pl->M * sizeof(R), &p)) return fail(GS_ENOMEM, "device allocation failed (pv)");
    pl->f.pv = (R*)p;
    for (int k = 0; k < 2; ++k) {
        if (!alloc(2 * field, &p)) return fail(GS_ENOMEM, "device allocation failed (scratch)");
        pl->t6[k] = (cpx<R>*)p;
    }
    for (int k = 0; k < 4; ++k) {
        if (!alloc(field, &p)) return fail(GS_ENOMEM, "device allocation failed (scratch)");
        pl->t[k] = (cpx<R>*)p;
    }
    // the middle pass runs along the last axis; its lines are the other points
    pl->nblk_mid = (int)mid_rows(g);
    if (!alloc((size_t)pl->nblk_mid * RED_MID_STRIDE * sizeof(double), &p)) return fail(GS_ENOMEM, "device allocation failed (reductions)");
    pl->red_mid = (double*)p;
    if (!alloc((size_t)pw_rows(g) * NS_MAX * sizeof(double), &p)) return fail(GS_ENOMEM, "device allocation failed (reductions)");
    pl->red_pw = (double*)p;
    for (int a = 0; a < g->dim; ++a) {
        int rc = get_twiddle<R>(cx, pl->n[a], &pl->tw[a]);
        if (rc) return rc;
    }
    *out = pl.get();
    mp[key] = std::move(pl);
    return GS_OK;
}

static int make_phys(Ctx& cx, const gs_grid* g, const gs_trap* t, const gs_params* p, Phys* ph) {
    std::memset(ph, 0, sizeof(*ph));
    ph->dim = g->dim;
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
        ph->omega = p->omega;
        ph->gamma = p->gamma;
        ph->c0 = p->c0;
        ph->c1 = p->c1;
        if (!std::isfinite(p->omega) || !std::isfinite(p->gamma) || !std::isfinite(p->c0) || !std::isfinite(p->c1))
            return fail(GS_EINVAL, "params must be finite");
    }
    if (t) {
        for (int a = 0; a < 3; ++a) ph->hg[a] = a < g->dim ? 0.5 * t->g[a] * t->g[a] : 0.0;
        ph->q2 = t->q2;
        ph->q4 = t->q4;
        if (t->V) {
            const size_t bytes = sizeof(double) * ph->M;
            for (long long i = 0; i < ph->M; ++i)
                if (!std::isfinite(t->V[i])) return fail(GS_EINVAL, "trap.V must be finite");
            if (cx.Vbytes < bytes) {
                if (cx.Vdev) (void)hipFree(cx.Vdev);
                cx.Vdev = nullptr;
                cx.Vbytes = 0;
                if (hipMalloc(&cx.Vdev, bytes) != hipSuccess) return fail(GS_ENOMEM, "device allocation failed (V)");
                cx.Vbytes = bytes;
            }
            HIPCHK(hipMemcpy(cx.Vdev, t->V, bytes, hipMemcpyHostToDevice));
            ph->V = cx.Vdev;
        }
    } else {
        ph->hg[0] = ph->hg[1] = 0.5;
        ph->hg[2] = g->dim == 3 ? 0.5 : 0.0;
    }
    return GS_OK;
}

template <typename R>
static RedBuf redbuf(Ctx& cx, const Plan<R>& pl) {
    RedBuf rb;
    rb.mid = pl.red_mid;
    rb.pw = pl.red_pw;
    rb.counter = cx.counters;
    rb.nblk_mid = pl.nblk_mid;
    rb.nblk_pw = pw_blocks(pl.M);
    return rb;
}

// ---------------------------------------------------------------------------
// operator chains
// ---------------------------------------------------------------------------
// out = H_L in  (H_L = -1/2 Lap + V - Omega L_z - gamma S), with the prologue
// `pro` applied to `in` first (see launch_fwdT). dual (with PRO_DIR): aux1 (Phi)
// is transformed with in, and the middle pass reduces the kinetic coefficients
// of both for the next iterate's alpha_l.
template <typename R>
static hipError_t chain_HL(Plan<R>& pl, const Phys& ph, int pro, int dual, cpx<R>* in, cpx<R>* out,
                           const cpx<R>* aux0, const cpx<R>* aux1, int use_invnP,
                           const SolveState* st, hipStream_t s, Timer* tm = nullptr) {
    const int rot = ph.omega != 0.0;
    const int Nx = pl.n[0], Ny = pl.n[1], Nz = pl.n[2];
    const long long M3 = 3 * pl.M;
    const double F = 3.0 * pl.M * sizeof(cpx<R>);
    const double b_fwd = dual ? 6 * F : (pro == PRO_DIR ? 5 * F : (pro == PRO_UPDATE ? 4 * F : 2 * F));
    const double b_mid = (rot ? 2 : 1) * F + (dual ? 2 : 1) * F, b_inv = (rot ? 4 : 3) * F;
    const int midop = dual ? MID_HLX : MID_HL;
    cpx<R>* S0 = pl.t6[0];
    cpx<R>* S1 = pl.t6[1];
    hipError_t e;
    if (pl.dim == 2) {
        if ((e = timed(tm, KK_HL_FWD, b_fwd, s, [&] { return launch_fwdT<R>(Nx, pro, dual, in, S0, 1, Ny, 3, aux0, aux1, st, pl.tw[0], s); }))) return e;
        if ((e = timed(tm, KK_HL_MID, b_mid, s, [&] { return launch_mid<R>(Ny, midop, rot, S0, S0 + M3, pl.t[0], pl.t[1], Nx, ph, st, pl.red_mid, pl.tw[1], s); }))) return e;
        return timed(tm, KK_HL_INV, b_inv, s, [&] {
            return launch_invT<R>(Nx, EPI_HL, rot ? 2 : 1, pl.t[0], pl.t[1], out, nullptr, 1, Ny, ph, in, 1.0,
                                  nullptr, st, use_invnP, pl.tw[0], s); });
    }
    const int nc = dual ? 6 : 3;
    if ((e = timed(tm, KK_HL_FWD, b_fwd, s, [&] { return launch_fwdT<R>(Nx, pro, dual, in, S0, Nz, Ny, 3, aux0, aux1, st, pl.tw[0], s); }))) return e;
    if ((e = timed(tm, KK_HL_FWD2, 2 * (nc / 3) * F, s, [&] { return launch_fwdT<R>(Ny, PRO_PLAIN, 0, S0, S1, Nx, Nz, nc, nullptr, nullptr, st, pl.tw[1], s); }))) return e;
    if ((e = timed(tm, KK_HL_MID, b_mid, s, [&] { return launch_mid<R>(Nz, midop, rot, S1, S1 + M3, pl.t[0], pl.t[1], Ny * Nx, ph, st, pl.red_mid, pl.tw[2], s); }))) return e;
    if ((e = timed(tm, KK_HL_INV2, (rot ? 5 : 2) * F, s, [&] {
             return launch_invT<R>(Ny, rot ? EPI_ROTX : EPI_SCALE, rot ? 2 : 1, pl.t[0], pl.t[1], pl.t[2], pl.t[3], Nx, Nz,
                                   ph, S0, 1.0, nullptr, st, 0, pl.tw[1], s); }))) return e;
    return timed(tm, KK_HL_INV, b_inv, s, [&] {
        return launch_invT<R>(Nx, EPI_HL, rot ? 2 : 1, pl.t[2], pl.t[3], out, nullptr, Nz, Ny, ph, in, 1.0, nullptr,
                              st, use_invnP, pl.tw[0], s); });
}

// pr = P_V^{1/2} P_Delta P_V^{1/2} r (the first factor is already applied: input in f.u);
// dir = 1 fuses the direction reductions and control into the last pass
template <typename R>
static hipError_t chain_pre(Plan<R>& pl, const Phys& ph, SolveState* st, RedBuf rb, int dir, hipStream_t s,
                            Timer* tm = nullptr) {
    const int Nx = pl.n[0], Ny = pl.n[1], Nz = pl.n[2];
    const double F = 3.0 * pl.M * sizeof(cpx<R>), Fr = 3.0 * pl.M * sizeof(R);
    const double b_inv = (dir ? 6 : 2) * F + Fr;
    cpx<R>* S0 = pl.t6[0];
    cpx<R>* S1 = pl.t6[1];
    hipError_t e;
    if (pl.dim == 2) {
        if ((e = timed(tm, KK_PRE_FWD, 2 * F, s, [&] { return launch_fwdT<R>(Nx, PRO_PLAIN, 0, pl.f.u, S0, 1, Ny, 3, nullptr, nullptr, st, pl.tw[0], s); }))) return e;
        if ((e = timed(tm, KK_PRE_MID, 2 * F, s, [&] { return launch_mid<R>(Ny, MID_PRE, 0, S0, nullptr, pl.t[0], nullptr, Nx, ph, st, nullptr, pl.tw[1], s); }))) return e;
        return timed(tm, KK_PRE_INV, b_inv, s, [&] {
            return launch_invT_pre<R>(Nx, pl.t[0], pl.f.pr, 1, Ny, pl.f.pv, pl.f, ph, st, rb, dir, pl.tw[0], s); });
    }
    if ((e = timed(tm, KK_PRE_FWD, 2 * F, s, [&] { return launch_fwdT<R>(Nx, PRO_PLAIN, 0, pl.f.u, S0, Nz, Ny, 3, nullptr, nullptr, st, pl.tw[0], s); }))) return e;
    if ((e = launch_fwdT<R>(Ny, PRO_PLAIN, 0, S0, S1, Nx, Nz, 3, nullptr, nullptr, st, pl.tw[1], s))) return e;
    if ((e = timed(tm, KK_PRE_MID, 2 * F, s, [&] { return launch_mid<R>(Nz, MID_PRE, 0, S1, nullptr, pl.t[0], nullptr, Ny * Nx, ph, st, nullptr, pl.tw[2], s); }))) return e;
    if ((e = launch_invT<R>(Ny, EPI_SCALE, 1, pl.t[0], nullptr, pl.t[1], nullptr, Nx, Nz, ph, nullptr, 1.0, nullptr,
                            st, 0, pl.tw[1], s))) return e;
    return timed(tm, KK_PRE_INV, b_inv, s, [&] {
        return launch_invT_pre<R>(Nx, pl.t[1], pl.f.pr, Nz, Ny, pl.f.pv, pl.f, ph, st, rb, dir, pl.tw[0], s); });
}

// Fresh evaluation of the current iterate: apply a pending update to Phi,
// H_L Phi from scratch, energy parts, mu, alpha_l.
template <typename R>
static hipError_t refresh(Plan<R>& pl, const Phys& ph, SolveState* st, RedBuf rb, int force, hipStream_t s, Timer* tm) {
    const double F = 3.0 * pl.M * sizeof(cpx<R>);
    hipError_t e;
    if ((e = chain_HL<R>(pl, ph, PRO_UPDATE, 0, pl.f.phi, pl.f.hl, pl.f.P, nullptr, 0, st, s, tm))) return e;
    return timed(tm, KK_EVAL, 2 * F, s, [&] { return launch_eval<R>(pl.f, ph, st, rb, force, s); });
}

// One PCG iteration (Algorithm 1 with Algorithm 2), entirely on the device:
//   0. (first iteration of a chunk) fresh H_L Phi, E, mu, alpha_l
//   1. pending update Phi <- (c Phi + s P^)/|.|, H_L Phi by the same combination;
//      r = H(Phi)Phi - mu Phi, P_V^{1/2} factors, stopping tests
//   2. preconditioned residual (3 or 5 FFT passes) with the PRP beta,
//      projection and descent test fused into its last pass
//   3. P^n = D - Re<D,Phi> Phi, H_L P^ (3 or 5 FFT passes; Phi transformed
//      alongside for the kinetic coefficients)
//   4. energy along the retraction, step size, backtracking, and the scalars
//      (mu, E, alpha_l) of the next iterate
template <typename R>
static hipError_t iterate(Plan<R>& pl, const Phys& ph, SolveState* st, RedBuf rb, int do_refresh, hipStream_t s,
                          Timer* tm) {
    const double F = 3.0 * pl.M * sizeof(cpx<R>), Fr = 3.0 * pl.M * sizeof(R);
    hipError_t e;
    if (do_refresh) {
        if (tm) tm->chain = 0;
        if ((e = refresh<R>(pl, ph, st, rb, 0, s, tm))) return e;
    }
    if (tm) tm->chain = 1;
    if ((e = timed(tm, KK_RESID, 8 * F + Fr, s, [&] { return launch_resid<R>(pl.f, ph, st, rb, 0, s); }))) return e;
    if (tm) tm->chain = 2;
    if ((e = chain_pre<R>(pl, ph, st, rb, 1, s, tm))) return e;
    if (tm) tm->chain = 3;
    if ((e = chain_HL<R>(pl, ph, PRO_DIR, 1, pl.f.P, pl.f.hlp, pl.f.pr, pl.f.phi, 1, st, s, tm))) return e;
    return timed(tm, KK_LSRED, 4 * F, s, [&] { return launch_lsred<R>(pl.f, ph, st, rb, s); });
}

// ---------------------------------------------------------------------------
// solve driver
// ---------------------------------------------------------------------------
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
    h->phase = phase;
    h->best_resid = INFINITY;
    h->inv_norm = 1.0;
    h->c = 1.0;
}

static int check_options(const gs_options* o) {
    if (!o) return fail(GS_EINVAL, "options is NULL");
    if (o->stop_kind < 0 || o->stop_kind > 2) return fail(GS_EINVAL, "options.stop_kind invalid");
    if (!(o->tol >= 0.0)) return fail(GS_EINVAL, "options.tol must be >= 0");
    if (o->max_iter < 0) return fail(GS_EINVAL, "options.max_iter must be >= 0");
    if (o->precision < GS_FP64 || o->precision > GS_MIXED) return fail(GS_EINVAL, "options.precision invalid");
    if (!(o->sigma > 0.0 && o->sigma < 1.0)) return fail(GS_EINVAL, "options.sigma must be in (0, 1)");
    if (!(o->theta_trial > 0.0)) return fail(GS_EINVAL, "options.theta_trial must be positive");
    if (o->max_backtrack < 0) return fail(GS_EINVAL, "options.max_backtrack must be >= 0");
    if (o->check_every < 1) return fail(GS_EINVAL, "options.check_every must be >= 1");
    return GS_OK;
}

// Iterate one precision phase to its end. Chunks of check_every iterations are
// enqueued between host checks; each chunk starts with a fresh evaluation of
// H_L Phi and the scalars, which also bounds the rounding drift of the
// H_L Phi recurrence. Unless the phase ends in a precision switch, a final
// fresh evaluation fills E, its parts, mu, mu_l and the residual of the result.
template <typename R>
static int run_phase(Ctx& cx, Plan<R>& pl, const Phys& ph, int check_every, hipStream_t s) {
    RedBuf rb = redbuf(cx, pl);
    HIPCHK(launch_normalize<R>(pl.f.phi, ph, cx.st, rb, s));
    Timer* tm = cx.timer.kind >= 0 ? &cx.timer : nullptr;
    int last_iter = -1;
    for (;;) {
        const int iter0 = cx.st_host->iter;
        for (int k = 0; k < check_every; ++k) {
            if (tm) tm->iter_in_chunk = k;
            HIPCHK(iterate<R>(pl, ph, cx.st, rb, k == 0, s, tm));
        }
        HIPCHK(hipMemcpyAsync(cx.st_host, cx.st, sizeof(SolveState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        HIPCHK(timer_collect(tm, cx.st_host->iter - iter0, cx.st_host->done != 0));
        if (cx.st_host->done) break;
        // every iteration either accepts a step or ends the solve
        if (cx.st_host->iter == last_iter) return fail(GS_EDEVICE, "solver made no progress (device state not updated)");
        last_iter = cx.st_host->iter;
    }
    if (!cx.st_host->switch_req) {
        // the kernels run while done == 0; restore the flag afterwards
        static const int zero = 0;
        HIPCHK(hipMemcpyAsync(&cx.st->done, &zero, sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(refresh<R>(pl, ph, cx.st, rb, 1, s, nullptr));
        HIPCHK(launch_resid<R>(pl.f, ph, cx.st, rb, 1, s));
        HIPCHK(hipMemcpyAsync(cx.st_host, cx.st, sizeof(SolveState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        cx.st_host->done = 1;
    }
    return GS_OK;
}

static void fill_result(const SolveState* h, gs_result* r, int iters_fp32, double wall) {
    if (!r) return;
    std::memset(r, 0, sizeof(*r));
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
    r->iters_fp32 = iters_fp32;
    r->backtracks = h->backtracks;
    r->resets = h->resets;
    r->status = h->status;
    r->wall_s = wall;
}

static int solve_impl(Ctx& cx, const gs_grid* g, const gs_trap* t, const gs_params* p, const gs_options* o,
                      const cpx<double>* d_psi0, cpx<double>* d_out, gs_result* res, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    int rc;
    if ((rc = check_grid(g))) return rc;
    if ((rc = check_options(o))) return rc;
    if (!p) return fail(GS_EINVAL, "params is NULL");
    HIPCHK(hipSetDevice(cx.device));
    Phys ph;
    if ((rc = make_phys(cx, g, t, p, &ph))) return rc;
    const long long n3 = 3 * ph.M;
    Plan<double>* p64 = nullptr;
    Plan<float>* p32 = nullptr;
    const bool use32 = o->precision != GS_FP64;
    const bool use64 = o->precision != GS_FP32;
    if (use64 && (rc = get_plan<double>(cx, g, &p64))) return rc;
    if (use32 && (rc = get_plan<float>(cx, g, &p32))) return rc;

    // initial guess into the first phase's Phi (the Gaussian guess is built in
    // double, then rounded when the first phase is in float)
    void* tmp = nullptr;
    const cpx<double>* guess = d_psi0;
    if (!guess) {
        cpx<double>* dst = use64 ? p64->f.phi : nullptr;
        if (!dst) {
            if (hipMalloc(&tmp, sizeof(cpx<double>) * n3) != hipSuccess) return fail(GS_ENOMEM, "device allocation failed (guess)");
            dst = (cpx<double>*)tmp;
        }
        HIPCHK(launch_gaussian(dst, ph, s));
        guess = dst;
    }
    if (use32) HIPCHK(launch_convert_d2f(guess, p32->f.phi, n3, s));
    else if (guess != p64->f.phi)
        HIPCHK(hipMemcpyAsync(p64->f.phi, guess, sizeof(cpx<double>) * n3, hipMemcpyDeviceToDevice, s));
    if (tmp) {
        HIPCHK(hipStreamSynchronize(s));
        (void)hipFree(tmp);
    }

    const int phase0 = o->precision == GS_MIXED ? PH_FP32 : PH_FP64;
    init_state(cx.st_host, o, phase0);
    HIPCHK(hipMemcpyAsync(cx.st, cx.st_host, sizeof(SolveState), hipMemcpyHostToDevice, s));
    int iters_fp32 = 0;
    bool out_from_32 = false;
    if (use32) {
        HIPCHK(hipMemsetAsync(p32->f.P, 0, sizeof(cpx<float>) * n3, s));
        if ((rc = run_phase<float>(cx, *p32, ph, o->check_every, s))) return rc;
        iters_fp32 = cx.st_host->iter;
        out_from_32 = true;
        if (o->precision == GS_MIXED && cx.st_host->switch_req && !cx.st_host->nonfinite) {
            // warm start of the double phase from the float iterate, beta reset to 0
            HIPCHK(launch_convert_f2d(p32->f.phi, p64->f.phi, n3, s));
            SolveState* h = cx.st_host;
            h->done = 0;
            h->switch_req = 0;
            h->phase = PH_FP64;
            h->have_prev = 0;
            h->pending_step = 0;
            h->final_pending = 0;
            h->iter_phase = 0;
            h->status = GS_OK;
            HIPCHK(hipMemcpyAsync(cx.st, h, sizeof(SolveState), hipMemcpyHostToDevice, s));
            out_from_32 = false;
        }
    }
    if (use64 && !out_from_32) {
        HIPCHK(hipMemsetAsync(p64->f.P, 0, sizeof(cpx<double>) * n3, s));
        if ((rc = run_phase<double>(cx, *p64, ph, o->check_every, s))) return rc;
    }
    const SolveState* h = cx.st_host;
    if (h->nonfinite) {
        const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        fill_result(h, res, iters_fp32, wall);
        return fail(GS_ENONFINITE, "non-finite value in the iteration (check the input and parameters)");
    }
    if (out_from_32) HIPCHK(launch_convert_f2d(p32->f.phi, d_out, n3, s));
    else HIPCHK(hipMemcpyAsync(d_out, p64->f.phi, sizeof(cpx<double>) * n3, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_result(h, res, iters_fp32, wall);
    return h->status;
}

// ---------------------------------------------------------------------------
// operator-level entry points
// ---------------------------------------------------------------------------
template <typename R>
static int fft_impl(Ctx& cx, const gs_grid* g, int sign, const cpx<R>* in, cpx<R>* out, hipStream_t s) {
    Plan<R>* pl;
    int rc;
    if ((rc = get_plan<R>(cx, g, &pl))) return rc;
    Phys ph;
    if ((rc = make_phys(cx, g, nullptr, nullptr, &ph))) return rc;
    const int Nx = pl->n[0], Ny = pl->n[1], Nz = pl->n[2];
    const double invM = 1.0 / (double)pl->M;
    cpx<R>* inw = const_cast<cpx<R>*>(in);
    if (sign < 0) {
        if (g->dim == 2) {
            HIPCHK(launch_fwdT<R>(Nx, PRO_PLAIN, 0, inw, pl->t[0], 1, Ny, 3, nullptr, nullptr, nullptr, pl->tw[0], s));
            HIPCHK(launch_fwdT<R>(Ny, PRO_PLAIN, 0, pl->t[0], out, 1, Nx, 3, nullptr, nullptr, nullptr, pl->tw[1], s));
        } else {
            HIPCHK(launch_fwdT<R>(Nx, PRO_PLAIN, 0, inw, pl->t[0], Nz, Ny, 3, nullptr, nullptr, nullptr, pl->tw[0], s));
            HIPCHK(launch_fwdT<R>(Ny, PRO_PLAIN, 0, pl->t[0], pl->t[1], Nx, Nz, 3, nullptr, nullptr, nullptr, pl->tw[1], s));
            HIPCHK(launch_fwdT<R>(Nz, PRO_PLAIN, 0, pl->t[1], out, Ny, Nx, 3, nullptr, nullptr, nullptr, pl->tw[2], s));
        }
    } else {
        if (g->dim == 2) {
            HIPCHK(launch_invT<R>(Ny, EPI_SCALE, 1, in, nullptr, pl->t[0], nullptr, 1, Nx, ph, nullptr, 1.0, nullptr, nullptr, 0, pl->tw[1], s));
            HIPCHK(launch_invT<R>(Nx, EPI_SCALE, 1, pl->t[0], nullptr, out, nullptr, 1, Ny, ph, nullptr, invM, nullptr, nullptr, 0, pl->tw[0], s));
        } else {
            HIPCHK(launch_invT<R>(Nz, EPI_SCALE, 1, in, nullptr, pl->t[0], nullptr, Ny, Nx, ph, nullptr, 1.0, nullptr, nullptr, 0, pl->tw[2], s));
            HIPCHK(launch_invT<R>(Ny, EPI_SCALE, 1, pl->t[0], nullptr, pl->t[1], nullptr, Nx, Nz, ph, nullptr, 1.0, nullptr, nullptr, 0, pl->tw[1], s));
            HIPCHK(launch_invT<R>(Nx, EPI_SCALE, 1, pl->t[1], nullptr, out, nullptr, Nz, Ny, ph, nullptr, invM, nullptr, nullptr, 0, pl->tw[0], s));
        }
    }
    return GS_OK;
}

// state for a single evaluation (no iteration)
static SolveState* eval_state(Ctx& cx, hipStream_t s, int* rc) {
    gs_options o;
    gs_default_options(&o);
    o.max_iter = 1 << 30;
    init_state(cx.st_host, &o, PH_FP64);
    hipError_t e = hipMemcpyAsync(cx.st, cx.st_host, sizeof(SolveState), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // the pinned mirror is reused by the next call
    *rc = e == hipSuccess ? GS_OK : fail(GS_EDEVICE, hipGetErrorString(e));
    return cx.st;
}

template <typename R>
static int ham_impl(Ctx& cx, const gs_grid* g, const gs_trap* t, const gs_params* p, const cpx<R>* psi,
                    cpx<R>* hpsi, gs_result* res, hipStream_t s) {
    Plan<R>* pl;
    int rc;
    if ((rc = get_plan<R>(cx, g, &pl))) return rc;
    Phys ph;
    if ((rc = make_phys(cx, g, t, p, &ph))) return rc;
    const long long n3 = 3 * ph.M;
    SolveState* st = eval_state(cx, s, &rc);
    if (rc) return rc;
    RedBuf rb = redbuf(cx, *pl);
    HIPCHK(hipMemcpyAsync(pl->f.phi, psi, sizeof(cpx<R>) * n3, hipMemcpyDeviceToDevice, s));
    HIPCHK(refresh<R>(*pl, ph, st, rb, 1, s, nullptr));
    HIPCHK(launch_resid<R>(pl->f, ph, st, rb, 1, s));
    HIPCHK(launch_hphi<R>(pl->f.phi, pl->f.hl, hpsi, ph, s));
    if (res) {
        HIPCHK(hipMemcpyAsync(cx.st_host, st, sizeof(SolveState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        fill_result(cx.st_host, res, 0, 0.0);
        res->status = GS_OK;
    }
    return GS_OK;
}

template <typename R>
static int pre_impl(Ctx& cx, const gs_grid* g, const gs_trap* t, const gs_params* p, const cpx<R>* psi,
                    const cpx<R>* r, cpx<R>* out, hipStream_t s) {
    Plan<R>* pl;
    int rc;
    if ((rc = get_plan<R>(cx, g, &pl))) return rc;
    Phys ph;
    if ((rc = make_phys(cx, g, t, p, &ph))) return rc;
    const long long n3 = 3 * ph.M;
    SolveState* st = eval_state(cx, s, &rc);
    if (rc) return rc;
    RedBuf rb = redbuf(cx, *pl);
    HIPCHK(hipMemcpyAsync(pl->f.phi, psi, sizeof(cpx<R>) * n3, hipMemcpyDeviceToDevice, s));
    HIPCHK(refresh<R>(*pl, ph, st, rb, 1, s, nullptr));
    HIPCHK(launch_pvin<R>(pl->f.phi, r, pl->f.pv, pl->f.u, ph, st, s));
    HIPCHK(chain_pre<R>(*pl, ph, st, rb, 0, s));
    HIPCHK(hipMemcpyAsync(out, pl->f.pr, sizeof(cpx<R>) * n3, hipMemcpyDeviceToDevice, s));
    return GS_OK;
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
}

size_t gs_footprint_bytes(const gs_grid* g, int precision) {
    if (check_grid(g) != GS_OK) return 0;
    switch (precision) {
    case GS_FP64: return plan_bytes<double>(g);
    case GS_FP32: return plan_bytes<float>(g);
    case GS_MIXED: return plan_bytes<double>(g) + plan_bytes<float>(g);
    default: return 0;
    }
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
    if (hipStreamCreate(&cx.stream) != hipSuccess) return fail(GS_EDEVICE, "hipStreamCreate failed");
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(SolveState)) != hipSuccess) return fail(GS_ENOMEM, "state allocation failed");
    cx.allocs.push_back(p);
    cx.st = (SolveState*)p;
    if (hipHostMalloc((void**)&cx.st_host, sizeof(SolveState), hipHostMallocDefault) != hipSuccess)
        return fail(GS_ENOMEM, "pinned allocation failed");
    if (hipMalloc(&p, 16 * sizeof(unsigned)) != hipSuccess) return fail(GS_ENOMEM, "counter allocation failed");
    cx.allocs.push_back(p);
    cx.counters = (unsigned*)p;
    if (hipMemset(cx.counters, 0, 16 * sizeof(unsigned)) != hipSuccess) return fail(GS_EDEVICE, "hipMemset failed");
    *out = c.release();
    return GS_OK;
}

void gs_destroy(gs_ctx* ctx) { delete ctx; }

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
    if (hipMalloc(&dout, bytes) != hipSuccess) return fail(GS_ENOMEM, "device allocation failed (psi)");
    if (psi0 && hipMalloc(&din, bytes) != hipSuccess) {
        (void)hipFree(dout);
        return fail(GS_ENOMEM, "device allocation failed (psi0)");
    }
    if (psi0 && hipMemcpy(din, psi0, bytes, hipMemcpyHostToDevice) != hipSuccess) rc = fail(GS_EDEVICE, "copy of psi0 failed");
    if (!rc) rc = solve_impl(cx, g, t, p, o, (const cpx<double>*)din, (cpx<double>*)dout, res, cx.stream);
    if (rc >= 0 && hipMemcpy(psi_out, dout, bytes, hipMemcpyDeviceToHost) != hipSuccess) rc = fail(GS_EDEVICE, "copy of psi failed");
    if (din) (void)hipFree(din);
    (void)hipFree(dout);
    return rc;
}

int gs_solve_device(gs_ctx* ctx, const gs_grid* g, const gs_trap* t, const gs_params* p, const gs_options* o,
                    const void* d_psi0, void* d_psi_out, gs_result* res, void* stream) {
    if (!ctx) return fail(GS_EINVAL, "ctx is NULL");
    if (!d_psi_out) return fail(GS_EINVAL, "d_psi_out is NULL");
    return solve_impl(ctx->impl, g, t, p, o, (const cpx<double>*)d_psi0, (cpx<double>*)d_psi_out, res,
                      (hipStream_t)stream);
}

int gs_kernel_timer_start(gs_ctx* ctx, int kind) {
    if (!ctx) return fail(GS_EINVAL, "ctx is NULL");
    if (kind < -1 || kind >= KK_COUNT) return fail(GS_EINVAL, "unknown kernel kind");
    Timer& t = ctx->impl.timer;
    t.kind = kind;
    t.rec.clear();
    t.ms = 0.0;
    t.bytes = 0.0;
    t.launches = 0;
    return GS_OK;
}

int gs_kernel_timer_read(gs_ctx* ctx, double* total_ms, double* total_bytes, long long* launches) {
    if (!ctx) return fail(GS_EINVAL, "ctx is NULL");
    const Timer& t = ctx->impl.timer;
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
