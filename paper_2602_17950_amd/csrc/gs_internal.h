// Internal declarations of the gfx950 ground-state library: complex helpers,
// the problem description handed to kernels, the device-resident solver state,
// the per-solve slot descriptors and the launch entry points of the kernel
// translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstddef>
#include <cstdint>

namespace gs {

// Events into which the next kernel launch on this thread writes its own
// start and end timestamps (used by the per-kernel timer); consumed by that
// launch. Every kernel of the library is launched through GS_LAUNCH.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
LaunchEvents& launch_events();

#define GS_LAUNCH(KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)                                          \
    do {                                                                                            \
        gs::LaunchEvents& le_ = gs::launch_events();                                                \
        if (le_.start) {                                                                            \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, le_.start, le_.stop, 0u,      \
                                  __VA_ARGS__);                                                     \
            le_.start = le_.stop = nullptr;                                                         \
        } else {                                                                                    \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);                    \
        }                                                                                           \
    } while (0)

// ---------------------------------------------------------------------------
// complex numbers (interleaved re, im; 8 or 16 bytes, naturally aligned)
// ---------------------------------------------------------------------------
template <typename R>
struct __attribute__((aligned(2 * sizeof(R)))) cpx {
    R x, y;
};

template <typename R> __host__ __device__ __forceinline__ cpx<R> cmk(R a, R b) { return cpx<R>{a, b}; }
template <typename R> __host__ __device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R> __host__ __device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R> __host__ __device__ __forceinline__ cpx<R> operator*(R s, cpx<R> a) { return {s * a.x, s * a.y}; }
// complex product
template <typename R> __host__ __device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename R> __host__ __device__ __forceinline__ cpx<R> cmulc(cpx<R> a, cpx<R> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename R> __host__ __device__ __forceinline__ cpx<R> cconj(cpx<R> a) { return {a.x, -a.y}; }
// i * a
template <typename R> __host__ __device__ __forceinline__ cpx<R> cmuli(cpx<R> a) { return {-a.y, a.x}; }
template <typename R> __host__ __device__ __forceinline__ R cabs2(cpx<R> a) { return a.x * a.x + a.y * a.y; }
// widen to double
template <typename R> __host__ __device__ __forceinline__ cpx<double> wid(cpx<R> a) { return {(double)a.x, (double)a.y}; }

// ---------------------------------------------------------------------------
// problem description of one solve
// ---------------------------------------------------------------------------
struct Phys {
    int dim;                  // 2 or 3
    int n[3];                 // Nx, Ny, Nz (Nz = 1 in 2D)
    double L[3];              // half-widths
    double h[3];              // h_a = 2 L_a / n_a
    long long M;              // points per component
    double cell;              // h^d (rectangle-rule weight)
    double hg[3];             // 1/2 gamma_a^2 (harmonic part)
    double q2, q4;            // isotropic r^2 and r^4 coefficients
    const double* V;          // user potential on the grid (device), or null
    double omega, gamma, c0, c1;
    int nyq_zero;             // odd-operator symbols vanish at the mode -n/2 (GS_NYQ_ZERO)
};

// Every pointer a kernel finds in a slot or a problem description is a device
// (global-memory) address. Kernels read such pointers through as_global, which
// loads the stored value as a pointer of the global address space, so the
// accesses through it compile to global rather than flat memory instructions.
// A flat access also counts as an LDS access: otherwise each LDS wait before a
// block barrier would also wait for the block's outstanding HBM loads and
// stores, prefetches included.
template <typename T> __device__ __forceinline__ T* as_global(T* const& field) {
    __attribute__((address_space(1))) T* g;
    __builtin_memcpy(&g, &field, sizeof g);   // the same 64 bits, read as a global pointer
    return (T*)g;
}

// trap potential, split into its degree-2 and degree-4 parts (V2 + V4 = V)
__device__ __forceinline__ void trap_at(const Phys& p, long long i, double x, double y, double z,
                                        double& V2, double& V4) {
    if (p.V) { V2 = as_global(p.V)[i]; V4 = 0.0; return; }
    double r2 = x * x + y * y + z * z;
    V2 = p.hg[0] * x * x + p.hg[1] * y * y + p.hg[2] * z * z + p.q2 * r2;
    V4 = p.q4 * r2 * r2;
}

// wavenumber of FFT index j on an axis of n points and half-width L:
// p = j for j < n/2 and j - n otherwise (the mode -n/2 is kept), k = pi p / L
__device__ __forceinline__ double wavenum(int j, int n, double L) {
    int p = (j < n / 2) ? j : j - n;
    // pi / L is the same for every point of a kernel: computed once per thread
    return (3.141592653589793238462643 / L) * (double)p;
}
// the same wavenumber in the symbol of an odd operator (D_x, D_y, D_z, hence
// L0, L1, L_z): zero at the mode -n/2 when the problem selects that reading
__device__ __forceinline__ double wavenum_odd(int j, int n, double L, int nyq_zero) {
    return (nyq_zero && j == n / 2) ? 0.0 : wavenum(j, n, L);
}

// ---------------------------------------------------------------------------
// device-resident solver state (one per solve). All control decisions of the
// PCG iteration are taken on the device from these scalars, so a chunk of
// iterations can be enqueued without host round trips.
// ---------------------------------------------------------------------------
enum : int { PH_FP64 = 0, PH_FP32 = 1 };

struct SolveState {
    // control flags
    int done;            // nonzero: every kernel of the iteration returns at once
    int status;          // GS_* code of the solve
    int iter;            // accepted PCG steps
    int iter_phase;      // accepted steps in the current precision phase
    int backtracks, resets;
    int pending_step;    // 1: Phi <- (c Phi + s P/|P|) * inv_norm before the next use
    int have_prev;       // r^{n-1}, P^{n-1} valid (beta may be nonzero)
    int cur;             // index of the r buffer that holds r^n
    int final_pending;   // energy criterion met: evaluate the new iterate, then stop
    int phase;           // PH_FP64 or PH_FP32
    int switch_req;      // FP32 phase finished: continue in FP64
    int best_iter;       // stagnation tracking (FP32 phase)
    int nonfinite;
    // options
    int stop_kind, max_iter, max_backtrack, phase_max_iter, stall_window, precond, exact_ls;
    double tol, switch_resid, theta_trial, sigma;
    // current iterate
    double E, mu, norm2, alpha[3];
    double e_kin, e_pot, e_rot, e_spin, e_soc, e_pot2, e_pot4, virial;
    double mu_comp[3], norm_comp[3];
    double lin;          // <H_L Phi, Phi>
    double resid_inf, best_resid;
    double wchange;      // max |Phi^{n+1} - Phi^n| of the last applied step (criterion (3.9))
    // direction
    double rpr, rpr_prev, beta, dphi, nP, invnP, bdir;
    double rP, phiP, PP;   // Re<r,P^{n-1}>, Re<Phi,P^{n-1}>, |P^{n-1}|^2 (from the residual pass)
    // step
    double a, b, theta, c, s, inv_norm, dE, dE_last;
};

// ---------------------------------------------------------------------------
// per-solve slot: device buffers, problem, state and reduction scratch. Every
// kernel serves all slots of one grid class at once (blockIdx.y = slot) and
// names the buffers it reads and writes by these indices.
// ---------------------------------------------------------------------------
enum BufSel : int {
    B_PHI = 0,   // Phi
    B_HL,        // H_L Phi
    B_R0, B_R1,  // r^n and r^{n-1} (double buffer, SolveState::cur)
    B_PR,        // preconditioned residual
    B_P,         // search direction P^n (P^{n-1} before the direction pass)
    B_HLP,       // H_L P^ (P^ = P / |P|)
    B_U,         // preconditioner input P_V^{1/2} r
    B_T6A, B_T6B,           // six-component scratch (P^ and Phi transformed together)
    B_T0, B_T1, B_T2, B_T3, // scratch
    B_X0, B_X1,             // caller buffers (operator-level entry points)
    NBUF,
    B_NONE = -1
};
constexpr int NS_MAX = 64;          // row stride of the pointwise partial sums
constexpr int W_ROW = NS_MAX - 1;    // row entry of the step's largest change (no other pass uses it)
constexpr int RED_MID_STRIDE = 12;  // row stride of the middle-pass partial sums
constexpr int RED_DIR_STRIDE = 8;   // row stride of the preconditioner's last-pass partial sums

// A slot's fields come in two precisions: the state (Phi, H_L Phi, r^n,
// r^{n-1}; type RS) and the direction (P_C r, P, H_L P^, u and the P_V factors;
// type RD). Scratch fields are sized for RS and used by the transforms of both.
// (RS, RD) is (double, double), (float, float), or (double, float) for the
// double phase of a mixed solve.
struct Slot {
    void* buf[NBUF];
    void* pv;            // [3][M] P_V^{1/2} factors (alpha_l + V + c0 rho)^{-1/2}, type RD
    SolveState* st;
    double* red_mid;     // [nblk_mid][RED_MID_STRIDE]
    double* red_pw;      // [nblk_pw][NS_MAX]
    double* red_dir;     // [nblk_dir][RED_DIR_STRIDE]
    Phys p;
};
template <typename T> __device__ __forceinline__ cpx<T>* fld(const Slot& S, int b) {
    return static_cast<cpx<T>*>(as_global(S.buf[b]));
}
template <typename T> __device__ __forceinline__ T* pvf(const Slot& S) { return static_cast<T*>(as_global(S.pv)); }
template <typename T, typename U> __host__ __device__ __forceinline__ cpx<T> cvt(cpx<U> a) {
    return cpx<T>{(T)a.x, (T)a.y};
}

// reduction geometry of a grid class (same for every slot of the class): the
// number of partial-sum rows each reducing pass writes
struct RedGeom {
    int nblk_mid;   // middle pass of an H_L application
    int nblk_pw;    // pointwise kernels
    int nblk_dir;   // last pass of the preconditioner
};

// ---------------------------------------------------------------------------
// FFT pass launchers (fft_fwd.hip, fft_inv.hip, fft_mid.hip); nslots = grid.y
// ---------------------------------------------------------------------------
enum Pro : int { PRO_PLAIN = 0, PRO_DIR = 2 };
enum Epi : int { EPI_SCALE = 0, EPI_HL = 1, EPI_ROTX = 2 };
enum MidOp : int { MID_HL = 0, MID_PRE = 1, MID_HLX = 2 };

// Launch schedule of an FFT pass: lines per block (the tile of a transposing
// pass, the line positions of a middle-pass group) and threads per block.
// Every pass has NCAND candidate schedules (candidate 0: the fixed table); all
// candidates of a pass compute the same bits, so the autotuner may choose any
// valid one (see fft_launch.h).
struct Cand {
    int tile, nt;
};
constexpr int NCAND = 3;

// Forward transform along the contiguous axis of in[ncomp][A][B][N], written
// with that axis moved to the slowest position: out[ncomp][N][A][B].
// Prologue (in place on the physical input, before the transform):
//   PRO_PLAIN:  transform in as is
//   PRO_DIR:    in <- -aux0 + beta in - dphi aux1 (written back), transform invnP * in
//               (with dual = 1 only: aux1 (Phi) is also transformed into components 3..5)
// in, out and (PRO_DIR) aux0 are of type R; aux1 (Phi) is of type RX.
template <typename R, typename RX>
hipError_t launch_fwdT(int N, int pro, int dual, const Slot* slots, int nslots, int in, int out, int aux0, int aux1,
                       int A, int B, int ncomp, const cpx<R>* tw, int cand, hipStream_t s);

// Inverse transform along the slowest axis of in[3][N][B][C] (and in2 when the
// slot rotates), written with that axis contiguous: out[3][B][Cc][N]; the
// epilogue adds the physical-space terms (see fft_core.h).
// rot_any: some slot of the launch rotates (LDS and buffers for the second
// input/output are provided); each slot decides from its own Omega.
template <typename R>
hipError_t launch_invT(int N, int epi, const Slot* slots, int nslots, int in, int in2, int out, int out2,
                       int uin, int B, int Cc, double scale, int use_invnP, int rot_any, const cpx<R>* tw, int cand,
                       hipStream_t s);

// Last pass of the preconditioner: out = pv * IFFT(in); with dir = 1 also the
// partial sums of the direction reductions (rows in red_dir). Transform, pv,
// out and P are of type R; r^n, r^{n-1} and Phi of type RS.
template <typename R, typename RS>
hipError_t launch_invT_pre(int N, const Slot* slots, int nslots, int in, int out, int B, int Cc, int dir,
                           const cpx<R>* tw, int cand, hipStream_t s);

// Middle pass: transform the contiguous axis of three component lines,
// apply the spectral operator (all three components at each wavenumber),
// transform back. in/outA/outB are [3][nlines][N]; for MID_HLX components 3..5
// of `in` hold the spectrum of Phi.
template <typename R>
hipError_t launch_mid(int N, int op, const Slot* slots, int nslots, int in, int outA, int outB, int nlines,
                      int rot_any, const cpx<R>* tw, int cand, hipStream_t s);

// Middle pass of lines longer than 1024 (2D), split in three launches:
// launch_lfft transforms the ncomp component lines of iin into iout (forward,
// or inverse with inv; in place allowed) and, with iin2 >= 0, the three of
// iin2 into iout2 for rotating slots; irot >= 0 adds the 2D rotation term
// Omega y k_x C / Nx with C = field irot to the inverse of iin. launch_lspec
// applies the spectral operator op to the whole spectrum in (the H_L output
// in outA, the k_y part in outB for rotating slots, the partial sums in
// red_mid rows, one per block of pw_blocks(N nlines)).
template <typename R>
hipError_t launch_lfft(int N, int inv, const Slot* slots, int nslots, int iin, int iout, int ncomp, int nlines,
                       int irot, int iin2, int iout2, const cpx<R>* tw, hipStream_t s);
template <typename R>
hipError_t launch_lspec(int op, const Slot* slots, int nslots, int in, int outA, int outB, int N, int nlines,
                        int rot_any, hipStream_t s);
constexpr int LONG_LINE = 1024;   // middle axes longer than this take the split pass

int mid_blocks(int N, int nlines);
// blocks (= partial-sum rows) of launch_invT_pre for these sizes
template <typename R> int invT_pre_blocks(int N, int B, int Cc);

// validity and description of candidate c for lines of length N (B / Cc: the
// number of line positions the tile must divide)
template <typename R> bool fwdT_cand_ok(int N, int c, int B);
template <typename R> bool invT_cand_ok(int N, int c, int Cc);
template <typename R> bool invT_pre_cand_ok(int N, int c);
bool mid_cand_ok(int N, int c);
template <typename R> Cand fwdT_cand_of(int N, int c);
template <typename R> Cand invT_cand_of(int N, int c);
template <typename R> Cand invT_pre_cand_of(int N, int c);
Cand mid_cand_of(int N, int c);

// ---------------------------------------------------------------------------
// pointwise kernels with fused partial sums (pw_kernels.hip), and the control
// kernel that reduces the rows and takes the decisions of the iteration
// ---------------------------------------------------------------------------
template <typename RS> hipError_t launch_eval(const Slot* slots, int nslots, RedGeom g, hipStream_t s);
template <typename RS, typename RD>
hipError_t launch_resid(const Slot* slots, int nslots, RedGeom g, int final_only, hipStream_t s);
template <typename RS, typename RD> hipError_t launch_lsred(const Slot* slots, int nslots, RedGeom g, hipStream_t s);
// partial sums of |Phi|^2 (the control step FIN_NORM sets the rescale Phi <- Phi / |Phi|)
template <typename RS> hipError_t launch_normalize(const Slot* slots, int nslots, RedGeom g, hipStream_t s);
// pending step Phi <- (c Phi + s P^) inv_norm of every slot, with the block
// maxima of |change| in entry W_ROW of the partial-sum rows
template <typename RS, typename RD> hipError_t launch_apply(const Slot* slots, int nslots, RedGeom g, hipStream_t s);
enum Fin : int {
    FIN_EVAL = 0,     // energy parts, mu, alpha_l of a fresh evaluation
    FIN_DIR = 1,      // stopping tests of the residual pass, then PRP beta and projection
    FIN_LS = 2,       // step size and the next iterate's scalars
    FIN_NORM = 3,     // normalisation
    FIN_RFINAL = 4,   // residual norm of the final iterate
};
// one block per slot: gather the partial-sum rows of the preceding pass(es) in
// a fixed order and run the scalar control on thread 0
hipError_t launch_fin(const Slot* slots, int nslots, RedGeom g, int what, hipStream_t s);
// precision conversion of a field of n complex values
hipError_t launch_convert_d2f(const cpx<double>* in, cpx<float>* out, long long n, hipStream_t s);
hipError_t launch_convert_f2d(const cpx<float>* in, cpx<double>* out, long long n, hipStream_t s);
// X1 = H_L Phi + nonlinear terms = H(Phi)Phi (operator-level entry point)
template <typename R> hipError_t launch_hphi(const Slot* slots, int nslots, RedGeom g, hipStream_t s);
// preconditioner input for the given r in X0: pv = (alpha_l + V + c0 rho)^{-1/2}, u = pv r
template <typename R> hipError_t launch_pvin(const Slot* slots, int nslots, RedGeom g, hipStream_t s);
// zero-padding of a [3][nc] spectrum to [3][nf] (n[2] = 1 in 2D), scaled by Mf/Mc
hipError_t launch_spec_pad(const cpx<double>* in, cpx<double>* out, int dim, const int nc[3], const int nf[3],
                           hipStream_t s);
// Gaussian (a, a, a) initial guess
hipError_t launch_gaussian(cpx<double>* out, const Phys& p, hipStream_t s);

int pw_blocks(long long M);

}  // namespace gs
