/*
 * gs.h - C ABI of the MI355X (gfx950) ground-state library for rotating
 * spin-orbit-coupled spin-1 Bose-Einstein condensates.
 *
 * The library computes
 *
 *     Phi_g = argmin E(Phi)  over  { Phi = (phi_1, phi_0, phi_-1) : N(Phi) = 1 },
 *
 * the ground state of eqs. (1.8)-(1.9) of Wang, Yang, Yuan and Zhang (arXiv
 * 2602.17950), with the energy E of eq. (1.7) and the mass N of eq. (1.6),
 * by the preconditioned nonlinear conjugate gradient method of Sec. 3.1
 * (Algorithm 1, line search and backtracking of Algorithm 2), the combined
 * preconditioner P_C of eq. (3.15) with the shifts of eq. (3.13), and the
 * Fourier spectral discretisation of Sec. 3.2 on the periodic box
 * prod_a [-L_a, L_a].
 *
 * Conventions shared by every entry point
 *   - Wave functions are three consecutive complex grid arrays in the order
 *     (phi_1, phi_0, phi_-1), each [Nz][Ny][Nx] (x fastest; Nz = 1 in 2D),
 *     complex numbers interleaved (re, im). Host arrays are complex128.
 *   - Grid points x_m = -L + m h, h = 2L/N; integrals are h^d times grid sums,
 *     so a normalised Phi has h^d sum |Phi|^2 = 1.
 *   - The caller owns every buffer. The library copies inputs and keeps no
 *     caller pointer after a call returns (after the stream has completed, for
 *     entry points that take a stream).
 *   - Return codes: GS_OK (0); negative = error, outputs untouched;
 *     positive = completed with a warning, outputs valid.
 *   - A context serves one device; calls on one context must not overlap
 *     (one context per host thread, or the caller serialises the calls).
 *   - Solves run in slots: per-solve device memory, state and reduction
 *     scratch. Running solves of the same grid shape, precision and
 *     check_every share every kernel launch; a solve's arithmetic does not
 *     depend on the other slots of its launches, so it returns the same bits
 *     alone, in a batch and under serving.
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_OK 0
#define GS_EINVAL (-1)       /* invalid argument (message in gs_last_error) */
#define GS_ENOMEM (-2)       /* device allocation failed */
#define GS_EDEVICE (-3)      /* HIP runtime error */
#define GS_ENONFINITE (-4)   /* NaN or Inf in the input or during the iteration */
#define GS_ECANCELED (-5)    /* request cancelled before it completed */
#define GS_WMAXITER 1        /* max_iter reached before the stopping criterion */
#define GS_WSTAGNATED 2      /* no descent step found: rounding floor reached */
#define GS_WEXISTENCE 3      /* converged, but the parameters lie outside the hypotheses of the
                                existence theorem of Sec. 2.1 (see gs_existence_check) */
#define GS_PENDING 16        /* gs_poll: the request has not completed yet (not an outcome) */

/* stopping criteria (Sec. 3.4) */
#define GS_STOP_ENERGY 0     /* |E(Phi^{n+1}) - E(Phi^n)| < tol, eq. (3.11) */
#define GS_STOP_RESIDUAL 1   /* max_l ||r_l^n||_inf < tol, eq. (3.10) */
#define GS_STOP_EITHER 2     /* stop at whichever of the two holds first */
#define GS_STOP_WAVEFN 3     /* max_l ||phi_l^{n+1} - phi_l^n||_inf < tol, eq. (3.9) */

/* Preconditioners of Sec. 3.4, all with the shifts alpha_l of eq. (3.13) */
#define GS_PC_COMBINED 0     /* P_V^{1/2} P_Delta P_V^{1/2}, eq. (3.15) (the paper's choice) */
#define GS_PC_KINETIC 1      /* P_Delta = (alpha_l - Lap/2)^{-1}, eq. (3.12) */
#define GS_PC_POTENTIAL 2    /* P_V = (alpha_l + V + c0 rho)^{-1}, eq. (3.14); runs the same
                                transforms with a unit spectral factor */

/* Step size */
#define GS_LS_ALG2 0         /* Algorithm 2: minimiser of the quadratic model (3.6)-(3.8), or
                                theta_trial, halved by sigma until the energy decreases */
#define GS_LS_EXACT 1        /* the step of Algorithm 2, then refined to a minimiser of the
                                energy along the curve cos t Phi + sin t P^ (Newton steps on
                                its explicit form in cos t and sin t; no transform involved) */

/* Symbol of the odd operators D_x, D_y, D_z (and so of L0, L1 and L_z) at the
 * wavenumber index p = -N/2 of Sec. 3.2 (the kinetic symbol always keeps it) */
#define GS_NYQ_KEEP 0        /* v_p = -pi N / (2L), the set Lambda_N as printed (default) */
#define GS_NYQ_ZERO 1        /* symbol 0 at p = -N/2 */

/* arithmetic of the iteration */
#define GS_FP64 0            /* all fields and transforms in double */
#define GS_FP32 1            /* fields and transforms in float, reductions in double */
#define GS_MIXED 2           /* float until the residual reaches switch_resid (or stalls), then double */

typedef struct gs_ctx gs_ctx;

/* Grid: dim = 2 or 3; n[a] points on [-L[a], L[a]] along x, y, z. Each n[a]
 * is 2^k in [16, 1024], 3 * 2^k in [24, 768], or one of 80, 160, 600,
 * 1200, 2400 (the 2400-point grid of Example 5's second case, eq. (4.1), and
 * its halvings down to 600; every length is a multiple of 8); lengths above
 * 1024 in 2D only. Sec. 3.2 requires N even; the
 * transforms are Stockham passes of radix 3, 5 and powers of two. */
typedef struct {
    int dim;
    int n[3];
    double L[3];
} gs_grid;

/* Trap: V = 1/2 sum_a g[a]^2 x_a^2 + q2 r^2 + q4 r^4 with r^2 = sum_a x_a^2
 * (harmonic trap eq. (1.4); harmonic-plus-quartic trap eq. (4.1)), or, when V
 * is not NULL, the sampled potential V[Nz][Ny][Nx] (host, double, copied). */
typedef struct {
    double g[3];
    double q2;
    double q4;
    const double* V;
} gs_trap;

/* Physical parameters (Sec. 1): rotation Omega, SOC strength gamma,
 * interactions c0 (spin independent) and c1 (spin exchange). */
typedef struct {
    double omega;
    double gamma;
    double c0;
    double c1;
} gs_params;

typedef struct {
    int stop_kind;        /* GS_STOP_* */
    double tol;           /* tolerance of the stopping criterion */
    int max_iter;         /* cap on accepted PCG steps (all phases) */
    int precision;        /* GS_FP64, GS_FP32 or GS_MIXED */
    double switch_resid;  /* GS_MIXED: leave float when max_l ||r_l||_inf < switch_resid */
    int fp32_max_iter;    /* GS_MIXED: cap on float steps */
    int stall_window;     /* GS_MIXED: leave float when the residual has not halved for this many steps */
    double theta_trial;   /* Algorithm 2: trial step when the quadratic model has no minimiser */
    double sigma;         /* Algorithm 2: backtracking factor in (0, 1) */
    int max_backtrack;    /* cap on backtracking steps per iteration */
    int check_every;      /* iterations enqueued between two host checks of completion */
    int cm_levels;        /* cascadic multigrid (Algorithm 3): solve on grids n/2^(L-1), ..., n/2, n
                             (every n[a]/2^(L-1) >= 16), each level warm-started from the
                             interpolated result of the previous one; 1 = plain PCG */
    int dir_precision;    /* precision of the search direction, of its preconditioning (3.15), of
                             H_L applied to it and of the stored residuals r^n, r^{n-1}, while Phi
                             and H_L Phi are double (GS_FP64 solves and the double phase of
                             GS_MIXED): GS_FP64 (default) or GS_FP32. The residual is formed in
                             double and every reduction stays double; the line search and the
                             stopping tests act on double quantities, so the limit is the same
                             and only the path to it changes. */
    int precond;          /* GS_PC_* (default GS_PC_COMBINED) */
    int line_search;      /* GS_LS_ALG2 (default) or GS_LS_EXACT */
    int nyquist_odd;      /* GS_NYQ_KEEP (default) or GS_NYQ_ZERO */
} gs_options;

/* Results; quantities refer to the returned Phi. */
typedef struct {
    double E;             /* energy, eq. (1.7) */
    double mu;            /* chemical potential, eq. (2.9) */
    double mu_comp[3];    /* Re<H_l(Phi), phi_l> / N_l; each equals mu at a stationary state */
    double norm_comp[3];  /* N_l = ||phi_l||^2 */
    double e_kin, e_pot, e_rot, e_spin, e_soc;   /* energy parts of the virial identity (2.11) */
    double virial;        /* 2 E_kin - 2 E_pot2 - 4 E_pot4 + d E_spin + E_soc (NaN for a sampled V) */
    double resid_inf;     /* max_l ||H_l(Phi) - mu phi_l||_inf */
    double dE_last;       /* energy change of the last accepted step */
    int iters;            /* accepted PCG steps, all phases */
    int iters_fp32;       /* of which in float arithmetic */
    int backtracks;       /* backtracking steps taken */
    int resets;           /* descent-safeguard resets of beta to 0 */
    int status;           /* return code of the solve */
    double wall_s;        /* wall time of the call */
    int iters_coarse;     /* accepted steps on the coarser levels of a cascadic multigrid solve */
    double dphi_inf;      /* max_l ||phi_l^{n+1} - phi_l^n||_inf of the last step (eq. (3.9));
                             infinity before the first step of the last precision phase */
} gs_result;

/* One solve request of the batch and serving entry points. The trap's V (host)
 * is copied at submission. d_psi0: device complex128 [3][Nz][Ny][Nx] initial
 * guess, or NULL for the Gaussian guess (a, a, a)/sqrt(3) of Sec. 4; it is read
 * when the request is admitted. d_psi_out: device complex128, same shape,
 * written when the request completes. Both stay owned by the caller and must
 * remain valid until the request has completed (or was cancelled). */
typedef struct {
    gs_grid grid;
    gs_trap trap;
    gs_params params;
    gs_options options;
    const void* d_psi0;
    void* d_psi_out;
} gs_request;

/* Create a context on HIP device `device`. Returns GS_OK and *out, or an error.
 * The device-memory budget for solves starts at 90% of the free memory. */
int gs_create(gs_ctx** out, int device);
/* Hypotheses of the existence theorem of Sec. 2.1 for a harmonic trap
 * (gs_trap with q4 = 0 and no sampled V; g_a^2 + 2 q2 taken as gamma_a^2):
 *   |Omega| < min(gamma_x, gamma_y), and
 *   d = 2: c0 > -C_b and c0 + c1 > -C_b, with C_b the best constant of the
 *          Gagliardo-Nirenberg inequality of Sec. 2.1 (5.8503..., half the
 *          mass of the ground state of -Q'' - Q'/r + Q = Q^3 in 2D);
 *   d = 3: c0 >= 0 and c1 >= 0, or c1 <= 0 and c0 + c1 >= 0.
 * Returns GS_OK when they hold or do not apply (a quartic part, which bounds
 * the energy from below for any Omega, or a sampled V), GS_WEXISTENCE when
 * they are violated, GS_EINVAL for invalid arguments. Host-only; a solve
 * that converges on parameters that fail the check returns GS_WEXISTENCE in
 * place of GS_OK (the theorem is sufficient, not necessary: the result may
 * still be a ground state). */
int gs_existence_check(const gs_grid* g, const gs_trap* t, const gs_params* p);

/* Release the context and all device memory it owns. NULL is ignored. */
void gs_destroy(gs_ctx* ctx);
/* Fill *o with the defaults: energy criterion, tol 1e-12, max_iter 100000,
 * FP64, switch_resid 1e-6, fp32_max_iter 20000, stall_window 50,
 * theta_trial 0.1, sigma 0.5, max_backtrack 40, check_every 32, cm_levels 1,
 * dir_precision GS_FP64, precond GS_PC_COMBINED, line_search GS_LS_ALG2,
 * nyquist_odd GS_NYQ_KEEP. */
void gs_default_options(gs_options* o);
/* Device bytes a solve of this grid needs with these options (GS_MIXED counts
 * both the float and the double working sets; dir_precision GS_FP32 halves the
 * direction fields of the double one). 0 for an invalid grid or options. */
size_t gs_footprint_bytes(const gs_grid* g, const gs_options* o);

/* Device-memory budget for solve slots (bytes; 0 = 90% of what is free plus
 * what the context holds). A request is admitted when the footprints
 * (gs_footprint_bytes, plus V) of all admitted, unfinished requests and its
 * own fit in the budget; idle slot memory is kept for reuse and released when
 * a new slot would not fit otherwise. */
int gs_set_hbm_budget(gs_ctx* ctx, size_t bytes);
/* Budget, bytes reserved by admitted requests, bytes of slot memory held. */
int gs_memory_stats(gs_ctx* ctx, size_t* budget, size_t* reserved, size_t* allocated);

/* Ground state from a host initial guess (Algorithm 1). psi0: host complex128
 * [3][Nz][Ny][Nx], or NULL for the Gaussian guess (a, a, a)/sqrt(3) of Sec. 4;
 * it is normalised before the iteration. With options.cm_levels = L > 1 the
 * guess lives on the coarsest grid (n[a] / 2^(L-1) points per axis), the
 * result on the grid g; a sampled trap V is not accepted then. psi_out: host complex128, same shape,
 * caller-allocated (may equal psi0). res: filled on success and on warnings.
 * Synchronous. */
int gs_solve(gs_ctx* ctx, const gs_grid* g, const gs_trap* t, const gs_params* p,
             const gs_options* o, const double* psi0, double* psi_out, gs_result* res);

/* As gs_solve with device buffers: d_psi0 and d_psi_out are complex128 device
 * arrays (d_psi0 may be NULL for the Gaussian guess). Work already queued on
 * `stream` (a hipStream_t; NULL = the null stream) is waited for first; the
 * solve runs on the library's own stream and the call returns after it has
 * finished, with d_psi_out written. */
int gs_solve_device(gs_ctx* ctx, const gs_grid* g, const gs_trap* t, const gs_params* p,
                    const gs_options* o, const void* d_psi0, void* d_psi_out, gs_result* res,
                    void* stream);

/* Many solves at once (grids, parameters and precisions may differ): every
 * request is submitted, then all are run to completion with continuous
 * batching. res[i] receives request i's result; res[i].status is its return
 * code (negative for a solve that failed). Returns GS_OK once every request
 * has completed, or a negative code when a request is invalid (nothing runs)
 * or the device fails. */
int gs_batch_solve(gs_ctx* ctx, int nreq, const gs_request* reqs, gs_result* res);

/* Serving. gs_submit validates and queues a request and returns its ticket;
 * requests are admitted into free slots at chunk boundaries, by footprint,
 * while earlier ones run (continuous batching). The scheduler advances inside
 * gs_submit, gs_progress, gs_poll and gs_wait. gs_progress(block) advances it
 * (block != 0: waits until at least one chunk has completed) and returns the
 * number of unfinished requests. gs_poll returns GS_PENDING, or the request's
 * final return code with *res filled (the ticket is then released; res.wall_s
 * is the time from submission to completion). gs_wait blocks until
 * completion. gs_cancel marks a request; it ends with GS_ECANCELED at its next
 * chunk boundary unless it completes first. */
int gs_submit(gs_ctx* ctx, const gs_request* req, uint64_t* ticket);
int gs_progress(gs_ctx* ctx, int block);
int gs_poll(gs_ctx* ctx, uint64_t ticket, gs_result* res);
int gs_wait(gs_ctx* ctx, uint64_t ticket, gs_result* res);
int gs_cancel(gs_ctx* ctx, uint64_t ticket);

/* Fourier interpolation between grids of the same box (Sec. 3.3, the
 * interpolation step of Algorithm 3): the spectrum of d_in on gc (complex128
 * [3][gc]) is zero-padded to gf (each gf->n[a] >= gc->n[a], same L), the
 * coarse Nyquist coefficient split equally between +n/2 and -n/2, and
 * transformed back, so the coarse grid points are reproduced. d_out: complex128
 * [3][gf]. The call first waits for work already queued on `stream`, then
 * enqueues the interpolation on it and returns. */
int gs_interpolate(gs_ctx* ctx, const gs_grid* gc, const void* d_in, const gs_grid* gf, void* d_out,
                   void* stream);

/* Forward (sign = -1, unnormalised) or inverse (sign = +1, divided by the
 * number of points) discrete Fourier transform of each of the three
 * components of d_in, written to d_out in the same [3][Nz][Ny][Nx] layout
 * with spectral index j_a <-> wavenumber pi p / L_a, p = j (j < n/2) or j - n
 * (Sec. 3.2). Element type: complex128 (GS_FP64) or complex64 (GS_FP32).
 * d_in is not modified. The call first waits for work already queued on
 * `stream`, then enqueues the transform on it and returns. */
int gs_fft(gs_ctx* ctx, const gs_grid* g, int precision, int sign, const void* d_in,
           void* d_out, void* stream);

/* gs_fft without device allocation, for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). Same transform, arguments and result as gs_fft, from the same
 * kernels and twiddle tables. Every buffer besides d_in and d_out (the slot
 * descriptor, the solver state, the scratch fields and the twiddle tables)
 * lives in one static device array per GPU, set up by gs_create; at most
 * 2^18 points per component (GS_EINVAL beyond). The call only enqueues
 * kernels on `stream` and returns (no allocation, no host synchronisation).
 * The array is shared by every call on the GPU and keeps the last call's
 * contents: calls that overlap in time on one GPU (other streams or threads)
 * race and must be serialised by the caller. */
int gs_fft_noalloc(gs_ctx* ctx, const gs_grid* g, int precision, int sign, const void* d_in, void* d_out,
                   void* stream);

/* H(Phi)Phi, the right-hand side of the Euler-Lagrange equations (2.6)-(2.8),
 * for the device field d_psi (taken as given, not normalised), written to
 * d_hpsi; when res is not NULL also E, its parts, mu, mu_l, N_l, the virial
 * residual and max_l ||H_l(Phi) - mu phi_l||_inf (mu from eq. (2.9)).
 * Element type as for gs_fft. Synchronous when res is not NULL. */
int gs_hamiltonian(gs_ctx* ctx, const gs_grid* g, const gs_trap* t, const gs_params* p,
                   int precision, const void* d_psi, void* d_hpsi, gs_result* res, void* stream);

/* Combined preconditioner of eq. (3.15): d_out = P_V^{1/2} P_Delta P_V^{1/2} d_r
 * with alpha_l of eq. (3.13) evaluated at d_psi. Element type as for gs_fft.
 * Queued on `stream` as for gs_fft (synchronous when the trap has a V). */
int gs_precondition(gs_ctx* ctx, const gs_grid* g, const gs_trap* t, const gs_params* p,
                    int precision, const void* d_psi, const void* d_r, void* d_out, void* stream);

/* Measurement helpers. Kernel kinds of one PCG iteration:
 *   0 first FFT pass of an H_L application, 1 its spectral middle pass,
 *   2 its last FFT pass, 3/4/5 the same for the preconditioner, 6 energy and
 *   mu sums, 7 residual, 8 (reserved), 9 step-size sums, 10/11 the second
 *   forward / inverse passes of a 3D H_L application, 12 the control steps
 *   (fixed-order totals of the partial sums and the scalar decisions).
 * gs_kernel_timer_start(ctx, kind) makes later solves on ctx bracket every
 * launch of that kernel with HIP events on the launch's stream (kind -1: off)
 * and resets the totals; gs_kernel_timer_read returns the summed elapsed time
 * (ms), the summed algorithmic bytes (each array the kernel reads or writes
 * counted once) and the number of launches timed. Launches that return at
 * once because the solve has already finished are not counted. */
int gs_kernel_timer_start(gs_ctx* ctx, int kind);
int gs_kernel_timer_read(gs_ctx* ctx, double* total_ms, double* total_bytes, long long* launches);

/* Launch schedules of the FFT passes (the coefficients by FFT of Sec. 3.2).
 * Every pass of the PCG iteration has a few candidate schedules (lines and
 * threads per block) that compute the same bits. With autotuning on (the
 * default), the first chunk of iterations of a grid class run with a given
 * number of running solves (bucketed by powers of two) cycles through every
 * pass's candidates, timing each launch with events, and the fastest is kept
 * for that class and bucket; off (on = 0): the fixed table. Results do not
 * depend on the setting. gs_autotune_report returns a JSON array (valid
 * until the next call on ctx, NULL for a NULL ctx): per class and bucket, the
 * chosen "TILExNT" of each pass and the mean launch time (us) of every
 * candidate. */
int gs_set_autotune(gs_ctx* ctx, int on);
const char* gs_autotune_report(gs_ctx* ctx);

/* Message of the last error on this thread ("" if none). */
const char* gs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
