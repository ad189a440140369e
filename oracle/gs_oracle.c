/*
 * gs_oracle.c - plain FP64 CPU oracle for the ground-state problem of rotating
 * spin-orbit-coupled spin-1 Bose-Einstein condensates solved by the Fourier
 * spectral preconditioned nonlinear conjugate gradient (PCG) method of
 * Wang, Yang, Yuan and Zhang, arXiv 2602.17950.
 *
 * TEST INFRASTRUCTURE. This file is the checker, not the product: only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no source, header, table or helper with the GPU library, and it
 * never calls into it.
 *
 * Style: everything is double precision and written to be checked by eye
 * against the paper. No blocking, fusion or reordering beyond what the
 * definitions state. The only parallelism is a loop over independent FFT lines.
 *
 * Conventions (paper Sec. 1 and Sec. 3.2):
 *   - wave function Phi = (phi_1, phi_0, phi_-1), stored as three consecutive
 *     complex grid arrays, component index c = 0, 1, 2 <-> l = +1, 0, -1;
 *   - grid array layout [Nz][Ny][Nx], x fastest; in 2D Nz = 1;
 *   - x_m = -L + m h, h = 2L/N (Sec. 3.2, sets O_N, Q_N);
 *   - Fourier index j <-> p = j (j < N/2) or j - N (j >= N/2), so that
 *     p runs over Lambda_N = [-N/2, N/2-1] including the mode -N/2;
 *     wavenumber v_p = pi p / L (Sec. 3.2);
 *   - forward transform sum_m f_m exp(-2 pi i p m / N), which is the paper's
 *     coefficient definition with the phase origin at -L; the inverse carries
 *     the 1/N factor so that inverse(forward(f)) = f;
 *   - integrals are the rectangle rule h^d sum over the periodic grid, and the
 *     inner product is <v,u> = h^d sum_l sum_grid v_l conj(u_l) (Sec. 2.2).
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* n[0]=Nx, n[1]=Ny, n[2]=Nz. nyq_zero selects the reading of the mode p = -N/2 in
 * the symbols of the odd operators D_a (hence L0, L1 and L_z): 0 keeps
 * v_p = -pi N / (2L) as the set Lambda_N of Sec. 3.2 lists it; 1 sets that
 * symbol to zero. The kinetic symbol keeps the mode in both readings. */
typedef struct { int dim; int n[3]; double L[3]; int nyq_zero; } orc_grid;
/* V(x) = 1/2 sum_a g_a^2 x_a^2 + q2 r^2 + q4 r^4 (r^2 = sum over all d axes),
 * or a sampled array when V != NULL (harmonic trap: Sec. 1 eq. (1.4);
 * harmonic-plus-quartic trap: eq. (4.1) of Example 5). */
typedef struct { double g[3]; double q2; double q4; const double* V; } orc_trap;
typedef struct { double omega, gamma, c0, c1; } orc_params;         /* Omega, gamma (SOC), c0, c1 */
enum { ORC_STOP_ENERGY = 0, ORC_STOP_RESIDUAL = 1, ORC_STOP_BOTH = 2, ORC_STOP_WAVEFN = 3 };
/* preconditioners of Sec. 3.4: combined (3.15), kinetic (3.12), potential (3.14) */
enum { ORC_PC_COMBINED = 0, ORC_PC_KINETIC = 1, ORC_PC_POTENTIAL = 2 };
typedef struct {
    int stop_kind;        /* stop on the energy difference (3.11), the residual (3.10), either of
                             the two, or the wave-function difference (3.9) */
    double tol;
    int max_iter;
    double theta_trial;   /* the "prescribed small positive number" of Algorithm 2 */
    double sigma;         /* backtracking factor of Algorithm 2 */
    int max_backtrack;    /* cap on Step 4 repetitions (the paper gives none) */
    int precond;          /* ORC_PC_*; every kind uses the shifts alpha_l of (3.13) */
    int exact_ls;         /* 0: Algorithm 2; 1: minimise E along the curve (see orc_exact_theta) */
} orc_options;
typedef struct {
    double E, e_kin, e_pot, e_rot, e_spin, e_soc, e_pot2, e_pot4;
    double mu, mu_comp[3], norm_comp[3], norm, alpha[3];
    double virial, resid_inf;
} orc_eval;
typedef struct { int iters, backtracks, resets, status; double dE_last, resid_inf; } orc_stats;
enum { ORC_OK = 0, ORC_MAXITER = 1, ORC_STAGNATED = 2, ORC_NONFINITE = -4, ORC_EINVAL = -1 };

static int g_threads = 1;
void orc_set_threads(int n) { g_threads = n > 0 ? n : 1; }
int orc_get_threads(void) { return g_threads; }

/* ------------------------------------------------------------------------- */
/* grid helpers (Sec. 3.2)                                                    */
/* ------------------------------------------------------------------------- */
static int nz_of(const orc_grid* g) { return g->dim == 3 ? g->n[2] : 1; }
static long npts(const orc_grid* g) { return (long)g->n[0] * g->n[1] * nz_of(g); }
static double hstep(const orc_grid* g, int a) { return 2.0 * g->L[a] / g->n[a]; }
static double cell(const orc_grid* g) {
    double v = hstep(g, 0) * hstep(g, 1);
    if (g->dim == 3) v *= hstep(g, 2);
    return v;
}
static double coord(const orc_grid* g, int a, int m) { return -g->L[a] + m * hstep(g, a); }
/* v_p = pi p / L with p in [-N/2, N/2-1] (the mode -N/2 is kept, as in Lambda_N) */
static double wavenum(const orc_grid* g, int a, int j) {
    int n = g->n[a];
    int p = (j < n / 2) ? j : j - n;
    return M_PI * p / g->L[a];
}
/* wavenumber in the symbol of an odd operator (D_a): as wavenum, except that
 * the mode p = -N/2 has symbol 0 when the grid selects that reading */
static double wavenum_odd(const orc_grid* g, int a, int j) {
    if (g->nyq_zero && j == g->n[a] / 2) return 0.0;
    return wavenum(g, a, j);
}
static void unpack(const orc_grid* g, long i, int* ix, int* iy, int* iz) {
    *ix = (int)(i % g->n[0]);
    *iy = (int)((i / g->n[0]) % g->n[1]);
    *iz = (int)(i / ((long)g->n[0] * g->n[1]));
}

/* ------------------------------------------------------------------------- */
/* Fourier transforms (Sec. 3.2, coefficients by FFT)                         */
/* ------------------------------------------------------------------------- */
/* Naive O(n^2) DFT straight from the definition: out_p = sum_m in_m e^{sign 2 pi i p m / n}. */
void orc_dft(int n, const cplx* in, cplx* out, int sign) {
    for (int p = 0; p < n; ++p) {
        cplx s = 0;
        for (int m = 0; m < n; ++m) {
            long pm = ((long)p * m) % n;
            double ang = sign * 2.0 * M_PI * (double)pm / n;
            s += in[m] * (cos(ang) + I * sin(ang));
        }
        out[p] = s;
    }
}

static int is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

/* Twiddle table w[k] = e^{sign 2 pi i k / n}, k < n/2, each entry from cos/sin. */
static cplx* twiddles(int n, int sign) {
    cplx* w = (cplx*)malloc(sizeof(cplx) * (n / 2 + 1));
    for (int k = 0; k < n / 2; ++k) {
        double ang = sign * 2.0 * M_PI * (double)k / n;
        w[k] = cos(ang) + I * sin(ang);
    }
    return w;
}

/* Iterative radix-2 Cooley-Tukey: bit-reversal permutation followed by
 * butterflies of growing length; w is the twiddle table of length n. */
static void fft_radix2(int n, cplx* a, const cplx* w) {
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cplx t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len / 2, step = n / len;
        for (int i = 0; i < n; i += len) {
            for (int k = 0; k < half; ++k) {
                cplx u = a[i + k];
                cplx v = a[i + k + half] * w[k * step];
                a[i + k] = u + v;
                a[i + k + half] = u - v;
            }
        }
    }
}

/* Full root table w[j] = e^{sign 2 pi i j / n}, j < n, each entry from cos/sin. */
static cplx* roots(int n, int sign) {
    cplx* w = (cplx*)malloc(sizeof(cplx) * n);
    for (int j = 0; j < n; ++j) {
        double ang = sign * 2.0 * M_PI * (double)j / n;
        w[j] = cos(ang) + I * sin(ang);
    }
    return w;
}

/* Mixed-radix Cooley-Tukey by decimation in time, recursive: with p the
 * smallest of 2, 3, 5 dividing n (the DFT definition itself when none does),
 * the p subsequences x[s], x[s + p], ... (stride `stride` apart in memory)
 * are transformed as sequences of length m = n/p into Y_s = X[s m ...], and
 * out_{k + q m} = sum_s e^{sign 2 pi i s (k + q m) / n} Y_s[k]. The roots of
 * unity of order n are w[(j mod n) wstep], w the root table of the top-level
 * length n wstep. tmp: n values. */
static void fft_mixed(int n, const cplx* x, long stride, cplx* X, cplx* tmp, const cplx* w, int wstep) {
    if (n == 1) { X[0] = x[0]; return; }
    int p = (n % 2 == 0) ? 2 : (n % 3 == 0) ? 3 : (n % 5 == 0) ? 5 : n;
    int m = n / p;
    if (p == n) {   /* no small factor: the definition */
        for (int k = 0; k < n; ++k) {
            cplx acc = 0;
            for (int j = 0; j < n; ++j) acc += x[j * stride] * w[(((long)j * k) % n) * wstep];
            X[k] = acc;
        }
        return;
    }
    for (int s0 = 0; s0 < p; ++s0) fft_mixed(m, x + s0 * stride, stride * p, X + s0 * m, tmp, w, wstep * p);
    for (int k = 0; k < m; ++k)
        for (int q = 0; q < p; ++q) {
            cplx acc = 0;
            for (int s0 = 0; s0 < p; ++s0) acc += X[s0 * m + k] * w[(((long)s0 * (k + q * m)) % n) * wstep];
            tmp[k + q * m] = acc;
        }
    memcpy(X, tmp, sizeof(cplx) * n);
}

/* One-dimensional transform, unnormalised in both directions: radix 2 for
 * powers of two, mixed radix otherwise. */
void orc_fft1d(int n, cplx* a, int sign) {
    if (is_pow2(n)) {
        cplx* w = twiddles(n, sign);
        fft_radix2(n, a, w);
        free(w);
        return;
    }
    cplx* in = (cplx*)malloc(sizeof(cplx) * n);
    cplx* tmp = (cplx*)malloc(sizeof(cplx) * n);
    cplx* w = roots(n, sign);
    memcpy(in, a, sizeof(cplx) * n);
    fft_mixed(n, in, 1, a, tmp, w, 1);
    free(in);
    free(tmp);
    free(w);
}

/* d-dimensional transform of one grid array, axis by axis (the DFT factorises).
 * sign = -1: forward, unnormalised. sign = +1: inverse, divided by the number
 * of points so that the pair is the identity. */
void orc_fftn(const orc_grid* g, cplx* f, int sign) {
    long M = npts(g);
    int naxes = g->dim;
    long stride = 1;
    for (int a = 0; a < naxes; ++a) {
        int n = g->n[a];
        long nlines = M / n;
        long st = stride;
        int p2 = is_pow2(n);
        cplx* w = p2 ? twiddles(n, sign) : roots(n, sign);
        #pragma omp parallel num_threads(g_threads)
        {
            cplx* line = (cplx*)malloc(sizeof(cplx) * n);
            cplx* tmp = p2 ? NULL : (cplx*)malloc(sizeof(cplx) * n);
            cplx* tmp2 = p2 ? NULL : (cplx*)malloc(sizeof(cplx) * n);
            #pragma omp for schedule(static)
            for (long l = 0; l < nlines; ++l) {
                long outer = l / st, inner = l % st;
                long start = outer * st * n + inner;
                for (int m = 0; m < n; ++m) line[m] = f[start + m * st];
                if (p2) fft_radix2(n, line, w);
                else { fft_mixed(n, line, 1, tmp, tmp2, w, 1); memcpy(line, tmp, sizeof(cplx) * n); }
                for (int m = 0; m < n; ++m) f[start + m * st] = line[m];
            }
            free(line);
            free(tmp);
            free(tmp2);
        }
        free(w);
        stride *= n;
    }
    if (sign > 0) {
        for (long i = 0; i < M; ++i) f[i] /= (double)M;
    }
}

/* ------------------------------------------------------------------------- */
/* trap potential (eq. (1.4); harmonic-plus-quartic form, eq. (4.1))         */
/* ------------------------------------------------------------------------- */
static double r2_at(const orc_grid* g, long i) {
    int ix, iy, iz;
    unpack(g, i, &ix, &iy, &iz);
    double x = coord(g, 0, ix), y = coord(g, 1, iy);
    double r2 = x * x + y * y;
    if (g->dim == 3) { double z = coord(g, 2, iz); r2 += z * z; }
    return r2;
}
/* degree-2 part of the parametric potential */
static double pot2_at(const orc_grid* g, const orc_trap* t, long i) {
    int ix, iy, iz;
    unpack(g, i, &ix, &iy, &iz);
    double x = coord(g, 0, ix), y = coord(g, 1, iy);
    double v = 0.5 * (t->g[0] * t->g[0] * x * x + t->g[1] * t->g[1] * y * y);
    if (g->dim == 3) { double z = coord(g, 2, iz); v += 0.5 * t->g[2] * t->g[2] * z * z; }
    return v + t->q2 * r2_at(g, i);
}
static double pot4_at(const orc_grid* g, const orc_trap* t, long i) {
    double r2 = r2_at(g, i);
    return t->q4 * r2 * r2;
}
static double pot_at(const orc_grid* g, const orc_trap* t, long i) {
    if (t->V) return t->V[i];
    return pot2_at(g, t, i) + pot4_at(g, t, i);
}
void orc_potential(const orc_grid* g, const orc_trap* t, double* V) {
    long M = npts(g);
    for (long i = 0; i < M; ++i) V[i] = pot_at(g, t, i);
}

/* ------------------------------------------------------------------------- */
/* inner products and norms (Sec. 2.2)                                        */
/* ------------------------------------------------------------------------- */
/* Re <v,u> = h^d sum_l sum_grid Re(v_l conj(u_l)) over the three components */
double orc_re_inner(const orc_grid* g, const cplx* v, const cplx* u) {
    long n3 = 3 * npts(g);
    double s = 0.0;
    for (long i = 0; i < n3; ++i) s += creal(v[i] * conj(u[i]));
    return s * cell(g);
}
static void normalise(const orc_grid* g, cplx* phi) {
    double nrm = sqrt(orc_re_inner(g, phi, phi));
    long n3 = 3 * npts(g);
    for (long i = 0; i < n3; ++i) phi[i] /= nrm;
}

/* ------------------------------------------------------------------------- */
/* spectral operators (Sec. 3.2)                                              */
/* ------------------------------------------------------------------------- */
/* spectra of the three components */
static cplx* spectra(const orc_grid* g, const cplx* u) {
    long M = npts(g);
    cplx* uh = (cplx*)malloc(sizeof(cplx) * 3 * M);
    memcpy(uh, u, sizeof(cplx) * 3 * M);
    for (int c = 0; c < 3; ++c) orc_fftn(g, uh + c * M, -1);
    return uh;
}
static void kvec(const orc_grid* g, long i, double* kx, double* ky, double* kz) {
    int jx, jy, jz;
    unpack(g, i, &jx, &jy, &jz);
    *kx = wavenum(g, 0, jx);
    *ky = wavenum(g, 1, jy);
    *kz = g->dim == 3 ? wavenum(g, 2, jz) : 0.0;
}
/* wavenumbers in the symbols of the odd operators D_x, D_y, D_z */
static void kvec_odd(const orc_grid* g, long i, double* kx, double* ky, double* kz) {
    int jx, jy, jz;
    unpack(g, i, &jx, &jy, &jz);
    *kx = wavenum_odd(g, 0, jx);
    *ky = wavenum_odd(g, 1, jy);
    *kz = g->dim == 3 ? wavenum_odd(g, 2, jz) : 0.0;
}
/* D_a f = -i d/dx_a f, symbol v^a (so that L_z = x D_y - y D_x, Sec. 3.2) */
void orc_apply_deriv(const orc_grid* g, int axis, const cplx* f, cplx* out) {
    long M = npts(g);
    memcpy(out, f, sizeof(cplx) * M);
    orc_fftn(g, out, -1);
    for (long i = 0; i < M; ++i) {
        double k[3];
        kvec_odd(g, i, &k[0], &k[1], &k[2]);
        out[i] *= k[axis];
    }
    orc_fftn(g, out, +1);
}
/* L_z f = -i (x d_y - y d_x) f = x D_y f - y D_x f (Sec. 1; symbol x v^y - y v^x in Sec. 3.2) */
static void apply_Lz_one(const orc_grid* g, const cplx* f, cplx* out) {
    long M = npts(g);
    cplx* dx = (cplx*)malloc(sizeof(cplx) * M);
    cplx* dy = (cplx*)malloc(sizeof(cplx) * M);
    orc_apply_deriv(g, 0, f, dx);
    orc_apply_deriv(g, 1, f, dy);
    for (long i = 0; i < M; ++i) {
        int ix, iy, iz;
        unpack(g, i, &ix, &iy, &iz);
        double x = coord(g, 0, ix), y = coord(g, 1, iy);
        out[i] = x * dy[i] - y * dx[i];
    }
    free(dx);
    free(dy);
}
void orc_apply_Lz(const orc_grid* g, const cplx* u, cplx* out) {
    long M = npts(g);
    for (int c = 0; c < 3; ++c) apply_Lz_one(g, u + c * M, out + c * M);
}
/* Symbols of the SOC operators (Sec. 3.2):
 *   L0 = i d_x + d_y  ->  -v^x + i v^y,
 *   L1 = i d_x - d_y  ->  -(v^x + i v^y). */
static cplx sym_L0(double kx, double ky) { return -kx + I * ky; }
static cplx sym_L1(double kx, double ky) { return -(kx + I * ky); }
/* S Phi with S = [[0, L0, 0], [L1, 0, L0], [0, L1, 0]] (Sec. 1) */
void orc_apply_soc(const orc_grid* g, const cplx* u, cplx* out) {
    long M = npts(g);
    cplx* uh = spectra(g, u);
    for (long i = 0; i < M; ++i) {
        double kx, ky, kz;
        kvec_odd(g, i, &kx, &ky, &kz);
        cplx s0 = sym_L0(kx, ky), s1 = sym_L1(kx, ky);
        out[0 * M + i] = s0 * uh[1 * M + i];
        out[1 * M + i] = s1 * uh[0 * M + i] + s0 * uh[2 * M + i];
        out[2 * M + i] = s1 * uh[1 * M + i];
    }
    for (int c = 0; c < 3; ++c) orc_fftn(g, out + c * M, +1);
    free(uh);
}
/* Linear part H_L u = (-1/2 Lap + V - Omega L_z) u_l - gamma (S u)_l, the
 * l-independent single-particle operator of H_0 (without c0 rho) plus SOC. */
void orc_apply_HL(const orc_grid* g, const orc_trap* t, const orc_params* p,
                  const cplx* u, cplx* out) {
    long M = npts(g);
    cplx* uh = spectra(g, u);
    /* kinetic: -1/2 Lap has symbol 1/2 |v|^2 */
    for (int c = 0; c < 3; ++c) {
        for (long i = 0; i < M; ++i) {
            double kx, ky, kz;
            kvec(g, i, &kx, &ky, &kz);
            out[c * M + i] = 0.5 * (kx * kx + ky * ky + kz * kz) * uh[c * M + i];
        }
        orc_fftn(g, out + c * M, +1);
    }
    free(uh);
    /* SOC */
    cplx* su = (cplx*)malloc(sizeof(cplx) * 3 * M);
    orc_apply_soc(g, u, su);
    for (long i = 0; i < 3 * M; ++i) out[i] -= p->gamma * su[i];
    /* rotation */
    if (p->omega != 0.0) {
        orc_apply_Lz(g, u, su);
        for (long i = 0; i < 3 * M; ++i) out[i] -= p->omega * su[i];
    }
    free(su);
    /* trap */
    for (int c = 0; c < 3; ++c)
        for (long i = 0; i < M; ++i) out[c * M + i] += pot_at(g, t, i) * u[c * M + i];
}

/* ------------------------------------------------------------------------- */
/* spin densities and nonlinear terms (Sec. 1)                                */
/* ------------------------------------------------------------------------- */
/* F = (Psi^dag f_x Psi, Psi^dag f_y Psi, Psi^dag f_z Psi), explicit formulas of Sec. 1 */
static void spin_vector(cplx p1, cplx p0, cplx pm, double* Fx, double* Fy, double* Fz) {
    const double s = 1.0 / sqrt(2.0);
    cplx fx = s * (conj(p1) * p0 + conj(p0) * (p1 + pm) + conj(pm) * p0);
    cplx fy = I * s * (-conj(p1) * p0 + conj(p0) * (p1 - pm) + conj(pm) * p0);
    *Fx = creal(fx);
    *Fy = creal(fy);
    *Fz = creal(p1 * conj(p1)) - creal(pm * conj(pm));
}
void orc_spin_density(const orc_grid* g, const cplx* phi, double* Fx, double* Fy, double* Fz) {
    long M = npts(g);
    for (long i = 0; i < M; ++i) spin_vector(phi[i], phi[M + i], phi[2 * M + i], &Fx[i], &Fy[i], &Fz[i]);
}
/* |F|^2 in the real form used by E_2 in Sec. 2.1 */
void orc_spin_sq_realform(const orc_grid* g, const cplx* phi, double* out) {
    long M = npts(g);
    for (long i = 0; i < M; ++i) {
        cplx p1 = phi[i], p0 = phi[M + i], pm = phi[2 * M + i];
        double a = creal((conj(p1) + conj(pm)) * p0);
        double b = cimag(p0 * (conj(pm) - conj(p1)));
        double z = creal(p1 * conj(p1)) - creal(pm * conj(pm));
        out[i] = 2 * a * a + 2 * b * b + z * z;
    }
}
/* H(Phi)Phi, the right-hand sides of the Euler-Lagrange equations (2.6)-(2.8),
 * written term by term as printed. */
void orc_apply_H(const orc_grid* g, const orc_trap* t, const orc_params* p,
                 const cplx* phi, cplx* out) {
    long M = npts(g);
    orc_apply_HL(g, t, p, phi, out);
    for (long i = 0; i < M; ++i) {
        cplx p1 = phi[i], p0 = phi[M + i], pm = phi[2 * M + i];
        double r1 = creal(p1 * conj(p1)), r0 = creal(p0 * conj(p0)), rm = creal(pm * conj(pm));
        double rho = r1 + r0 + rm;
        out[i] += (p->c0 * rho + p->c1 * (r0 + r1 - rm)) * p1 + p->c1 * conj(pm) * p0 * p0;
        out[M + i] += (p->c0 * rho + p->c1 * (r1 + rm)) * p0 + 2 * p->c1 * pm * conj(p0) * p1;
        out[2 * M + i] += (p->c0 * rho + p->c1 * (r0 + rm - r1)) * pm + p->c1 * p0 * p0 * conj(p1);
    }
}
/* H_Phi u: the Hamiltonian with rho and F frozen at Phi, applied to u, using the
 * compact form [H_0 + c1 F.f - gamma S] of Sec. 1 (matrix F.f with F_pm = F_x +- i F_y). */
void orc_apply_H_frozen(const orc_grid* g, const orc_trap* t, const orc_params* p,
                        const cplx* phi, const cplx* u, cplx* out) {
    long M = npts(g);
    const double s = 1.0 / sqrt(2.0);
    orc_apply_HL(g, t, p, u, out);
    for (long i = 0; i < M; ++i) {
        cplx p1 = phi[i], p0 = phi[M + i], pm = phi[2 * M + i];
        double rho = creal(p1 * conj(p1) + p0 * conj(p0) + pm * conj(pm));
        double Fx, Fy, Fz;
        spin_vector(p1, p0, pm, &Fx, &Fy, &Fz);
        cplx Fp = Fx + I * Fy, Fm = Fx - I * Fy;
        cplx u1 = u[i], u0 = u[M + i], um = u[2 * M + i];
        out[i] += p->c0 * rho * u1 + p->c1 * (Fz * u1 + s * Fm * u0);
        out[M + i] += p->c0 * rho * u0 + p->c1 * (s * Fp * u1 + s * Fm * um);
        out[2 * M + i] += p->c0 * rho * um + p->c1 * (s * Fp * u0 - Fz * um);
    }
}

/* ------------------------------------------------------------------------- */
/* energy functional (1.7), chemical potential (2.9), virial identity (2.11)  */
/* ------------------------------------------------------------------------- */
/* Per-component kinetic energy 1/2 int |grad phi_l|^2, by Parseval. */
static void kinetic_parts(const orc_grid* g, const cplx* phi, double K[3]) {
    long M = npts(g);
    cplx* uh = spectra(g, phi);
    double sc = cell(g) / (double)M;
    for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (long i = 0; i < M; ++i) {
            double kx, ky, kz;
            kvec(g, i, &kx, &ky, &kz);
            s += 0.5 * (kx * kx + ky * ky + kz * kz) * creal(uh[c * M + i] * conj(uh[c * M + i]));
        }
        K[c] = s * sc;
    }
    free(uh);
}

/* Energy and its parts E_kin, E_pot, E_rot, E_spin, E_soc (as defined with the
 * virial identity (2.11)), each
 * written from its own definition. Does not evaluate H. */
static void energy_parts(const orc_grid* g, const orc_trap* t, const orc_params* p,
                         const cplx* phi, orc_eval* e) {
    long M = npts(g);
    double hd = cell(g);
    double K[3];
    kinetic_parts(g, phi, K);
    e->e_kin = K[0] + K[1] + K[2];
    double ep = 0, ep2 = 0, ep4 = 0, es = 0;
    for (long i = 0; i < M; ++i) {
        cplx p1 = phi[i], p0 = phi[M + i], pm = phi[2 * M + i];
        double rho = creal(p1 * conj(p1) + p0 * conj(p0) + pm * conj(pm));
        double Fx, Fy, Fz;
        spin_vector(p1, p0, pm, &Fx, &Fy, &Fz);
        ep += pot_at(g, t, i) * rho;
        if (!t->V) { ep2 += pot2_at(g, t, i) * rho; ep4 += pot4_at(g, t, i) * rho; }
        es += 0.5 * p->c0 * rho * rho + 0.5 * p->c1 * (Fx * Fx + Fy * Fy + Fz * Fz);
    }
    e->e_pot = ep * hd;
    e->e_pot2 = ep2 * hd;
    e->e_pot4 = ep4 * hd;
    e->e_spin = es * hd;
    cplx* w = (cplx*)malloc(sizeof(cplx) * 3 * M);
    if (p->omega != 0.0) {
        orc_apply_Lz(g, phi, w);
        e->e_rot = -p->omega * orc_re_inner(g, w, phi);
    } else {
        e->e_rot = 0.0;
    }
    orc_apply_soc(g, phi, w);
    e->e_soc = -p->gamma * orc_re_inner(g, w, phi);
    free(w);
    e->E = e->e_kin + e->e_pot + e->e_rot + e->e_spin + e->e_soc;
}

double orc_energy(const orc_grid* g, const orc_trap* t, const orc_params* p, const cplx* phi) {
    orc_eval e;
    energy_parts(g, t, p, phi, &e);
    return e.E;
}

/* Shift alpha_l of the preconditioners, eq. (3.13). */
void orc_alpha(const orc_grid* g, const orc_trap* t, const orc_params* p, const cplx* phi, double alpha[3]) {
    long M = npts(g);
    double K[3];
    kinetic_parts(g, phi, K);
    for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (long i = 0; i < M; ++i) {
            double rho = creal(phi[i] * conj(phi[i]) + phi[M + i] * conj(phi[M + i]) +
                               phi[2 * M + i] * conj(phi[2 * M + i]));
            double rc = creal(phi[c * M + i] * conj(phi[c * M + i]));
            s += (pot_at(g, t, i) + p->c0 * rho) * rc;
        }
        alpha[c] = K[c] + s * cell(g);
    }
}

/* Full evaluation: energy parts, mu (2.9), mu_l, N_l, alpha_l, residual, virial. */
void orc_evaluate(const orc_grid* g, const orc_trap* t, const orc_params* p,
                  const cplx* phi, orc_eval* e) {
    long M = npts(g);
    double hd = cell(g);
    energy_parts(g, t, p, phi, e);
    cplx* hphi = (cplx*)malloc(sizeof(cplx) * 3 * M);
    orc_apply_H(g, t, p, phi, hphi);
    e->mu = orc_re_inner(g, hphi, phi);
    e->norm = 0.0;
    for (int c = 0; c < 3; ++c) {
        double sn = 0.0, sh = 0.0;
        for (long i = 0; i < M; ++i) {
            sn += creal(phi[c * M + i] * conj(phi[c * M + i]));
            sh += creal(hphi[c * M + i] * conj(phi[c * M + i]));
        }
        e->norm_comp[c] = sn * hd;
        e->norm += sn * hd;
        e->mu_comp[c] = sh * hd / (sn * hd);
    }
    double rinf = 0.0;
    for (int c = 0; c < 3; ++c)
        for (long i = 0; i < M; ++i) {
            double a = cabs(hphi[c * M + i] - e->mu * phi[c * M + i]);
            if (a > rinf) rinf = a;
        }
    e->resid_inf = rinf;
    free(hphi);
    orc_alpha(g, t, p, phi, e->alpha);
    /* virial identity (2.11); for a potential with degree-2 and degree-4 parts
     * the same scaling argument gives -2 E_pot2 - 4 E_pot4 in place of -2 E_pot */
    if (t->V) e->virial = NAN;
    else e->virial = 2 * e->e_kin - 2 * e->e_pot2 - 4 * e->e_pot4 + g->dim * e->e_spin + e->e_soc;
}

/* ------------------------------------------------------------------------- */
/* combined preconditioner P_C = P_V^{1/2} P_Delta P_V^{1/2}, eqs. (3.12)-(3.15) */
/* ------------------------------------------------------------------------- */
void orc_precond(const orc_grid* g, const orc_trap* t, const orc_params* p,
                 const cplx* phi, const double alpha[3], const cplx* r, cplx* out) {
    long M = npts(g);
    double amax = fmax(1.0, fmax(alpha[0], fmax(alpha[1], alpha[2])));
    double floor_ = 1e-12 * amax;   /* positivity guard; inactive for the trap and c0 used here */
    cplx* w = (cplx*)malloc(sizeof(cplx) * M);
    for (int c = 0; c < 3; ++c) {
        /* P_V^{1/2}: divide by sqrt(alpha_l + V + c0 rho) */
        for (long i = 0; i < M; ++i) {
            double rho = creal(phi[i] * conj(phi[i]) + phi[M + i] * conj(phi[M + i]) +
                               phi[2 * M + i] * conj(phi[2 * M + i]));
            double d = fmax(alpha[c] + pot_at(g, t, i) + p->c0 * rho, floor_);
            w[i] = r[c * M + i] / sqrt(d);
        }
        /* P_Delta: (alpha_l - Lap/2)^{-1}, diagonal in Fourier space */
        orc_fftn(g, w, -1);
        for (long i = 0; i < M; ++i) {
            double kx, ky, kz;
            kvec(g, i, &kx, &ky, &kz);
            w[i] /= fmax(alpha[c] + 0.5 * (kx * kx + ky * ky + kz * kz), floor_);
        }
        orc_fftn(g, w, +1);
        /* P_V^{1/2} again */
        for (long i = 0; i < M; ++i) {
            double rho = creal(phi[i] * conj(phi[i]) + phi[M + i] * conj(phi[M + i]) +
                               phi[2 * M + i] * conj(phi[2 * M + i]));
            double d = fmax(alpha[c] + pot_at(g, t, i) + p->c0 * rho, floor_);
            out[c * M + i] = w[i] / sqrt(d);
        }
    }
    free(w);
}

/* The three preconditioners of Sec. 3.4 by kind (ORC_PC_*), with the shifts
 * alpha_l of (3.13) for both the kinetic and the potential factor:
 *   kinetic   (3.12): (alpha_l - Lap/2)^{-1}, diagonal in Fourier space;
 *   potential (3.14): (alpha_l + V + c0 rho)^{-1}, pointwise;
 *   combined  (3.15): the potential factor's square root on both sides of the
 *                     kinetic one (orc_precond). */
void orc_precond_kind(const orc_grid* g, const orc_trap* t, const orc_params* p,
                      const cplx* phi, const double alpha[3], int kind, const cplx* r, cplx* out) {
    long M = npts(g);
    double amax = fmax(1.0, fmax(alpha[0], fmax(alpha[1], alpha[2])));
    double floor_ = 1e-12 * amax;
    if (kind == ORC_PC_COMBINED) {
        orc_precond(g, t, p, phi, alpha, r, out);
        return;
    }
    for (int c = 0; c < 3; ++c) {
        if (kind == ORC_PC_KINETIC) {
            memcpy(out + c * M, r + c * M, sizeof(cplx) * M);
            orc_fftn(g, out + c * M, -1);
            for (long i = 0; i < M; ++i) {
                double kx, ky, kz;
                kvec(g, i, &kx, &ky, &kz);
                out[c * M + i] /= fmax(alpha[c] + 0.5 * (kx * kx + ky * ky + kz * kz), floor_);
            }
            orc_fftn(g, out + c * M, +1);
        } else {
            for (long i = 0; i < M; ++i) {
                double rho = creal(phi[i] * conj(phi[i]) + phi[M + i] * conj(phi[M + i]) +
                                   phi[2 * M + i] * conj(phi[2 * M + i]));
                out[c * M + i] = r[c * M + i] / fmax(alpha[c] + pot_at(g, t, i) + p->c0 * rho, floor_);
            }
        }
    }
}

/* ------------------------------------------------------------------------- */
/* line search coefficients a_n, b_n, eqs. (3.6)-(3.8)                         */
/* ------------------------------------------------------------------------- */
/* conjugate bilinear forms F~_alpha(v, u) of Sec. 3.1 */
static void spin_bilinear(cplx v1, cplx v0, cplx vm, cplx u1, cplx u0, cplx um,
                          cplx* Fx, cplx* Fy, cplx* Fz) {
    const double s = 1.0 / sqrt(2.0);
    *Fx = s * (conj(u1) * v0 + conj(u0) * (v1 + vm) + conj(um) * v0);
    *Fy = I * s * (-conj(u1) * v0 + conj(u0) * (v1 - vm) + conj(um) * v0);
    *Fz = conj(u1) * v1 - conj(um) * vm;
}
/* a_n, b_n of the quadratic model E(theta) ~ a theta^2 + b theta + c for the
 * unnormalised direction P. H_l(P) in a_n is read as H with rho and F frozen
 * at Phi (the reading under which the expansion of E(cos t Phi + sin t P^) to
 * second order reproduces the printed coefficient). hphi = H(Phi)Phi. */
void orc_linesearch_coeffs(const orc_grid* g, const orc_trap* t, const orc_params* p,
                           const cplx* phi, const cplx* hphi, const cplx* P, double mu,
                           double* a, double* b) {
    long M = npts(g);
    double nP2 = orc_re_inner(g, P, P);
    cplx* hp = (cplx*)malloc(sizeof(cplx) * 3 * M);
    orc_apply_H_frozen(g, t, p, phi, P, hp);
    double t1 = orc_re_inner(g, hp, P);
    free(hp);
    double t2 = 0.0;
    for (long i = 0; i < M; ++i) {
        cplx v1 = phi[i], v0 = phi[M + i], vm = phi[2 * M + i];
        cplx u1 = P[i], u0 = P[M + i], um = P[2 * M + i];
        double rphip = creal(conj(v1) * u1 + conj(v0) * u0 + conj(vm) * um);  /* Re(Phi^dag P) */
        cplx Fx, Fy, Fz;
        spin_bilinear(v1, v0, vm, u1, u0, um, &Fx, &Fy, &Fz);
        t2 += p->c0 * rphip * rphip +
              p->c1 * (creal(Fx) * creal(Fx) + creal(Fy) * creal(Fy) + creal(Fz) * creal(Fz));
    }
    t2 *= cell(g);
    *a = -mu + t1 / nP2 + 2.0 * t2 / nP2;
    *b = 2.0 * orc_re_inner(g, hphi, P) / sqrt(nP2);
}

/* ------------------------------------------------------------------------- */
/* energy along the retraction, written explicitly in cos and sin (Sec. 3.1)  */
/* ------------------------------------------------------------------------- */
/* For Phi(t) = cos t Phi + sin t Ph (Ph = P/|P|) the energy (1.7) is
 *   E(t) = c^2 A + 2 c s B + s^2 C + c^4 e0 + 4 c^3 s e1 + c^2 s^2 e2 + 4 c s^3 e3 + s^4 e4,
 * c = cos t, s = sin t, with A = <H_L Phi, Phi>, B = Re<H_L Phi, Ph>, C = <H_L Ph, Ph>
 * (H_L linear and Hermitian) and e_j the integrals of the quartic terms: every
 * density q in (c0/2) rho^2 + (c1/2) sum_a F_a^2 is q(t) = c^2 q0 + 2 c s q1 + s^2 q2
 * (q0 = q(Phi), q1 = Re of the mixed form, q2 = q(Ph)), so q(t)^2 has coefficients
 * q0^2, 4 q0 q1, 2 q0 q2 + 4 q1^2, 4 q1 q2, q2^2. The change E(t) - E(0) is
 * returned with c^2 - 1 = -s^2 and c^4 - 1 = -s^2 (1 + c^2) so that it carries
 * no cancellation between the two energies. */
typedef struct { double A, B, C, e[5]; } orc_tpoly;

void orc_tpoly_coeffs(const orc_grid* g, const orc_trap* t, const orc_params* p,
                      const cplx* phi, const cplx* ph, orc_tpoly* q) {
    long M = npts(g), n3 = 3 * M;
    cplx* hl = (cplx*)malloc(sizeof(cplx) * n3);
    orc_apply_HL(g, t, p, phi, hl);
    q->A = orc_re_inner(g, hl, phi);
    q->B = orc_re_inner(g, hl, ph);
    orc_apply_HL(g, t, p, ph, hl);
    q->C = orc_re_inner(g, hl, ph);
    free(hl);
    double e[5] = {0, 0, 0, 0, 0};
    for (long i = 0; i < M; ++i) {
        cplx v1 = phi[i], v0 = phi[M + i], vm = phi[2 * M + i];
        cplx u1 = ph[i], u0 = ph[M + i], um = ph[2 * M + i];
        double r0 = creal(v1 * conj(v1) + v0 * conj(v0) + vm * conj(vm));
        double r1 = creal(conj(v1) * u1 + conj(v0) * u0 + conj(vm) * um);
        double r2 = creal(u1 * conj(u1) + u0 * conj(u0) + um * conj(um));
        double F0[3], F2[3];
        spin_vector(v1, v0, vm, &F0[0], &F0[1], &F0[2]);
        spin_vector(u1, u0, um, &F2[0], &F2[1], &F2[2]);
        cplx Fx, Fy, Fz;
        spin_bilinear(v1, v0, vm, u1, u0, um, &Fx, &Fy, &Fz);
        double F1[3] = {creal(Fx), creal(Fy), creal(Fz)};
        double w0 = 0.5 * p->c0, w1 = 0.5 * p->c1;
        e[0] += w0 * r0 * r0;
        e[1] += w0 * r0 * r1;
        e[2] += w0 * (2 * r0 * r2 + 4 * r1 * r1);
        e[3] += w0 * r1 * r2;
        e[4] += w0 * r2 * r2;
        for (int a = 0; a < 3; ++a) {
            e[0] += w1 * F0[a] * F0[a];
            e[1] += w1 * F0[a] * F1[a];
            e[2] += w1 * (2 * F0[a] * F2[a] + 4 * F1[a] * F1[a]);
            e[3] += w1 * F1[a] * F2[a];
            e[4] += w1 * F2[a] * F2[a];
        }
    }
    for (int j = 0; j < 5; ++j) q->e[j] = e[j] * cell(g);
}

double orc_tpoly_energy(const orc_tpoly* q, double theta) {
    double c = cos(theta), s = sin(theta);
    return c * c * q->A + 2 * c * s * q->B + s * s * q->C + c * c * c * c * q->e[0] +
           4 * c * c * c * s * q->e[1] + c * c * s * s * q->e[2] + 4 * c * s * s * s * q->e[3] +
           s * s * s * s * q->e[4];
}

double orc_tpoly_change(const orc_tpoly* q, double theta) {
    double c = cos(theta), s = sin(theta);
    return -s * s * q->A + 2 * c * s * q->B + s * s * q->C - s * s * (1 + c * c) * q->e[0] +
           4 * c * c * c * s * q->e[1] + c * c * s * s * q->e[2] + 4 * c * s * s * s * q->e[3] +
           s * s * s * s * q->e[4];
}

/* Exact line search along Phi(t) = cos t Phi + sin t Ph: the minimiser of the
 * explicit energy change over (0, pi/2]. Starting from t0 (halved until the
 * energy decreases, as in Algorithm 2), t is doubled while the energy keeps
 * decreasing, which brackets a minimum in [t/2... 2t]; golden-section search
 * then narrows the bracket to a relative width of 1e-12. Returns 0 when no
 * decrease was found within max_halvings halvings. */
double orc_exact_theta(const orc_tpoly* q, double t0, int max_halvings, int* halvings) {
    const double tmax = 1.5707963267948966;
    double t = fmin(t0, tmax);
    double f = orc_tpoly_change(q, t);
    int k = 0;
    while (!(f < 0.0)) {
        if (k >= max_halvings) { *halvings = k; return 0.0; }
        t *= 0.5;
        f = orc_tpoly_change(q, t);
        k++;
    }
    *halvings = k;
    /* bracket: lo < t < hi with f(t) below both ends (f(0) = 0 > f(t)) */
    double lo = 0.0, hi = fmin(2.0 * t, tmax);
    double fhi = orc_tpoly_change(q, hi);
    while (fhi < f && hi < tmax) {
        lo = t;
        t = hi;
        f = fhi;
        hi = fmin(2.0 * hi, tmax);
        fhi = orc_tpoly_change(q, hi);
    }
    if (fhi < f) return hi;   /* decreasing up to pi/2 */
    /* golden-section search on [lo, hi] */
    const double gr = 0.6180339887498949;
    double a = lo, b = hi;
    double x1 = b - gr * (b - a), x2 = a + gr * (b - a);
    double f1 = orc_tpoly_change(q, x1), f2 = orc_tpoly_change(q, x2);
    for (int it = 0; it < 200 && (b - a) > 1e-12 * b; ++it) {
        if (f1 < f2) {
            b = x2; x2 = x1; f2 = f1;
            x1 = b - gr * (b - a);
            f1 = orc_tpoly_change(q, x1);
        } else {
            a = x1; x1 = x2; f1 = f2;
            x2 = a + gr * (b - a);
            f2 = orc_tpoly_change(q, x2);
        }
    }
    double tm = f1 < f2 ? x1 : x2;
    double fm = f1 < f2 ? f1 : f2;
    return fm < f ? tm : t;
}

/* ------------------------------------------------------------------------- */
/* PCG, Algorithm 1 with the line search of Algorithm 2                      */
/* ------------------------------------------------------------------------- */
int orc_pcg(const orc_grid* g, const orc_trap* t, const orc_params* p, const orc_options* o,
            cplx* phi, orc_stats* st, double* etrace) {
    long M = npts(g), n3 = 3 * M;
    size_t bytes = sizeof(cplx) * n3;
    cplx* hphi = (cplx*)malloc(bytes);
    cplx* r = (cplx*)malloc(bytes);
    /* no previous residual or direction exists at n = 0 (beta = 0 there);
     * zero them so that 0 * P^{-1} is exactly 0 */
    cplx* r_prev = (cplx*)calloc((size_t)n3, sizeof(cplx));
    cplx* pr = (cplx*)malloc(bytes);
    cplx* D = (cplx*)malloc(bytes);
    cplx* P = (cplx*)malloc(bytes);
    cplx* P_prev = (cplx*)calloc((size_t)n3, sizeof(cplx));
    cplx* trial = (cplx*)malloc(bytes);
    memset(st, 0, sizeof(*st));
    int status = ORC_OK;
    normalise(g, phi);
    double E_cur = orc_energy(g, t, p, phi);
    if (etrace) etrace[0] = E_cur;
    double rpr_prev = 0.0;
    int n = 0;
    int use_e = (o->stop_kind == ORC_STOP_ENERGY || o->stop_kind == ORC_STOP_BOTH);
    int use_r = (o->stop_kind == ORC_STOP_RESIDUAL || o->stop_kind == ORC_STOP_BOTH);
    int use_w = (o->stop_kind == ORC_STOP_WAVEFN);
    for (;;) {
        if (!isfinite(E_cur)) { status = ORC_NONFINITE; break; }
        /* mu_n and the residual r^n */
        orc_apply_H(g, t, p, phi, hphi);
        double mu = orc_re_inner(g, hphi, phi);
        double rinf = 0.0;
        for (long i = 0; i < n3; ++i) {
            r[i] = hphi[i] - mu * phi[i];
            double a = cabs(r[i]);
            if (a > rinf) rinf = a;
        }
        st->resid_inf = rinf;
        if (use_r && rinf < o->tol) { status = ORC_OK; break; }
        if (n >= o->max_iter) { status = ORC_MAXITER; break; }
        /* preconditioned residual */
        double alpha[3];
        orc_alpha(g, t, p, phi, alpha);
        orc_precond_kind(g, t, p, phi, alpha, o->precond, r, pr);
        double rpr = orc_re_inner(g, r, pr);
        /* PRP beta, clipped at zero */
        double beta = 0.0;
        if (n > 0) {
            beta = (rpr - orc_re_inner(g, r_prev, pr)) / rpr_prev;
            if (beta < 0.0) beta = 0.0;
        }
        /* Algorithm 2, Steps 1-2: direction, projection, descent safeguard */
        double a = 0, b = 0, nP = 0;
        int stalled = 0;
        for (;;) {
            for (long i = 0; i < n3; ++i) D[i] = -pr[i] + beta * P_prev[i];
            double dphi = orc_re_inner(g, D, phi);
            for (long i = 0; i < n3; ++i) P[i] = D[i] - dphi * phi[i];
            nP = sqrt(orc_re_inner(g, P, P));
            if (!(nP > 0.0)) { stalled = 1; break; }
            orc_linesearch_coeffs(g, t, p, phi, hphi, P, mu, &a, &b);
            if (b > 0.0 || (b == 0.0 && a >= 0.0)) {
                if (beta != 0.0) { beta = 0.0; st->resets++; continue; }
                stalled = 1;   /* steepest-descent direction does not descend: rounding floor */
            }
            break;
        }
        if (stalled) { status = ORC_STAGNATED; break; }
        double theta = (a > 0.0 && b < 0.0) ? -b / (2.0 * a) : o->theta_trial;
        /* Steps 3-4: accept when the energy decreases, else shrink theta. The
         * change E(theta) - E(0) comes from the explicit form in cos/sin. */
        for (long i = 0; i < n3; ++i) trial[i] = P[i] / nP;
        orc_tpoly tp;
        orc_tpoly_coeffs(g, t, p, phi, trial, &tp);
        int accepted = 0;
        double dE = 0.0;
        if (o->exact_ls) {
            int nh = 0;
            theta = orc_exact_theta(&tp, theta, o->max_backtrack, &nh);
            st->backtracks += nh;
            if (theta > 0.0) {
                dE = orc_tpoly_change(&tp, theta);
                accepted = dE < 0.0;
            }
        } else {
            for (int k = 0; k <= o->max_backtrack; ++k) {
                dE = orc_tpoly_change(&tp, theta);
                if (dE < 0.0) { accepted = 1; break; }
                theta *= o->sigma;
                st->backtracks++;
            }
        }
        if (!accepted || !isfinite(dE)) { status = ORC_STAGNATED; break; }
        double cs = cos(theta), sn = sin(theta);
        for (long i = 0; i < n3; ++i) trial[i] = cs * phi[i] + sn * trial[i];
        normalise(g, trial);
        /* criterion (3.9): max over components and points of |phi^{n+1} - phi^n| */
        double werr = 0.0;
        for (long i = 0; i < n3; ++i) {
            double a = cabs(trial[i] - phi[i]);
            if (a > werr) werr = a;
        }
        memcpy(phi, trial, bytes);
        E_cur = orc_energy(g, t, p, phi);
        memcpy(r_prev, r, bytes);
        memcpy(P_prev, P, bytes);
        rpr_prev = rpr;
        n++;
        st->dE_last = dE;
        if (etrace) etrace[n] = E_cur;
        if (use_e && fabs(dE) < o->tol) { status = ORC_OK; break; }
        if (use_w && werr < o->tol) { status = ORC_OK; break; }
    }
    st->iters = n;
    st->status = status;
    free(hphi); free(r); free(r_prev); free(pr); free(D); free(P); free(P_prev); free(trial);
    return status;
}

/* ------------------------------------------------------------------------- */
/* cascadic multigrid interpolation (Sec. 3.3, Algorithm 3)                   */
/* ------------------------------------------------------------------------- */
/* Trigonometric interpolation of a coarse-grid field onto a finer grid on the
 * same domain: the coarse spectrum is copied to the same wavenumbers of the
 * fine spectrum (the coarse mode -N/2 is split equally between +-N/2), the
 * rest is zero, and the result is transformed back. The fine grid contains
 * the coarse points, where the interpolant reproduces the coarse values. */
static double interp_weight(int jf, int nf, int nc, int* jc) {
    int p = (jf < nf / 2) ? jf : jf - nf;
    if (p > -nc / 2 && p < nc / 2) { *jc = (p + nc) % nc; return 1.0; }
    if (p == nc / 2 || p == -nc / 2) { *jc = nc / 2; return (nf == nc) ? 1.0 : 0.5; }
    *jc = 0;
    return 0.0;
}
int orc_interp(const orc_grid* gc, const cplx* in, const orc_grid* gf, cplx* out) {
    long Mc = npts(gc), Mf = npts(gf);
    int d = gc->dim;
    for (int a = 0; a < d; ++a)
        if (gf->n[a] < gc->n[a] || gf->L[a] != gc->L[a]) return ORC_EINVAL;
    cplx* ch = spectra(gc, in);
    double scale = (double)Mf / (double)Mc;
    for (int c = 0; c < 3; ++c) {
        for (long i = 0; i < Mf; ++i) {
            int jx, jy, jz, cx, cy, cz = 0;
            unpack(gf, i, &jx, &jy, &jz);
            double w = interp_weight(jx, gf->n[0], gc->n[0], &cx) *
                       interp_weight(jy, gf->n[1], gc->n[1], &cy);
            if (d == 3) w *= interp_weight(jz, gf->n[2], gc->n[2], &cz);
            long ic = ((long)cz * gc->n[1] + cy) * gc->n[0] + cx;
            out[c * Mf + i] = w == 0.0 ? 0.0 : scale * w * ch[c * Mc + ic];
        }
        orc_fftn(gf, out + c * Mf, +1);
    }
    free(ch);
    return ORC_OK;
}
