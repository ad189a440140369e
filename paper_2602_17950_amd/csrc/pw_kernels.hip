// Pointwise kernels of the PCG iteration with fused FP64 reductions and the
// device-side control logic of Algorithms 1 and 2 of the paper.
//
// Every reducing kernel writes one row of per-block partial sums; the last
// block to finish (completion counter) sums the rows in a fixed order and runs
// the scalar part of the iteration on thread 0, writing SolveState. The grid
// size depends only on the number of grid points, so the reduction order, and
// with it every scalar, is reproducible run to run.
#include "gs_internal.h"
#include "../../include/gs.h"

namespace gs {

constexpr int PT = 256;   // threads per block of the pointwise kernels

int pw_blocks(long long M) {
    long long b = (M + PT - 1) / PT;
    return (int)(b < 2048 ? b : 2048);
}

template <int NV>
__device__ __forceinline__ void bsum(double (&v)[NV]) {
    __shared__ double sh[PT / 64][NV];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[wv][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < PT / 64; ++w) s += sh[w][k];
            v[k] = s;
        }
    __syncthreads();
}

__device__ __forceinline__ double bmax(double v) {
    __shared__ double sh[PT / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = sh[0];
        for (int w = 1; w < PT / 64; ++w) m = fmax(m, sh[w]);
        v = m;
    }
    __syncthreads();
    return v;
}

// Write this block's partials, then report whether it is the last block of the grid.
template <int NV>
__device__ __forceinline__ bool publish(const double (&v)[NV], double* rows, unsigned* counter) {
    __shared__ int last;
    if (threadIdx.x == 0) {
        for (int k = 0; k < NV; ++k) rows[(long long)blockIdx.x * NS_MAX + k] = v[k];
        __threadfence();
        const unsigned prev = atomicAdd(counter, 1u);
        last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (last) __threadfence();
    return last != 0;
}

// In the last block: totals over all rows (fixed order), available on thread 0.
template <int NV>
__device__ __forceinline__ void gather(double (&tot)[NV], const double* rows, int nrows, int stride) {
    for (int k = 0; k < NV; ++k) tot[k] = 0.0;
    const volatile double* vr = rows;
    for (int b = threadIdx.x; b < nrows; b += PT)
        for (int k = 0; k < NV; ++k) tot[k] += vr[(long long)b * stride + k];
    bsum<NV>(tot);
}

__device__ __forceinline__ void coords(const Phys& p, long long i, double& x, double& y, double& z) {
    const int nx = p.n[0], ny = p.n[1];
    const long long ix = i % nx, iy = (i / nx) % ny, iz = i / ((long long)nx * ny);
    x = -p.L[0] + ix * p.h[0];
    y = -p.L[1] + iy * p.h[1];
    z = p.dim == 3 ? -p.L[2] + iz * p.h[2] : 0.0;
}

// Nonlinear part of H(Phi)Phi (Euler-Lagrange equations (2.6)-(2.8)) in the
// compact form c0 rho phi + c1 (F.f) phi with G = conj(phi_1) phi_0 +
// conj(phi_0) phi_-1 and F_z = |phi_1|^2 - |phi_-1|^2:
//   (F.f)u = (F_z u1 + conj(G) u0, G u1 + conj(G) u-1, G u0 - F_z u-1).
struct Spin {
    double rho, rho_c[3], Fz;
    cpx<double> G;
};
__device__ __forceinline__ Spin spin_of(const cpx<double> (&f)[3]) {
    Spin s;
    s.rho_c[0] = cabs2(f[0]);
    s.rho_c[1] = cabs2(f[1]);
    s.rho_c[2] = cabs2(f[2]);
    s.rho = s.rho_c[0] + s.rho_c[1] + s.rho_c[2];
    s.Fz = s.rho_c[0] - s.rho_c[2];
    s.G = cmul(cconj(f[0]), f[1]) + cmul(cconj(f[1]), f[2]);
    return s;
}
__device__ __forceinline__ void nonlin(const Phys& p, const Spin& s, const cpx<double> (&u)[3],
                                       cpx<double> (&out)[3]) {
    const cpx<double> Gc = cconj(s.G);
    out[0] = p.c0 * s.rho * u[0] + p.c1 * (s.Fz * u[0] + cmul(Gc, u[1]));
    out[1] = p.c0 * s.rho * u[1] + p.c1 * (cmul(s.G, u[0]) + cmul(Gc, u[2]));
    out[2] = p.c0 * s.rho * u[2] + p.c1 * (cmul(s.G, u[1]) - s.Fz * u[2]);
}

template <typename R>
__device__ __forceinline__ void load3(const cpx<R>* f, long long i, long long M, cpx<double> (&v)[3]) {
    v[0] = wid(f[i]);
    v[1] = wid(f[M + i]);
    v[2] = wid(f[2 * M + i]);
}

__device__ __forceinline__ double re_dot(const cpx<double>& a, const cpx<double>& b) { return a.x * b.x + a.y * b.y; }

// ---------------------------------------------------------------------------
// evaluation of the current iterate: energy parts, mu, alpha_l (after H_L Phi)
// ---------------------------------------------------------------------------
constexpr int NS_EVAL = 18;

__device__ void ctrl_eval(SolveState* st, const Phys& p, const double (&s)[NS_EVAL], const double (&m)[4]) {
    const double hd = p.cell, kM = hd / (double)p.M;
    double Nc[3], K[3];
    for (int c = 0; c < 3; ++c) {
        Nc[c] = s[c] * hd;
        K[c] = m[c] * kM;
        st->norm_comp[c] = Nc[c];
        st->alpha[c] = K[c] + (s[3 + c] + s[6 + c]) * hd;    // eq. (3.13)
        st->mu_comp[c] = (s[9 + c] + s[12 + c]) * hd / Nc[c];
    }
    st->norm2 = Nc[0] + Nc[1] + Nc[2];
    st->e_kin = K[0] + K[1] + K[2];
    st->e_pot = (s[3] + s[4] + s[5]) * hd;
    st->e_pot4 = s[17] * hd;
    st->e_pot2 = st->e_pot - st->e_pot4;
    st->e_soc = -p.gamma * m[3] * kM;
    st->lin = (s[9] + s[10] + s[11]) * hd;
    st->e_spin = (s[15] + s[16]) * hd;
    st->E = st->lin + st->e_spin;
    st->e_rot = st->lin - st->e_kin - st->e_pot - st->e_soc;
    st->mu = (s[9] + s[10] + s[11] + s[12] + s[13] + s[14]) * hd;   // eq. (2.9)
    st->virial = p.V ? __builtin_nan("") :
                 2.0 * st->e_kin - 2.0 * st->e_pot2 - 4.0 * st->e_pot4 + p.dim * st->e_spin + st->e_soc;
    st->pending_step = 0;
    if (!isfinite(st->E) || !isfinite(st->mu)) {
        st->nonfinite = 1;
        st->status = GS_ENONFINITE;
        st->done = 1;
    }
}

template <typename R>
__global__ __launch_bounds__(PT) void k_eval(Fields<R> f, Phys p, SolveState* st, RedBuf rb) {
    if (st->done) return;
    const long long M = p.M;
    double acc[NS_EVAL];
    for (int k = 0; k < NS_EVAL; ++k) acc[k] = 0.0;
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < M; i += (long long)gridDim.x * PT) {
        double x, y, z, V2, V4;
        coords(p, i, x, y, z);
        trap_at(p, i, x, y, z, V2, V4);
        cpx<double> ph[3], hl[3], nl[3];
        load3(f.phi, i, M, ph);
        load3(f.hl, i, M, hl);
        const Spin sp = spin_of(ph);
        nonlin(p, sp, ph, nl);
        for (int c = 0; c < 3; ++c) {
            acc[c] += sp.rho_c[c];
            acc[3 + c] += (V2 + V4) * sp.rho_c[c];
            acc[6 + c] += p.c0 * sp.rho * sp.rho_c[c];
            acc[9 + c] += re_dot(hl[c], ph[c]);
            acc[12 + c] += re_dot(nl[c], ph[c]);
        }
        acc[15] += 0.5 * p.c0 * sp.rho * sp.rho;
        acc[16] += 0.5 * p.c1 * (2.0 * cabs2(sp.G) + sp.Fz * sp.Fz);   // |F|^2 = 2|G|^2 + F_z^2
        acc[17] += V4 * sp.rho;
    }
    bsum<NS_EVAL>(acc);
    if (publish<NS_EVAL>(acc, rb.pw, rb.counter + 0)) {
        double tot[NS_EVAL], mt[4];
        gather<NS_EVAL>(tot, rb.pw, gridDim.x, NS_MAX);
        gather<4>(mt, rb.mid, rb.nblk_mid, 4);
        if (threadIdx.x == 0) {
            ctrl_eval(st, p, tot, mt);
            rb.counter[0] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// residual r = H(Phi)Phi - mu Phi, preconditioner factors and input
// ---------------------------------------------------------------------------
__device__ void ctrl_resid(SolveState* st, double rinf) {
    st->resid_inf = rinf;
    if (!isfinite(rinf)) { st->nonfinite = 1; st->status = GS_ENONFINITE; st->done = 1; return; }
    if (st->final_pending) { st->done = 1; return; }
    if (st->stop_kind != GS_STOP_ENERGY && rinf < st->tol) { st->done = 1; return; }   // criterion (3.10)
    if (st->iter >= st->max_iter) { st->status = GS_WMAXITER; st->done = 1; return; }
    if (st->phase == PH_FP32) {
        if (rinf < st->switch_resid) { st->switch_req = 1; st->done = 1; return; }
        if (rinf < 0.5 * st->best_resid) { st->best_resid = rinf; st->best_iter = st->iter_phase; }
        else if (st->iter_phase - st->best_iter >= st->stall_window) { st->switch_req = 1; st->done = 1; return; }
        if (st->iter_phase >= st->phase_max_iter) { st->switch_req = 1; st->done = 1; return; }
    }
}

template <typename R>
__global__ __launch_bounds__(PT) void k_resid(Fields<R> f, Phys p, SolveState* st, RedBuf rb) {
    if (st->done) return;
    const long long M = p.M;
    const double mu = st->mu;
    const double al[3] = {st->alpha[0], st->alpha[1], st->alpha[2]};
    const double fl = 1e-12 * fmax(1.0, fmax(al[0], fmax(al[1], al[2])));
    cpx<R>* r = f.r[st->cur];
    double rinf = 0.0;
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < M; i += (long long)gridDim.x * PT) {
        double x, y, z, V2, V4;
        coords(p, i, x, y, z);
        trap_at(p, i, x, y, z, V2, V4);
        cpx<double> ph[3], hl[3], nl[3];
        load3(f.phi, i, M, ph);
        load3(f.hl, i, M, hl);
        const Spin sp = spin_of(ph);
        nonlin(p, sp, ph, nl);
        for (int c = 0; c < 3; ++c) {
            const cpx<double> rc = hl[c] + nl[c] - mu * ph[c];
            const cpx<R> rr = cmk((R)rc.x, (R)rc.y);
            rinf = fmax(rinf, sqrt(cabs2(rc)));
            r[c * M + i] = rr;
            // P_V^{1/2} = (alpha_l + V + c0 rho)^{-1/2}, eq. (3.14)
            const double d = fmax(al[c] + V2 + V4 + p.c0 * sp.rho, fl);
            const R w = (R)(1.0 / sqrt(d));
            f.pv[c * M + i] = w;
            f.u[c * M + i] = w * rr;
        }
    }
    double v[1] = {bmax(rinf)};
    if (publish<1>(v, rb.pw, rb.counter + 1)) {
        double m = 0.0;
        const volatile double* vr = rb.pw;
        for (int b = threadIdx.x; b < (int)gridDim.x; b += PT) m = fmax(m, vr[(long long)b * NS_MAX]);
        m = bmax(m);
        if (threadIdx.x == 0) {
            ctrl_resid(st, m);
            rb.counter[1] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// direction scalars: PRP beta, projection, |P|, descent test (Algorithm 2, Steps 1-2)
// ---------------------------------------------------------------------------
constexpr int NS_DIR = 8;

__device__ void stop_stagnated(SolveState* st) {
    if (st->phase == PH_FP32) st->switch_req = 1;
    else st->status = GS_WSTAGNATED;
    st->done = 1;
}

__device__ void ctrl_dir(SolveState* st, const Phys& p, const double (&s)[NS_DIR]) {
    const double h = p.cell;
    const double rpr = s[0] * h, rprp = s[1] * h, phipr = s[2] * h, prpr = s[3] * h;
    double prP = s[4] * h, rP = s[5] * h, phiP = s[6] * h, PP = s[7] * h;
    if (!st->have_prev) { prP = rP = phiP = PP = 0.0; }
    const double mu = st->mu;
    double beta = 0.0;
    if (st->have_prev) {
        beta = (rpr - rprp) / st->rpr_prev;      // Polak-Ribiere-Polyak
        if (!(beta > 0.0)) beta = 0.0;
    }
    double dphi = 0.0, nP2 = 0.0, bdir = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        dphi = -phipr + beta * phiP;                              // Re<D, Phi>
        const double DD = prpr - 2.0 * beta * prP + beta * beta * PP;
        nP2 = DD - 2.0 * dphi * dphi + dphi * dphi * st->norm2;   // |D - Re<D,Phi> Phi|^2
        // Re<H Phi, P> with H Phi = r + mu Phi and Re<H Phi, Phi> = mu
        const double HD = -(rpr + mu * phipr) + beta * (rP + mu * phiP);
        const double HP = HD - dphi * mu;
        bdir = nP2 > 0.0 ? 2.0 * HP / sqrt(nP2) : 0.0;
        if (nP2 > 0.0 && bdir < 0.0) break;
        if (beta != 0.0) { beta = 0.0; st->resets++; continue; }   // switch to steepest descent
        stop_stagnated(st);
        return;
    }
    if (!(nP2 > 0.0) || !(bdir < 0.0)) { stop_stagnated(st); return; }
    st->rpr = rpr;
    st->beta = beta;
    st->dphi = dphi;
    st->nP = sqrt(nP2);
    st->invnP = 1.0 / st->nP;
    st->bdir = bdir;
}

template <typename R>
__global__ __launch_bounds__(PT) void k_dirred(Fields<R> f, Phys p, SolveState* st, RedBuf rb) {
    if (st->done) return;
    const long long M = p.M;
    const cpx<R>* r = f.r[st->cur];
    const cpx<R>* rp = f.r[st->cur ^ 1];
    double acc[NS_DIR];
    for (int k = 0; k < NS_DIR; ++k) acc[k] = 0.0;
    const long long n3 = 3 * M;
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < n3; i += (long long)gridDim.x * PT) {
        const cpx<double> ri = wid(r[i]), rpi = wid(rp[i]), ph = wid(f.phi[i]), pr = wid(f.pr[i]), P = wid(f.P[i]);
        acc[0] += re_dot(ri, pr);
        acc[1] += re_dot(rpi, pr);
        acc[2] += re_dot(ph, pr);
        acc[3] += re_dot(pr, pr);
        acc[4] += re_dot(pr, P);
        acc[5] += re_dot(ri, P);
        acc[6] += re_dot(ph, P);
        acc[7] += re_dot(P, P);
    }
    bsum<NS_DIR>(acc);
    if (publish<NS_DIR>(acc, rb.pw, rb.counter + 2)) {
        double tot[NS_DIR];
        gather<NS_DIR>(tot, rb.pw, gridDim.x, NS_MAX);
        if (threadIdx.x == 0) {
            ctrl_dir(st, p, tot);
            rb.counter[2] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// step size (Algorithm 2, Steps 2-4) from the exact energy along the retraction
// ---------------------------------------------------------------------------
// Along Phi(t) = cos t Phi + sin t P^ the linear part of the energy is
// cos^2 <H_L Phi,Phi> + 2 cos sin Re<H_L Phi,P^> + sin^2 <H_L P^,P^>, and rho
// and each F_a are cos^2 q0 + 2 cos sin q1 + sin^2 q2 pointwise. With
// d = sin^2 (q2 - q0) + 2 cos sin q1, q(t)^2 - q0^2 = 2 q0 d + d^2, so
// E(t) - E(0) is a trigonometric polynomial in five integrals per density:
//   I01 = w q0 q1, I02 = w q0 (q2 - q0), I11 = w q1^2, I21 = w (q2 - q0) q1, I22 = w (q2 - q0)^2
// (w = c0/2 for rho, c1/2 for each F_a), summed over rho, F_x, F_y, F_z.
// Its second-order expansion gives a_n and b_n of eqs. (3.7)-(3.8).
constexpr int NS_LS = 9;

__device__ __forceinline__ double dE_at(double c, double s, double CmA, double B, const double (&I)[5]) {
    return s * s * CmA + 2.0 * c * s * B + 2.0 * s * s * I[1] + 4.0 * c * s * I[0] + s * s * s * s * I[4] +
           4.0 * c * s * s * s * I[3] + 4.0 * c * c * s * s * I[2];
}

__device__ void ctrl_ls(SolveState* st, const Phys& p, const double (&s)[NS_LS]) {
    const double h = p.cell;
    const double Cq = s[0] * h, B = s[1] * h, PhPh = s[2] * h, phiPh = s[3] * h;
    const double I[5] = {s[4] * h, s[5] * h, s[6] * h, s[7] * h, s[8] * h};
    const double CmA = Cq - st->lin;
    const double a = CmA + 2.0 * I[1] + 4.0 * I[2];
    const double b = 2.0 * B + 4.0 * I[0];
    st->a = a;
    st->b = b;
    double theta = (a > 0.0 && b < 0.0) ? -b / (2.0 * a) : st->theta_trial;
    int accepted = 0;
    double dE = 0.0, c = 1.0, sn = 0.0;
    for (int k = 0; k <= st->max_backtrack; ++k) {
        c = cos(theta);
        sn = sin(theta);
        dE = dE_at(c, sn, CmA, B, I);
        if (dE < 0.0) { accepted = 1; break; }   // the energy decreases
        theta *= st->sigma;
        st->backtracks++;
    }
    if (!accepted || !isfinite(dE)) { stop_stagnated(st); return; }
    st->theta = theta;
    st->c = c;
    st->s = sn;
    st->dE = dE;
    st->dE_last = dE;
    const double n2 = c * c * st->norm2 + 2.0 * c * sn * phiPh + sn * sn * PhPh;
    st->inv_norm = 1.0 / sqrt(n2);
    st->pending_step = 1;
    st->iter++;
    st->iter_phase++;
    st->rpr_prev = st->rpr;
    st->have_prev = 1;
    st->cur ^= 1;
    if (st->stop_kind != GS_STOP_RESIDUAL && fabs(dE) < st->tol) st->final_pending = 1;   // criterion (3.11)
}

// Re(v^dag f_a u) for the spin-1 matrices f_x, f_y, f_z (Sec. 1)
__device__ __forceinline__ void spin_bil(const cpx<double> (&v)[3], const cpx<double> (&u)[3], double (&F)[3]) {
    const double r2 = 0.70710678118654752440;
    // v^dag f_x u = (conj v1 u0 + conj v0 (u1 + u-1) + conj v-1 u0) / sqrt2
    const cpx<double> tx = cmul(cconj(v[0]), u[1]) + cmul(cconj(v[1]), u[0] + u[2]) + cmul(cconj(v[2]), u[1]);
    // v^dag f_y u = i (-conj v1 u0 + conj v0 (u1 - u-1) + conj v-1 u0) / sqrt2
    const cpx<double> ty = cmul(cconj(v[2]), u[1]) - cmul(cconj(v[0]), u[1]) + cmul(cconj(v[1]), u[0] - u[2]);
    F[0] = r2 * tx.x;
    F[1] = -r2 * ty.y;   // Re(i t) = -Im t
    F[2] = re_dot(v[0], u[0]) - re_dot(v[2], u[2]);
}

template <typename R>
__global__ __launch_bounds__(PT) void k_lsred(Fields<R> f, Phys p, SolveState* st, RedBuf rb) {
    if (st->done) return;
    const long long M = p.M;
    const double ip = st->invnP;
    const double w0 = 0.5 * p.c0, w1 = 0.5 * p.c1;
    double acc[NS_LS];
    for (int k = 0; k < NS_LS; ++k) acc[k] = 0.0;
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < M; i += (long long)gridDim.x * PT) {
        cpx<double> ph[3], P[3], hl[3], hp[3];
        load3(f.phi, i, M, ph);
        load3(f.P, i, M, P);
        load3(f.hl, i, M, hl);
        load3(f.hlp, i, M, hp);
        for (int c = 0; c < 3; ++c) P[c] = ip * P[c];
        double q1r = 0.0, q0r = 0.0, q2r = 0.0;
        for (int c = 0; c < 3; ++c) {
            acc[0] += re_dot(hp[c], P[c]);
            acc[1] += re_dot(hl[c], P[c]);
            acc[2] += cabs2(P[c]);
            acc[3] += re_dot(ph[c], P[c]);
            q0r += cabs2(ph[c]);
            q1r += re_dot(ph[c], P[c]);
            q2r += cabs2(P[c]);
        }
        double F0[3], F1[3], F2[3];
        spin_bil(ph, ph, F0);
        spin_bil(ph, P, F1);
        spin_bil(P, P, F2);
        {
            const double d = q2r - q0r;
            acc[4] += w0 * q0r * q1r;
            acc[5] += w0 * q0r * d;
            acc[6] += w0 * q1r * q1r;
            acc[7] += w0 * d * q1r;
            acc[8] += w0 * d * d;
        }
        for (int a = 0; a < 3; ++a) {
            const double d = F2[a] - F0[a];
            acc[4] += w1 * F0[a] * F1[a];
            acc[5] += w1 * F0[a] * d;
            acc[6] += w1 * F1[a] * F1[a];
            acc[7] += w1 * d * F1[a];
            acc[8] += w1 * d * d;
        }
    }
    bsum<NS_LS>(acc);
    if (publish<NS_LS>(acc, rb.pw, rb.counter + 3)) {
        double tot[NS_LS];
        gather<NS_LS>(tot, rb.pw, gridDim.x, NS_MAX);
        if (threadIdx.x == 0) {
            ctrl_ls(st, p, tot);
            rb.counter[3] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// normalisation: sets the pending rescale Phi <- Phi / |Phi|
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(PT) void k_normalize(const cpx<R>* phi, Phys p, SolveState* st, RedBuf rb) {
    const long long n3 = 3 * p.M;
    double acc[1] = {0.0};
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < n3; i += (long long)gridDim.x * PT)
        acc[0] += cabs2(wid(phi[i]));
    bsum<1>(acc);
    if (publish<1>(acc, rb.pw, rb.counter + 4)) {
        double tot[1];
        gather<1>(tot, rb.pw, gridDim.x, NS_MAX);
        if (threadIdx.x == 0) {
            const double n2 = tot[0] * p.cell;
            if (!(n2 > 0.0) || !isfinite(n2)) {
                st->nonfinite = 1;
                st->status = GS_ENONFINITE;
                st->done = 1;
            } else {
                st->c = 1.0 / sqrt(n2);
                st->s = 0.0;
                st->inv_norm = 1.0;
                st->pending_step = 1;
            }
            rb.counter[4] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------
__global__ void k_d2f(const cpx<double>* in, cpx<float>* out, long long n) {
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < n; i += (long long)gridDim.x * PT)
        out[i] = cmk((float)in[i].x, (float)in[i].y);
}
__global__ void k_f2d(const cpx<float>* in, cpx<double>* out, long long n) {
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < n; i += (long long)gridDim.x * PT)
        out[i] = cmk((double)in[i].x, (double)in[i].y);
}

template <typename R>
__global__ void k_hphi(const cpx<R>* phi, const cpx<R>* hl, cpx<R>* out, Phys p) {
    const long long M = p.M;
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < M; i += (long long)gridDim.x * PT) {
        cpx<double> ph[3], h[3], nl[3];
        load3(phi, i, M, ph);
        load3(hl, i, M, h);
        const Spin sp = spin_of(ph);
        nonlin(p, sp, ph, nl);
        for (int c = 0; c < 3; ++c) {
            const cpx<double> v = h[c] + nl[c];
            out[c * M + i] = cmk((R)v.x, (R)v.y);
        }
    }
}

template <typename R>
__global__ void k_pv_apply(const R* pv, const cpx<R>* r, cpx<R>* out, long long n3) {
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < n3; i += (long long)gridDim.x * PT)
        out[i] = pv[i] * r[i];
}

// (a, a, a)/sqrt(3) with phi_a = pi^{-d/4} exp(-|x|^2/2) (Sec. 4, guess (a))
__global__ void k_gaussian(cpx<double>* out, Phys p) {
    const long long M = p.M;
    const double amp = pow(3.141592653589793238462643, -0.25 * p.dim) / sqrt(3.0);
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < M; i += (long long)gridDim.x * PT) {
        double x, y, z;
        coords(p, i, x, y, z);
        const double v = amp * exp(-0.5 * (x * x + y * y + z * z));
        for (int c = 0; c < 3; ++c) out[c * M + i] = cmk(v, 0.0);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename R> hipError_t launch_eval(const Fields<R>& f, const Phys& p, SolveState* st, RedBuf rb, hipStream_t s) {
    GS_LAUNCH(k_eval<R>, dim3(rb.nblk_pw), dim3(PT), 0, s, f, p, st, rb);
    return hipGetLastError();
}
template <typename R> hipError_t launch_resid(const Fields<R>& f, const Phys& p, SolveState* st, RedBuf rb, hipStream_t s) {
    GS_LAUNCH(k_resid<R>, dim3(rb.nblk_pw), dim3(PT), 0, s, f, p, st, rb);
    return hipGetLastError();
}
template <typename R> hipError_t launch_dirred(const Fields<R>& f, const Phys& p, SolveState* st, RedBuf rb, hipStream_t s) {
    GS_LAUNCH(k_dirred<R>, dim3(rb.nblk_pw), dim3(PT), 0, s, f, p, st, rb);
    return hipGetLastError();
}
template <typename R> hipError_t launch_lsred(const Fields<R>& f, const Phys& p, SolveState* st, RedBuf rb, hipStream_t s) {
    GS_LAUNCH(k_lsred<R>, dim3(rb.nblk_pw), dim3(PT), 0, s, f, p, st, rb);
    return hipGetLastError();
}
template <typename R> hipError_t launch_normalize(const cpx<R>* phi, const Phys& p, SolveState* st, RedBuf rb, hipStream_t s) {
    GS_LAUNCH(k_normalize<R>, dim3(rb.nblk_pw), dim3(PT), 0, s, phi, p, st, rb);
    return hipGetLastError();
}
hipError_t launch_convert_d2f(const cpx<double>* in, cpx<float>* out, long long n, hipStream_t s) {
    GS_LAUNCH(k_d2f, dim3(pw_blocks(n)), dim3(PT), 0, s, in, out, n);
    return hipGetLastError();
}
hipError_t launch_convert_f2d(const cpx<float>* in, cpx<double>* out, long long n, hipStream_t s) {
    GS_LAUNCH(k_f2d, dim3(pw_blocks(n)), dim3(PT), 0, s, in, out, n);
    return hipGetLastError();
}
template <typename R> hipError_t launch_hphi(const cpx<R>* phi, const cpx<R>* hl, cpx<R>* out, const Phys& p, hipStream_t s) {
    GS_LAUNCH(k_hphi<R>, dim3(pw_blocks(p.M)), dim3(PT), 0, s, phi, hl, out, p);
    return hipGetLastError();
}
template <typename R> hipError_t launch_pv_apply(const R* pv, const cpx<R>* r, cpx<R>* out, long long n3, hipStream_t s) {
    GS_LAUNCH(k_pv_apply<R>, dim3(pw_blocks(n3)), dim3(PT), 0, s, pv, r, out, n3);
    return hipGetLastError();
}
hipError_t launch_gaussian(cpx<double>* out, const Phys& p, hipStream_t s) {
    GS_LAUNCH(k_gaussian, dim3(pw_blocks(p.M)), dim3(PT), 0, s, out, p);
    return hipGetLastError();
}

#define GS_INST(R)                                                                                          \
    template hipError_t launch_eval<R>(const Fields<R>&, const Phys&, SolveState*, RedBuf, hipStream_t);    \
    template hipError_t launch_resid<R>(const Fields<R>&, const Phys&, SolveState*, RedBuf, hipStream_t);   \
    template hipError_t launch_dirred<R>(const Fields<R>&, const Phys&, SolveState*, RedBuf, hipStream_t);  \
    template hipError_t launch_lsred<R>(const Fields<R>&, const Phys&, SolveState*, RedBuf, hipStream_t);   \
    template hipError_t launch_normalize<R>(const cpx<R>*, const Phys&, SolveState*, RedBuf, hipStream_t);  \
    template hipError_t launch_hphi<R>(const cpx<R>*, const cpx<R>*, cpx<R>*, const Phys&, hipStream_t); \
    template hipError_t launch_pv_apply<R>(const R*, const cpx<R>*, cpx<R>*, long long, hipStream_t);
GS_INST(double)
GS_INST(float)

}  // namespace gs
