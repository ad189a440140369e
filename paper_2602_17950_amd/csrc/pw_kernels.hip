// Pointwise kernels of the PCG iteration with fused FP64 reductions, and the
// control kernel.
//
// Every reducing kernel writes one row of per-block partial sums with plain
// stores. A following control kernel (one block per slot) sums the rows in a
// fixed order and runs the scalar part of the iteration (control.h) on thread
// 0; the kernel boundary between them makes the rows visible, so no block
// needs a device-wide fence. The grid size depends only on the number of grid
// points, so the reduction order, and with it every scalar, is the same run to
// run and whatever other slots share the launch.
#include "device_common.h"
#include "control.h"

namespace gs {

// blocks per slot of the pointwise passes (= partial-sum rows): two points per
// thread, so that a block's reduction is shared by 512 points, but at least
// min(M/256, 64) blocks for small grids, and at most 2048
int pw_blocks(long long M) {
    long long b = (M + 512 - 1) / 512;
    const long long lo = std::min<long long>((M + PT - 1) / PT, 64);
    b = std::max(b, lo);
    return (int)(b < 2048 ? b : 2048);
}

// ---------------------------------------------------------------------------
// fresh evaluation after an H_L application: energy parts, mu (2.9), alpha_l
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(PT) void k_eval(const Slot* slots, RedGeom g) {
    const Slot& S = slots[blockIdx.y];
    SolveState* st = as_global(S.st);
    if (st->done) return;
    const Phys p = S.p;
    const long long M = p.M;
    const cpx<R>* phi = fld<R>(S, B_PHI);
    const cpx<R>* hlf = fld<R>(S, B_HL);
    double acc[NS_EVAL];
    for (int k = 0; k < NS_EVAL; ++k) acc[k] = 0.0;
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < M; i += (long long)gridDim.x * PT) {
        double x, y, z, V2, V4;
        coords(p, i, x, y, z);
        trap_at(p, i, x, y, z, V2, V4);
        cpx<double> ph[3], hl[3], nl[3];
        load3(phi, i, M, ph);
        load3(hlf, i, M, hl);
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
    block_row<NS_EVAL>(acc, as_global(S.red_pw), NS_MAX);
}

// ---------------------------------------------------------------------------
// update and residual:
//   if a step is pending: Phi <- (c Phi + s P/|P|) inv_norm and, by linearity of
//   H_L, H_L Phi <- (c H_L Phi + s H_L P^) inv_norm;
//   r = H(Phi)Phi - mu Phi, P_V^{1/2} = (alpha_l + V + c0 rho)^{-1/2} (3.14),
//   preconditioner input u = P_V^{1/2} r;
//   reductions: max |r| and the P^{n-1} terms of the next direction.
// final_only: residual norm of the current iterate only (no writes, no control).
// ---------------------------------------------------------------------------
template <typename R, typename RD>
__global__ __launch_bounds__(PT) void k_resid(const Slot* slots, RedGeom g, int final_only) {
    const Slot& S = slots[blockIdx.y];
    SolveState* st = as_global(S.st);
    if (st->done && !final_only) return;
    const Phys p = S.p;
    const long long M = p.M;
    cpx<R>* phif = fld<R>(S, B_PHI);
    cpx<R>* hlf = fld<R>(S, B_HL);
    const cpx<RD>* Pf = fld<RD>(S, B_P);
    const cpx<RD>* hlpf = fld<RD>(S, B_HLP);
    cpx<RD>* uf = fld<RD>(S, B_U);
    RD* pvv = pvf<RD>(S);
    const int pending = st->pending_step && !final_only;
    const double k0 = st->c, k1 = st->s * st->invnP, ks = st->s, k2 = st->inv_norm;
    const double mu = st->mu;
    const double al[3] = {st->alpha[0], st->alpha[1], st->alpha[2]};
    const double fl = 1e-12 * fmax(1.0, fmax(al[0], fmax(al[1], al[2])));
    cpx<RD>* r = fld<RD>(S, B_R0 + st->cur);   // held in the direction type (beta sums, P_C input)
    const bool kinetic = st->precond == GS_PC_KINETIC;   // no potential factor (3.12)
    double acc[NS_RES] = {0.0, 0.0, 0.0, 0.0};
    double wmax = 0.0;
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < M; i += (long long)gridDim.x * PT) {
        double x, y, z, V2, V4;
        coords(p, i, x, y, z);
        trap_at(p, i, x, y, z, V2, V4);
        cpx<double> ph[3], hl[3], nl[3], P[3];
        load3(phif, i, M, ph);
        load3(hlf, i, M, hl);
        if (!final_only) load3(Pf, i, M, P);
        if (pending) {
            cpx<double> hp[3];
            const cpx<double> old[3] = {ph[0], ph[1], ph[2]};
            load3(hlpf, i, M, hp);
            for (int c = 0; c < 3; ++c) {
                ph[c] = k2 * (k0 * ph[c] + k1 * P[c]);
                hl[c] = k2 * (k0 * hl[c] + ks * hp[c]);
            }
            store3(phif, i, M, ph);
            store3(hlf, i, M, hl);
            // continue from the stored (rounded) values
            load3(phif, i, M, ph);
            load3(hlf, i, M, hl);
            for (int c = 0; c < 3; ++c) wmax = fmax(wmax, sqrt(cabs2(ph[c] - old[c])));
        }
        const Spin sp = spin_of(ph);
        nonlin(p, sp, ph, nl);
        for (int c = 0; c < 3; ++c) {
            const cpx<double> rc = hl[c] + nl[c] - mu * ph[c];
            acc[0] = fmax(acc[0], sqrt(cabs2(rc)));
            if (final_only) continue;
            const cpx<RD> rr = cmk((RD)rc.x, (RD)rc.y);
            r[c * M + i] = rr;
            const double d = fmax(al[c] + V2 + V4 + p.c0 * sp.rho, fl);
            const RD w = kinetic ? (RD)1 : (RD)(1.0 / sqrt(d));
            pvv[c * M + i] = w;
            uf[c * M + i] = w * rr;
            const cpx<double> rw = wid(rr);
            acc[1] += re_dot(rw, P[c]);
            acc[2] += re_dot(ph[c], P[c]);
            acc[3] += cabs2(P[c]);
        }
    }
    const double m = bmax(acc[0]);
    if (threadIdx.x == 0) as_global(S.red_pw)[(long long)blockIdx.x * NS_MAX] = m;
    if (pending) {   // uniform over the block
        const double wm = bmax(wmax);
        if (threadIdx.x == 0) as_global(S.red_pw)[(long long)blockIdx.x * NS_MAX + W_ROW] = wm;
    }
    const double t[3] = {acc[1], acc[2], acc[3]};
    block_row<3>(t, as_global(S.red_pw) + 1, NS_MAX);   // entries 1..3 of the row
}

// ---------------------------------------------------------------------------
// line-search integrals and the coefficients of the next iterate's scalars
// (layout in control.h, NS_LS); the kinetic coefficients come from the middle
// pass of the H_L P^ application
// ---------------------------------------------------------------------------
template <typename R, typename RD>
__global__ __launch_bounds__(PT, 3) void k_lsred(const Slot* slots, RedGeom g) {
    const Slot& S = slots[blockIdx.y];
    SolveState* st = as_global(S.st);
    if (st->done) return;
    const Phys p = S.p;
    const long long M = p.M;
    const double ip = st->invnP;
    const double w0 = 0.5 * p.c0, w1 = 0.5 * p.c1;
    double acc[NS_LS];
    for (int k = 0; k < NS_LS; ++k) acc[k] = 0.0;
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < M; i += (long long)gridDim.x * PT) {
        double x, y, z, V2, V4;
        coords(p, i, x, y, z);
        trap_at(p, i, x, y, z, V2, V4);
        const double V = V2 + V4;
        cpx<double> ph[3], P[3], hl[3], hp[3];
        // generic (flat) loads on purpose: this loop uses no LDS, and with
        // global-address loads the compiler's schedule needs more registers
        // than three blocks per SIMD allow and spills inside the loop
        load3(static_cast<const cpx<R>*>(S.buf[B_PHI]), i, M, ph);
        load3(static_cast<const cpx<RD>*>(S.buf[B_P]), i, M, P);
        load3(static_cast<const cpx<R>*>(S.buf[B_HL]), i, M, hl);
        load3(static_cast<const cpx<RD>*>(S.buf[B_HLP]), i, M, hp);
        for (int c = 0; c < 3; ++c) P[c] = ip * P[c];
        double n0[3], n1[3], n2[3];
        for (int c = 0; c < 3; ++c) {
            acc[0] += re_dot(hp[c], P[c]);
            acc[1] += re_dot(hl[c], P[c]);
            n0[c] = cabs2(ph[c]);
            n1[c] = re_dot(ph[c], P[c]);
            n2[c] = cabs2(P[c]);
        }
        const double q0r = n0[0] + n0[1] + n0[2], q1r = n1[0] + n1[1] + n1[2], q2r = n2[0] + n2[1] + n2[2];
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
            acc[9] += w0 * q0r * q0r;
        }
        for (int a = 0; a < 3; ++a) {
            const double d = F2[a] - F0[a];
            acc[4] += w1 * F0[a] * F1[a];
            acc[5] += w1 * F0[a] * d;
            acc[6] += w1 * F1[a] * F1[a];
            acc[7] += w1 * d * F1[a];
            acc[8] += w1 * d * d;
            acc[9] += w1 * F0[a] * F0[a];
        }
        for (int c = 0; c < 3; ++c) {
            acc[10 + c] += n0[c];
            acc[13 + c] += n1[c];
            acc[16 + c] += n2[c];
            acc[19 + c] += V * n0[c];
            acc[22 + c] += V * n1[c];
            acc[25 + c] += V * n2[c];
            double* T = acc + 28 + 5 * c;
            T[0] += p.c0 * q0r * n0[c];
            T[1] += p.c0 * (q0r * n1[c] + q1r * n0[c]);
            T[2] += p.c0 * (q0r * n2[c] + q2r * n0[c] + 4.0 * q1r * n1[c]);
            T[3] += p.c0 * (q1r * n2[c] + q2r * n1[c]);
            T[4] += p.c0 * q2r * n2[c];
        }
    }
    block_row<NS_LS>(acc, as_global(S.red_pw), NS_MAX);
}

// ---------------------------------------------------------------------------
// pending step before a fresh evaluation: Phi <- (c Phi + s P^) inv_norm (a
// rescale when s = 0), formed in double and rounded once; block maxima of
// |Phi^{n+1} - Phi^n| (criterion (3.9)) in entry W_ROW of the rows
// ---------------------------------------------------------------------------
template <typename R, typename RD>
__global__ __launch_bounds__(PT) void k_apply(const Slot* slots, RedGeom g) {
    const Slot& S = slots[blockIdx.y];
    const SolveState* st = as_global(S.st);
    if (st->done || !st->pending_step) return;
    const long long n3 = 3 * S.p.M;
    cpx<R>* phi = fld<R>(S, B_PHI);
    const cpx<RD>* P = fld<RD>(S, B_P);
    const double k0 = st->c, k1 = st->s * st->invnP, k2 = st->inv_norm;
    const bool rescale = st->s == 0.0;
    double wmax = 0.0;
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < n3; i += (long long)gridDim.x * PT) {
        const cpx<double> v = wid(phi[i]);
        const cpx<R> nv = rescale ? cvt<R>(k2 * (k0 * v)) : cvt<R>(k2 * (k0 * v + k1 * wid(P[i])));
        phi[i] = nv;
        wmax = fmax(wmax, sqrt(cabs2(wid(nv) - v)));
    }
    const double wm = bmax(wmax);
    if (threadIdx.x == 0) as_global(S.red_pw)[(long long)blockIdx.x * NS_MAX + W_ROW] = wm;
}

// ---------------------------------------------------------------------------
// normalisation: sets the pending rescale Phi <- Phi / |Phi|
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(PT) void k_normalize(const Slot* slots, RedGeom g) {
    const Slot& S = slots[blockIdx.y];
    const Phys p = S.p;
    const cpx<R>* phi = fld<R>(S, B_PHI);
    const long long n3 = 3 * p.M;
    double acc[1] = {0.0};
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < n3; i += (long long)gridDim.x * PT)
        acc[0] += cabs2(wid(phi[i]));
    block_row<1>(acc, as_global(S.red_pw), NS_MAX);
}

// ---------------------------------------------------------------------------
// control: one block per slot gathers the rows of the preceding pass(es)
// ---------------------------------------------------------------------------
//   FIN_EVAL:   eval rows + middle-pass rows -> ctrl_eval
//   FIN_DIR:    residual rows -> ctrl_resid; unless that ended the solve,
//               preconditioner rows -> ctrl_dir
//   FIN_LS:     line-search rows + middle-pass rows -> ctrl_ls
//   FIN_NORM:   |Phi|^2 rows -> rescale of Phi (pending step with s = 0)
//   FIN_RFINAL: residual rows of a final-only residual pass
__global__ __launch_bounds__(PT) void k_fin(const Slot* slots, RedGeom g, int what) {
    const Slot& S = slots[blockIdx.y];
    SolveState* gst = as_global(S.st);
    const Phys p = S.p;
    if (what != FIN_NORM && what != FIN_RFINAL && gst->done) return;
    // Thread 0's control steps read and write the state field by field; they
    // run on a copy in LDS that the whole block loads at once and stores back
    // at the end, so those accesses are LDS accesses, not dependent round
    // trips to memory.
    static_assert(sizeof(SolveState) % 8 == 0, "state copied in 8-byte words");
    constexpr int NW = (int)(sizeof(SolveState) / 8);
    __shared__ SolveState sst;
    for (int w = threadIdx.x; w < NW; w += PT)
        reinterpret_cast<unsigned long long*>(&sst)[w] = reinterpret_cast<const unsigned long long*>(gst)[w];
    __syncthreads();
    SolveState* st = &sst;
    // the pass before this control step applied a PCG step: its largest change
    // (3.9); a normalisation rescale (s = 0) leaves the recorded change alone
    if (what == FIN_EVAL || what == FIN_DIR) {
        // read by every thread before thread 0 changes the state
        const int had_step = st->pending_step && st->s != 0.0;
        if (had_step) {
            double wc[1];
            gather<1>(wc, as_global(S.red_pw) + W_ROW, g.nblk_pw, NS_MAX, 1u);
            if (threadIdx.x == 0) st->wchange = wc[0];
        }
    }
    if (what == FIN_EVAL) {
        double tot[NS_EVAL], mt[4];
        gather<NS_EVAL>(tot, as_global(S.red_pw), g.nblk_pw, NS_MAX);
        gather<4>(mt, as_global(S.red_mid), g.nblk_mid, RED_MID_STRIDE);
        if (threadIdx.x == 0) ctrl_eval(st, p, tot, mt);
    } else if (what == FIN_DIR) {
        double tot[NS_RES];
        gather<NS_RES>(tot, as_global(S.red_pw), g.nblk_pw, NS_MAX, 1u);
        __shared__ int stop;
        if (threadIdx.x == 0) {
            ctrl_resid(st, p, tot, 0);
            stop = st->done;
        }
        __syncthreads();
        if (!stop) {   // uniform over the block
            double dt[NS_DIR];
            gather<NS_DIR>(dt, as_global(S.red_dir), g.nblk_dir, RED_DIR_STRIDE);
            if (threadIdx.x == 0) ctrl_dir(st, p, dt);
        }
    } else if (what == FIN_LS) {
        double tot[NS_LS], kin[NS_KIN];
        gather<NS_LS>(tot, as_global(S.red_pw), g.nblk_pw, NS_MAX);
        gather<NS_KIN>(kin, as_global(S.red_mid), g.nblk_mid, RED_MID_STRIDE);
        if (threadIdx.x == 0) ctrl_ls(st, p, tot, kin);
    } else if (what == FIN_NORM) {
        double tot[1];
        gather<1>(tot, as_global(S.red_pw), g.nblk_pw, NS_MAX);
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
        }
    } else if (what == FIN_RFINAL) {
        double tot[NS_RES];
        gather<NS_RES>(tot, as_global(S.red_pw), g.nblk_pw, NS_MAX, 1u);
        if (threadIdx.x == 0) ctrl_resid(st, p, tot, 1);
    }
    __syncthreads();
    for (int w = threadIdx.x; w < NW; w += PT)
        reinterpret_cast<unsigned long long*>(gst)[w] = reinterpret_cast<const unsigned long long*>(&sst)[w];
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
__global__ void k_hphi(const Slot* slots) {
    const Slot& S = slots[blockIdx.y];
    const Phys p = S.p;
    const cpx<R>* phi = fld<R>(S, B_PHI);
    const cpx<R>* hl = fld<R>(S, B_HL);
    cpx<R>* out = fld<R>(S, B_X1);
    const long long M = p.M;
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < M; i += (long long)gridDim.x * PT) {
        cpx<double> ph[3], h[3], nl[3];
        load3(phi, i, M, ph);
        load3(hl, i, M, h);
        const Spin sp = spin_of(ph);
        nonlin(p, sp, ph, nl);
        for (int c = 0; c < 3; ++c) h[c] = h[c] + nl[c];
        store3(out, i, M, h);
    }
}

// preconditioner input for a given r: pv = (alpha_l + V + c0 rho)^{-1/2}, u = pv r
template <typename R>
__global__ void k_pvin(const Slot* slots) {
    const Slot& S = slots[blockIdx.y];
    const Phys p = S.p;
    const SolveState* st = as_global(S.st);
    const cpx<R>* phi = fld<R>(S, B_PHI);
    const cpx<R>* r = fld<R>(S, B_X0);
    R* pv = pvf<R>(S);
    cpx<R>* u = fld<R>(S, B_U);
    const long long M = p.M;
    const double al[3] = {st->alpha[0], st->alpha[1], st->alpha[2]};
    const double fl = 1e-12 * fmax(1.0, fmax(al[0], fmax(al[1], al[2])));
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < M; i += (long long)gridDim.x * PT) {
        double x, y, z, V2, V4;
        coords(p, i, x, y, z);
        trap_at(p, i, x, y, z, V2, V4);
        cpx<double> ph[3];
        load3(phi, i, M, ph);
        const Spin sp = spin_of(ph);
        for (int c = 0; c < 3; ++c) {
            const R w = (R)(1.0 / sqrt(fmax(al[c] + V2 + V4 + p.c0 * sp.rho, fl)));
            pv[c * M + i] = w;
            u[c * M + i] = w * r[c * M + i];
        }
    }
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

// Zero-padding of a spectrum from grid nc to grid nf (both in natural FFT
// order, [3][Nz][Ny][Nx]): the coefficient of wavenumber index p (|p| < nc/2)
// moves to the fine index of p; the coarse Nyquist coefficient (p = -nc/2)
// goes half to +nc/2 and half to -nc/2 of the fine grid (whole when the axis
// is not refined); all other fine coefficients are zero. `scale` = Mf/Mc keeps
// the values after the 1/Mf of the inverse transform.
__device__ __forceinline__ double pad_weight(int jf, int nf, int nc, int& jc) {
    const int p = (jf < nf / 2) ? jf : jf - nf;
    if (p > -nc / 2 && p < nc / 2) { jc = (p + nc) % nc; return 1.0; }
    if (p == nc / 2 || p == -nc / 2) { jc = nc / 2; return nf == nc ? 1.0 : 0.5; }
    jc = 0;
    return 0.0;
}
__global__ void k_spec_pad(const cpx<double>* in, cpx<double>* out, int dim, int ncx, int ncy, int ncz, int nfx,
                           int nfy, int nfz, double scale) {
    const long long Mf = (long long)nfx * nfy * nfz, Mc = (long long)ncx * ncy * ncz;
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < Mf; i += (long long)gridDim.x * PT) {
        const int jx = (int)(i % nfx), jy = (int)((i / nfx) % nfy), jz = (int)(i / ((long long)nfx * nfy));
        int cx, cy, cz = 0;
        double w = pad_weight(jx, nfx, ncx, cx) * pad_weight(jy, nfy, ncy, cy);
        if (dim == 3) w *= pad_weight(jz, nfz, ncz, cz);
        const long long ic = ((long long)cz * ncy + cy) * ncx + cx;
        for (int c = 0; c < 3; ++c)
            out[c * Mf + i] = w == 0.0 ? cmk(0.0, 0.0) : (scale * w) * in[c * Mc + ic];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename R> hipError_t launch_eval(const Slot* slots, int nslots, RedGeom g, hipStream_t s) {
    GS_LAUNCH(k_eval<R>, dim3(g.nblk_pw, nslots), dim3(PT), 0, s, slots, g);
    return hipGetLastError();
}
template <typename R, typename RD>
hipError_t launch_resid(const Slot* slots, int nslots, RedGeom g, int final_only, hipStream_t s) {
    GS_LAUNCH((k_resid<R, RD>), dim3(g.nblk_pw, nslots), dim3(PT), 0, s, slots, g, final_only);
    return hipGetLastError();
}
template <typename R, typename RD> hipError_t launch_lsred(const Slot* slots, int nslots, RedGeom g, hipStream_t s) {
    GS_LAUNCH((k_lsred<R, RD>), dim3(g.nblk_pw, nslots), dim3(PT), 0, s, slots, g);
    return hipGetLastError();
}
template <typename R, typename RD> hipError_t launch_apply(const Slot* slots, int nslots, RedGeom g, hipStream_t s) {
    GS_LAUNCH((k_apply<R, RD>), dim3(g.nblk_pw, nslots), dim3(PT), 0, s, slots, g);
    return hipGetLastError();
}
template <typename R> hipError_t launch_normalize(const Slot* slots, int nslots, RedGeom g, hipStream_t s) {
    GS_LAUNCH(k_normalize<R>, dim3(g.nblk_pw, nslots), dim3(PT), 0, s, slots, g);
    return hipGetLastError();
}
hipError_t launch_fin(const Slot* slots, int nslots, RedGeom g, int what, hipStream_t s) {
    GS_LAUNCH(k_fin, dim3(1, nslots), dim3(PT), 0, s, slots, g, what);
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
template <typename R> hipError_t launch_hphi(const Slot* slots, int nslots, RedGeom g, hipStream_t s) {
    GS_LAUNCH(k_hphi<R>, dim3(g.nblk_pw, nslots), dim3(PT), 0, s, slots);
    return hipGetLastError();
}
template <typename R> hipError_t launch_pvin(const Slot* slots, int nslots, RedGeom g, hipStream_t s) {
    GS_LAUNCH(k_pvin<R>, dim3(g.nblk_pw, nslots), dim3(PT), 0, s, slots);
    return hipGetLastError();
}
hipError_t launch_spec_pad(const cpx<double>* in, cpx<double>* out, int dim, const int nc[3], const int nf[3],
                           hipStream_t s) {
    const long long Mf = (long long)nf[0] * nf[1] * nf[2], Mc = (long long)nc[0] * nc[1] * nc[2];
    GS_LAUNCH(k_spec_pad, dim3(pw_blocks(Mf)), dim3(PT), 0, s, in, out, dim, nc[0], nc[1], nc[2], nf[0], nf[1],
              nf[2], (double)Mf / (double)Mc);
    return hipGetLastError();
}
hipError_t launch_gaussian(cpx<double>* out, const Phys& p, hipStream_t s) {
    GS_LAUNCH(k_gaussian, dim3(pw_blocks(p.M)), dim3(PT), 0, s, out, p);
    return hipGetLastError();
}

#define GS_INST(R)                                                                              \
    template hipError_t launch_eval<R>(const Slot*, int, RedGeom, hipStream_t);                 \
    template hipError_t launch_normalize<R>(const Slot*, int, RedGeom, hipStream_t);            \
    template hipError_t launch_hphi<R>(const Slot*, int, RedGeom, hipStream_t);                 \
    template hipError_t launch_pvin<R>(const Slot*, int, RedGeom, hipStream_t);
#define GS_INST2(R, RD)                                                                         \
    template hipError_t launch_resid<R, RD>(const Slot*, int, RedGeom, int, hipStream_t);       \
    template hipError_t launch_lsred<R, RD>(const Slot*, int, RedGeom, hipStream_t);             \
    template hipError_t launch_apply<R, RD>(const Slot*, int, RedGeom, hipStream_t);
GS_INST(double)
GS_INST(float)
GS_INST2(double, double)
GS_INST2(float, float)
GS_INST2(double, float)

}  // namespace gs
