// Scalar control of the PCG iteration (Algorithms 1 and 2 of the paper), run on
// thread 0 of the last block of the reducing kernels. All decisions are taken
// on the device from reduced FP64 sums and written to SolveState.
#pragma once
#include "gs_internal.h"
#include "../../include/gs.h"

namespace gs {

// ---------------------------------------------------------------------------
// fresh evaluation of the current iterate (after an H_L application)
// ---------------------------------------------------------------------------
// s[0..2]   sum |phi_l|^2                   s[3..5]   sum V |phi_l|^2
// s[6..8]   sum c0 rho |phi_l|^2            s[9..11]  sum Re conj(phi_l) (H_L Phi)_l
// s[12..14] sum Re conj(phi_l) NL_l          s[15]     sum c0/2 rho^2
// s[16]     sum c1/2 |F|^2                  s[17]     sum V4 rho (degree-4 part)
// m[0..2]   spectral sum 1/2|k|^2 |phi^_l|^2, m[3] spectral sum Re phi^dag S(k) phi
constexpr int NS_EVAL = 18;

__device__ inline void ctrl_eval(SolveState* st, const Phys& p, const double (&s)[NS_EVAL], const double (&m)[4]) {
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

__device__ inline void stop_stagnated(SolveState* st) {
    if (st->phase == PH_FP32) st->switch_req = 1;
    else st->status = GS_WSTAGNATED;
    st->done = 1;
}

// ---------------------------------------------------------------------------
// residual: stopping tests (criterion (3.10), max_iter, the FP32 exit)
// ---------------------------------------------------------------------------
// r[0] = max |r|, r[1] = sum Re r conj(P^{n-1}), r[2] = sum Re phi conj(P^{n-1}), r[3] = sum |P^{n-1}|^2
constexpr int NS_RES = 4;

__device__ inline void ctrl_resid(SolveState* st, const Phys& p, const double (&r)[NS_RES], int final_only) {
    const double rinf = r[0];
    st->resid_inf = rinf;
    st->pending_step = 0;
    if (final_only) return;
    st->rP = r[1] * p.cell;
    st->phiP = r[2] * p.cell;
    st->PP = r[3] * p.cell;
    if (!isfinite(rinf)) { st->nonfinite = 1; st->status = GS_ENONFINITE; st->done = 1; return; }
    if (st->final_pending) { st->done = 1; return; }
    if (st->phase == PH_FP32) {
        if (rinf < st->switch_resid) { st->switch_req = 1; st->done = 1; return; }
        if (rinf < 0.5 * st->best_resid) { st->best_resid = rinf; st->best_iter = st->iter_phase; }
        else if (st->iter_phase - st->best_iter >= st->stall_window) { st->switch_req = 1; st->done = 1; return; }
        if (st->iter_phase >= st->phase_max_iter) { st->switch_req = 1; st->done = 1; return; }
    } else if ((st->stop_kind == GS_STOP_RESIDUAL || st->stop_kind == GS_STOP_EITHER) && rinf < st->tol) {
        st->done = 1;   // criterion (3.10)
        return;
    } else if (st->stop_kind == GS_STOP_WAVEFN && st->iter_phase > 0 && st->wchange < st->tol) {
        // criterion (3.9), for the PCG step of this precision phase that produced
        // this iterate (never for a normalisation, nor for the float phase's last step)
        st->done = 1;
        return;
    }
    if (st->iter >= st->max_iter) { st->status = GS_WMAXITER; st->done = 1; return; }
}

// ---------------------------------------------------------------------------
// direction: PRP beta, projection, |P|, descent test (Algorithm 2, Steps 1-2)
// ---------------------------------------------------------------------------
// s[0] = Re<r, Pr>, s[1] = Re<r_prev, Pr>, s[2] = Re<phi, Pr>, s[3] = |Pr|^2,
// s[4] = Re<Pr, P^{n-1}> (grid sums); the P^{n-1} terms with r and phi come from
// the residual pass (SolveState::rP, phiP, PP).
constexpr int NS_DIR = 5;

__device__ inline void ctrl_dir(SolveState* st, const Phys& p, const double (&s)[NS_DIR]) {
    const double h = p.cell;
    const double rpr = s[0] * h, rprp = s[1] * h, phipr = s[2] * h, prpr = s[3] * h;
    double prP = s[4] * h, rP = st->rP, phiP = st->phiP, PP = st->PP;
    if (!st->have_prev) { prP = rP = phiP = PP = 0.0; }
    const double mu = st->mu;
    double beta = 0.0;
    if (st->have_prev) {
        beta = (rpr - rprp) / st->rpr_prev;      // Polak-Ribiere-Polyak, clipped at 0
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
        if (beta != 0.0) { beta = 0.0; st->resets++; continue; }   // steepest descent
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

// ---------------------------------------------------------------------------
// step size (Algorithm 2, Steps 2-4) and the scalars of the next iterate
// ---------------------------------------------------------------------------
// Along Phi(t) = cos t Phi + sin t P^ (c = cos t, s = sin t):
//  - linear part: c^2 <H_L Phi,Phi> + 2cs Re<H_L Phi,P^> + s^2 <H_L P^,P^>;
//  - every density q in c0/2 rho^2 + c1/2 sum_a F_a^2 is c^2 q0 + 2cs q1 + s^2 q2,
//    and with d = s^2 (q2 - q0) + 2cs q1, q(t)^2 - q0^2 = 2 q0 d + d^2, so the
//    change of the quartic energy is a polynomial in five integrals per density
//      I01 = w q0 q1, I02 = w q0 (q2-q0), I11 = w q1^2, I21 = w (q2-q0) q1, I22 = w (q2-q0)^2,
//    (w = c0/2 for rho, c1/2 for each F_a); its value at 0 is I00 = w q0^2;
//  - per component, |phi_l|^2, V |phi_l|^2 and the kinetic density are
//    quadratic forms (coefficients n0 n1 n2, V0 V1 V2, K0 X K2), and
//    c0 rho |phi_l|^2 is quartic with coefficients T0..T4.
// The second-order expansion of the energy change gives a_n, b_n of
// eqs. (3.7)-(3.8); the same polynomial evaluates every trial step.
// s[0] Re<H_L P^,P^>  s[1] Re<H_L Phi,P^>  s[2], s[3] unused (|P^|^2 and Re<Phi,P^>
// are the sums of n2_l and n1_l)
// s[4..8] I01 I02 I11 I21 I22   s[9] I00
// s[10..12] n0_l  s[13..15] n1_l  s[16..18] n2_l  s[19..21] V0_l  s[22..24] V1_l  s[25..27] V2_l
// s[28+5l+j] T_j,l (j = 0..4)
// kin[3l+0..2] = K0_l, X_l, K2_l (spectral sums)
constexpr int NS_LS = 43;
constexpr int NS_KIN = 9;

// Energy change along the normalised curve (c Phi + s P^)/|c Phi + s P^|, formed
// without subtracting two energies. With N = |Phi|^2, X = Re<Phi,P^>, Y = |P^|^2
// and n = c^2 N + 2cs X + s^2 Y (so n - N = 2cs X + s^2 (Y - N)), the quadratic
// part is (N L(t) - A n)/(N n) = (2cs (N B - A X) + s^2 (N C - A Y))/(N n) and the
// quartic part (N^2 (D(t) - D0) - D0 (n - N)(n + N))/(N n)^2, D(t) - D0 being the
// polynomial in I01..I22. For a unit P^ orthogonal to Phi (N = Y = 1, X = 0) this
// is the plain expansion; a direction rounded to float is neither, to its
// rounding, and the X and Y - N terms keep that rounding (a spurious first-order
// term A X) out of the descent test.
struct LsPoly {
    double N, A, B, C, X, Y, D0, I[5];
};
__device__ __forceinline__ double dE_at(double c, double s, const LsPoly& k) {
    const double cs2 = 2.0 * c * s, ss = s * s;
    const double n = c * c * k.N + cs2 * k.X + ss * k.Y;
    const double dn = cs2 * k.X + ss * (k.Y - k.N);
    const double dL = cs2 * (k.N * k.B - k.A * k.X) + ss * (k.N * k.C - k.A * k.Y);
    const double dD = 2.0 * ss * k.I[1] + 2.0 * cs2 * k.I[0] + ss * ss * k.I[4] + 2.0 * cs2 * ss * k.I[3] +
                      cs2 * cs2 * k.I[2];
    const double Nn = k.N * n;
    return dL / Nn + (k.N * k.N * dD - k.D0 * dn * (n + k.N)) / (Nn * Nn);
}

__device__ inline void ctrl_ls(SolveState* st, const Phys& p, const double (&s)[NS_LS], const double (&kin)[NS_KIN]) {
    const double h = p.cell, kM = h / (double)p.M;
    const double Cq = s[0] * h, B = s[1] * h;
    const double PhPh = (s[16] + s[17] + s[18]) * h, phiPh = (s[13] + s[14] + s[15]) * h;
    const double I[5] = {s[4] * h, s[5] * h, s[6] * h, s[7] * h, s[8] * h};
    const double I00 = s[9] * h;
    const LsPoly K{st->norm2, st->lin, B, Cq, phiPh, PhPh, I00, {I[0], I[1], I[2], I[3], I[4]}};
    // second-order model (3.7)-(3.8), the direction's Phi component and norm error removed
    const double a = (Cq - st->lin * PhPh) + 2.0 * I[1] + 4.0 * I[2];
    const double b = 2.0 * (B - st->lin * phiPh) + 4.0 * (I[0] - I00 * phiPh);
    st->a = a;
    st->b = b;
    double theta = (a > 0.0 && b < 0.0) ? -b / (2.0 * a) : st->theta_trial;
    int accepted = 0;
    double dE = 0.0, c = 1.0, sn = 0.0;
    for (int k = 0; k <= st->max_backtrack; ++k) {
        c = cos(theta);
        sn = sin(theta);
        dE = dE_at(c, sn, K);
        if (dE < 0.0) { accepted = 1; break; }   // the energy decreases
        theta *= st->sigma;
        st->backtracks++;
    }
    if (!accepted || !isfinite(dE)) { stop_stagnated(st); return; }
    if (st->exact_ls) {
        // minimise the energy change along the curve: Newton steps on dE(t)
        // from the accepted t, derivatives by central differences (the
        // points t +- h by rotating (c, s)), a step kept only when it lowers
        // dE; ends when the step is below 1e-9 t
        const double h = 1e-4 * theta;
        const double ch = cos(h), sh = sin(h);
        for (int it = 0; it < 8; ++it) {
            const double fp = dE_at(c * ch - sn * sh, sn * ch + c * sh, K);
            const double fm = dE_at(c * ch + sn * sh, sn * ch - c * sh, K);
            const double d1 = (fp - fm) / (2.0 * h), d2 = (fp - 2.0 * dE + fm) / (h * h);
            if (!(d2 > 0.0)) break;
            const double tn = fmin(fmax(theta - d1 / d2, 0.25 * theta), fmin(4.0 * theta, 1.5707963267948966));
            const double cn = cos(tn), snn = sin(tn);
            const double fn = dE_at(cn, snn, K);
            if (!(fn < dE)) break;
            const bool small = fabs(tn - theta) < 1e-9 * theta;
            theta = tn;
            c = cn;
            sn = snn;
            dE = fn;
            if (small) break;
        }
    }
    st->theta = theta;
    st->c = c;
    st->s = sn;
    st->dE = dE;
    st->dE_last = dE;
    const double n2 = c * c * st->norm2 + 2.0 * c * sn * phiPh + sn * sn * PhPh;
    const double q = 1.0 / n2;
    st->inv_norm = sqrt(q);
    // scalars of Phi^{n+1} = (c Phi + s P^) / |c Phi + s P^|
    const double cc = c * c, cs2 = 2.0 * c * sn, ss = sn * sn;
    const double lin1 = (cc * st->lin + cs2 * B + ss * Cq) * q;
    const double enl = I00 + 2.0 * ss * I[1] + 2.0 * cs2 * I[0] + ss * ss * I[4] + 2.0 * cs2 * ss * I[3] +
                       cs2 * cs2 * I[2];
    const double espin1 = enl * q * q;
    st->lin = lin1;
    st->E = lin1 + espin1;
    st->mu = lin1 + 2.0 * espin1;
    double nsum = 0.0;
    for (int l = 0; l < 3; ++l) {
        const double nl = (cc * s[10 + l] + cs2 * s[13 + l] + ss * s[16 + l]) * h * q;
        const double vl = (cc * s[19 + l] + cs2 * s[22 + l] + ss * s[25 + l]) * h * q;
        const double kl = (cc * kin[3 * l] + cs2 * kin[3 * l + 1] + ss * kin[3 * l + 2]) * kM * q;
        const double* T = s + 28 + 5 * l;
        const double tl = (cc * cc * T[0] + cc * cs2 * T[1] + cc * ss * T[2] + cs2 * ss * T[3] + ss * ss * T[4]) * h * q * q;
        st->norm_comp[l] = nl;
        st->alpha[l] = kl + vl + tl;                 // eq. (3.13) at Phi^{n+1}
        nsum += nl;
    }
    st->norm2 = nsum;
    st->pending_step = 1;
    st->iter++;
    st->iter_phase++;
    st->rpr_prev = st->rpr;
    st->have_prev = 1;
    st->cur ^= 1;
    if (st->phase != PH_FP32 && (st->stop_kind == GS_STOP_ENERGY || st->stop_kind == GS_STOP_EITHER) &&
        fabs(dE) < st->tol)
        st->final_pending = 1;   // criterion (3.11)
}

}  // namespace gs
