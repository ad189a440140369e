// Batched three-component FFT passes for gfx950.
//
// The d-dimensional transforms of the Fourier spectral method (Sec. 3.2 of the
// paper: coefficients by FFT, derivatives as multipliers) are done one axis per
// pass. Every pass works on whole lines in LDS and moves the transformed axis
// between the contiguous and the slowest position on its way out, so that
// every global access is a run of contiguous elements:
//
//   fwdT:  in[3][A][B][N]  --FFT along N-->  out[3][N][A][B]
//   invT:  in[3][N][B][C]  --IFFT along N--> out[3][B][C][N]
//   mid:   in[3][L][N]     --FFT, spectral operator on all 3 components, IFFT--> out[3][L][N]
//
// In 2D the H_L chain is fwdT (x) -> mid (y) -> invT (x); in 3D it is
// fwdT (x) -> fwdT (y) -> mid (z) -> invT (y) -> invT (x). Line transforms are
// Stockham autosort radix-4 stages plus one radix-2 stage for odd log2 N, with
// the data of all lines of a block resident in LDS and the butterflies of a
// stage held in registers between two barriers.
//
// Every pass serves all slots (independent solves of one grid shape) of a
// launch at once: blockIdx.y selects the slot, whose descriptor names the
// buffers, the problem and the solver state. A slot whose solve has finished
// returns at once.
#include "device_common.h"
#include "control.h"

namespace gs {

constexpr int NT = PT;   // threads per block of every FFT pass

template <int N> struct Log2 { static constexpr int v = 1 + Log2<N / 2>::v; };
template <> struct Log2<1> { static constexpr int v = 0; };

template <typename R, bool INV>
__device__ __forceinline__ cpx<R> twid(const cpx<R>* __restrict__ tw, int m) {
    cpx<R> w = tw[m];
    if (INV) w.y = -w.y;
    return w;
}

// in-place 4-point DFT, kernel e^{-+2 pi i r q / 4}
template <typename R, bool INV>
__device__ __forceinline__ void dft4(cpx<R>& v0, cpx<R>& v1, cpx<R>& v2, cpx<R>& v3) {
    const cpx<R> a = v0 + v2, b = v0 - v2, c = v1 + v3, d = v1 - v3;
    const cpx<R> id = cmuli(d);
    v0 = a + c;
    v2 = a - c;
    if (INV) { v1 = b + id; v3 = b - id; }
    else     { v1 = b - id; v3 = b + id; }
}

// Transform NL lines of length N held in LDS at buf + l * PITCH (natural order
// in and out, unnormalised). tw[m] = exp(-2 pi i m / N).
template <typename R, int N, int NL, int PITCH, bool INV>
__device__ __forceinline__ void lds_fft(cpx<R>* buf, const cpx<R>* __restrict__ tw) {
    constexpr int LOG2N = Log2<N>::v;
    constexpr int N4 = N / 4;
    constexpr int NB4 = NL * N4;
    constexpr int BPT4 = (NB4 + NT - 1) / NT;
    const int tid = threadIdx.x;
#pragma unroll
    for (int st = 0; st < LOG2N / 2; ++st) {
        const int Ns = 1 << (2 * st);
        cpx<R> v[BPT4][4];
        int jj[BPT4], ll[BPT4];
#pragma unroll
        for (int i = 0; i < BPT4; ++i) {
            const int b = tid + i * NT;
            ll[i] = -1;
            jj[i] = 0;
            if (b < NB4) {
                const int l = b / N4, j = b - l * N4;
                ll[i] = l;
                jj[i] = j;
                const cpx<R>* src = buf + l * PITCH + j;
                v[i][0] = src[0];
                v[i][1] = src[N4];
                v[i][2] = src[2 * N4];
                v[i][3] = src[3 * N4];
                if (st > 0) {
                    const int k = j & (Ns - 1);
                    const int step = k * (N / (4 * Ns));
                    v[i][1] = cmul(v[i][1], twid<R, INV>(tw, step));
                    v[i][2] = cmul(v[i][2], twid<R, INV>(tw, 2 * step));
                    v[i][3] = cmul(v[i][3], twid<R, INV>(tw, 3 * step));
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < BPT4; ++i) {
            if (ll[i] >= 0) {
                dft4<R, INV>(v[i][0], v[i][1], v[i][2], v[i][3]);
                const int j = jj[i];
                const int k = j & (Ns - 1);
                cpx<R>* dst = buf + ll[i] * PITCH + ((j - k) << 2) + k;
                dst[0] = v[i][0];
                dst[Ns] = v[i][1];
                dst[2 * Ns] = v[i][2];
                dst[3 * Ns] = v[i][3];
            }
        }
        __syncthreads();
    }
    if (LOG2N & 1) {
        // last stage, radix 2 with Ns = N/2: reads and writes the same pair
        constexpr int N2 = N / 2;
        constexpr int NB2 = NL * N2;
        for (int b = tid; b < NB2; b += NT) {
            const int l = b / N2, j = b - l * N2;
            cpx<R>* p = buf + l * PITCH + j;
            const cpx<R> u = p[0];
            const cpx<R> w = cmul(p[N2], twid<R, INV>(tw, j));
            p[0] = u + w;
            p[N2] = u - w;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// forward pass with transposed store
// ---------------------------------------------------------------------------
// DUAL (with PRO_DIR): components 3..5 of the output are the plain transform
// of aux1 (Phi), so that the middle pass sees both spectra.
template <typename R, int N, int TILE, int PRO, bool DUAL>
__global__ __launch_bounds__(NT) void k_fwdT(const Slot<R>* __restrict__ slots, int iin, int iout, int iaux0,
                                             int iaux1, int A, int B, const cpx<R>* __restrict__ tw) {
    const Slot<R>& S = slots[blockIdx.y];
    const SolveState* st = S.st;
    if (st->done) return;
    cpx<R>* inp = S.buf[iin];
    cpx<R>* __restrict__ out = S.buf[iout];
    const cpx<R>* __restrict__ aux0 = iaux0 >= 0 ? S.buf[iaux0] : nullptr;
    const cpx<R>* __restrict__ aux1 = iaux1 >= 0 ? S.buf[iaux1] : nullptr;
    constexpr int PITCH = N + 1;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    const int tiles = B / TILE;
    int blk = blockIdx.x;
    const int bt = blk % tiles;
    blk /= tiles;
    const int a = blk % A;
    const int c = blk / A;
    const int b0 = bt * TILE;
    const bool second = DUAL && c >= 3;
    const int cin = second ? c - 3 : c;
    const long long base = (((long long)cin * A + a) * B + b0) * N;

    int mode = second ? PRO_PLAIN : PRO;
    R k0 = 1, k1 = 0, k2 = 1;
    if (PRO == PRO_UPDATE) {
        if (!st->pending_step) mode = PRO_PLAIN;
        else {
            k0 = (R)st->c;
            k1 = (R)(st->s * st->invnP);
            k2 = (R)st->inv_norm;
            if (st->s == 0.0) mode = -1;   // rescale only
        }
    } else if (PRO == PRO_DIR) {
        k0 = (R)st->beta;
        k1 = (R)st->dphi;
        k2 = (R)st->invnP;
    }
    const cpx<R>* src = second ? aux1 : inp;
    for (int e = threadIdx.x; e < TILE * N; e += NT) {
        const int l = e / N, m = e - l * N;
        const long long gi = base + (long long)l * N + m;
        cpx<R> v = src[gi];
        if (mode == PRO_UPDATE) {
            v = k2 * (k0 * v + k1 * aux0[gi]);
            inp[gi] = v;
        } else if (mode == -1) {
            v = k2 * (k0 * v);
            inp[gi] = v;
        } else if (mode == PRO_DIR) {
            // D = -P r + beta P^{n-1};  P^n = D - Re<D,Phi> Phi  (stored), transform P^n / |P^n|
            v = k0 * v - aux0[gi] - k1 * aux1[gi];
            inp[gi] = v;
            v = k2 * v;
        }
        lds[l * PITCH + m] = v;
    }
    __syncthreads();
    lds_fft<R, N, TILE, PITCH, false>(lds, tw);
    for (int e = threadIdx.x; e < TILE * N; e += NT) {
        const int l = e % TILE, m = e / TILE;
        out[(((long long)c * N + m) * A + a) * B + b0 + l] = lds[l * PITCH + m];
    }
}

// ---------------------------------------------------------------------------
// inverse pass with transposed load and physical-space epilogue
// ---------------------------------------------------------------------------
//   EPI_SCALE: out = scale * v
//   EPI_HL:    last pass of the H_L chain, physical [z][y][x]:
//              out = IFFT(A) + V u - Omega x IFFT(B)      (u = uin, times 1/|P| if use_invnP)
//   EPI_ROTX:  3D y-pass of the H_L chain, layout [kx][z][y]:
//              out = IFFT(A) + Omega y k_x uin / Nx, out2 = IFFT(B)
//              (uin = the x-transformed input, same layout)
template <typename R, int N, int TILE, int EPI>
__global__ __launch_bounds__(NT) void k_invT(const Slot<R>* __restrict__ slots, int iin, int iin2, int iout,
                                             int iout2, int iuin, int B, int Cc, double scale, int use_invnP,
                                             int rot_any, const cpx<R>* __restrict__ tw) {
    const Slot<R>& S = slots[blockIdx.y];
    const SolveState* st = S.st;
    if (st->done) return;
    const Phys p = S.p;
    // the rotation input/output pair exists for rotating slots of the H_L chain
    const int nin = (EPI != EPI_SCALE && rot_any && p.omega != 0.0) ? 2 : 1;
    const cpx<R>* __restrict__ in = S.buf[iin];
    const cpx<R>* __restrict__ in2 = nin == 2 ? S.buf[iin2] : nullptr;
    cpx<R>* __restrict__ out = S.buf[iout];
    cpx<R>* __restrict__ out2 = (nin == 2 && iout2 >= 0) ? S.buf[iout2] : nullptr;
    const cpx<R>* __restrict__ uin = iuin >= 0 ? S.buf[iuin] : nullptr;
    constexpr int PITCH = N + 1;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    cpx<R>* lds2 = lds + TILE * PITCH;
    const int tiles = Cc / TILE;
    int blk = blockIdx.x;
    const int ct = blk % tiles;
    blk /= tiles;
    const int bb = blk % B;
    const int c = blk / B;
    const int c0 = ct * TILE;
    for (int e = threadIdx.x; e < TILE * N; e += NT) {
        const int l = e % TILE, m = e / TILE;
        const long long gi = (((long long)c * N + m) * B + bb) * Cc + c0 + l;
        lds[l * PITCH + m] = in[gi];
        if (nin == 2) lds2[l * PITCH + m] = in2[gi];
    }
    __syncthreads();
    lds_fft<R, N, TILE, PITCH, true>(lds, tw);
    if (nin == 2) lds_fft<R, N, TILE, PITCH, true>(lds2, tw);
    const R uscale = (EPI == EPI_HL && use_invnP) ? (R)st->invnP : (R)1;
    for (int e = threadIdx.x; e < TILE * N; e += NT) {
        const int l = e / N, m = e - l * N;
        const long long go = (((long long)c * B + bb) * Cc + c0 + l) * N + m;
        cpx<R> v = lds[l * PITCH + m];
        if (EPI == EPI_SCALE) {
            out[go] = (R)scale * v;
        } else if (EPI == EPI_HL) {
            const int ix = m, iy = c0 + l, iz = bb;
            const double x = -p.L[0] + ix * p.h[0];
            const double y = -p.L[1] + iy * p.h[1];
            const double z = p.dim == 3 ? -p.L[2] + iz * p.h[2] : 0.0;
            double V2, V4;
            trap_at(p, go - (long long)c * p.M, x, y, z, V2, V4);
            const cpx<R> u = uscale * uin[go];
            v = v + (R)(V2 + V4) * u;
            if (nin == 2) v = v - (R)(p.omega * x) * lds2[l * PITCH + m];
            out[go] = v;
        } else if (EPI == EPI_ROTX) {
            if (nin == 2) {
                const int jx = bb, iy = m;
                const double kx = wavenum(jx, p.n[0], p.L[0]);
                const double y = -p.L[1] + iy * p.h[1];
                v = v + (R)(p.omega * y * kx / p.n[0]) * uin[go];
                out2[go] = lds2[l * PITCH + m];
            }
            out[go] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// last pass of the preconditioner: P r = P_V^{1/2} (inverse transform), with the
// partial sums of the direction reductions of the next step fused in
// (Re<r,Pr>, Re<r_prev,Pr>, Re<phi,Pr>, |Pr|^2, Re<Pr,P^{n-1}>).
// ---------------------------------------------------------------------------
template <typename R, int N, int TILE>
__global__ __launch_bounds__(NT) void k_invT_pre(const Slot<R>* __restrict__ slots, int iin, int iout, int B,
                                                 int Cc, int dir, const cpx<R>* __restrict__ tw) {
    const Slot<R>& S = slots[blockIdx.y];
    SolveState* st = S.st;
    if (st->done) return;
    const cpx<R>* __restrict__ in = S.buf[iin];
    cpx<R>* __restrict__ out = S.buf[iout];
    const R* __restrict__ pv = S.pv;
    constexpr int PITCH = N + 1;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    const int tiles = Cc / TILE;
    int blk = blockIdx.x;
    const int ct = blk % tiles;
    blk /= tiles;
    const int bb = blk % B;
    const int c = blk / B;
    const int c0 = ct * TILE;
    for (int e = threadIdx.x; e < TILE * N; e += NT) {
        const int l = e % TILE, m = e / TILE;
        lds[l * PITCH + m] = in[(((long long)c * N + m) * B + bb) * Cc + c0 + l];
    }
    __syncthreads();
    lds_fft<R, N, TILE, PITCH, true>(lds, tw);
    double acc[NS_DIR] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const cpx<R>* r = dir ? S.buf[B_R0 + st->cur] : nullptr;
    const cpx<R>* rp = dir ? S.buf[B_R0 + (st->cur ^ 1)] : nullptr;
    const cpx<R>* phi = S.buf[B_PHI];
    const cpx<R>* Pprev = S.buf[B_P];
    for (int e = threadIdx.x; e < TILE * N; e += NT) {
        const int l = e / N, m = e - l * N;
        const long long go = (((long long)c * B + bb) * Cc + c0 + l) * N + m;
        const cpx<R> v = pv[go] * lds[l * PITCH + m];
        out[go] = v;
        if (dir) {
            const cpx<double> w = wid(v);
            acc[0] += re_dot(wid(r[go]), w);
            acc[1] += re_dot(wid(rp[go]), w);
            acc[2] += re_dot(wid(phi[go]), w);
            acc[3] += cabs2(w);
            acc[4] += re_dot(wid(Pprev[go]), w);
        }
    }
    if (!dir) return;
    block_row<NS_DIR>(acc, S.red_dir, RED_DIR_STRIDE);
}

// ---------------------------------------------------------------------------
// middle pass: spectral operators acting on all three components at each k
// ---------------------------------------------------------------------------
//   MID_HL:  A = (1/2 |k|^2 - gamma S(k)) v / M, B = k_y v / M (rotation only),
//            S(k) = [[0, s0, 0], [s1, 0, s0], [0, s1, 0]], s0 = -k_x + i k_y (L0),
//            s1 = -k_x - i k_y (L1); block sums of 1/2|k|^2 |v_l|^2 and Re v^dag S v.
//            In 2D the rotation term Omega y k_x C / Nx (C the input, x-transformed
//            and y-physical) is added to A after the inverse transform.
//   MID_HLX: as MID_HL for v = P^, and in2 holds the spectrum of Phi: block sums
//            of 1/2|k|^2 |Phi^_l|^2, 1/2|k|^2 Re Phi^_l conj(v_l), 1/2|k|^2 |v_l|^2.
//   MID_PRE: A = v_l / (alpha_l + 1/2 |k|^2) / M.
template <typename R, int N, int LPB, int OP>
__global__ __launch_bounds__(NT) void k_mid(const Slot<R>* __restrict__ slots, int iin, int ioutA, int ioutB,
                                            int nlines, int rot_any, const cpx<R>* __restrict__ tw) {
    const Slot<R>& S = slots[blockIdx.y];
    const SolveState* st = S.st;
    if (st->done) return;
    const Phys p = S.p;
    const int rot = rot_any && p.omega != 0.0;
    const cpx<R>* __restrict__ in = S.buf[iin];
    const cpx<R>* __restrict__ in2 = (OP == MID_HLX) ? in + 3 * p.M : nullptr;
    cpx<R>* __restrict__ outA = S.buf[ioutA];
    cpx<R>* __restrict__ outB = ioutB >= 0 ? S.buf[ioutB] : nullptr;
    double* __restrict__ red = S.red_mid;
    constexpr int PITCH = N + 1;
    constexpr int NLN = 3 * LPB;
    constexpr bool HL = OP == MID_HL || OP == MID_HLX;
    constexpr bool X2 = OP == MID_HLX;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cpx<R>* X = reinterpret_cast<cpx<R>*>(smem_raw);
    cpx<R>* Z = X + NLN * PITCH;                       // spectrum of Phi (MID_HLX)
    cpx<R>* Y = X + (X2 ? 2 : 1) * NLN * PITCH;        // rotation output B
    const bool doB = HL && rot;
    const int l0 = blockIdx.x * LPB;
    const long long cs = (long long)nlines * N;
    for (int e = threadIdx.x; e < NLN * N; e += NT) {
        const int L = e / N, m = e - L * N;
        const int c = L / LPB, q = L - c * LPB;
        const long long gi = c * cs + (long long)(l0 + q) * N + m;
        X[L * PITCH + m] = in[gi];
        if (X2) Z[L * PITCH + m] = in2[gi];
    }
    __syncthreads();
    lds_fft<R, N, (X2 ? 2 : 1) * NLN, PITCH, false>(X, tw);
    const double invM = 1.0 / (double)p.M;
    double acc[X2 ? NS_KIN : 4];
    for (int k = 0; k < (X2 ? NS_KIN : 4); ++k) acc[k] = 0.0;
    double al[3] = {0.0, 0.0, 0.0}, fl = 0.0;
    if (OP == MID_PRE) {
        al[0] = st->alpha[0]; al[1] = st->alpha[1]; al[2] = st->alpha[2];
        fl = 1e-12 * fmax(1.0, fmax(al[0], fmax(al[1], al[2])));
    }
    for (int e = threadIdx.x; e < LPB * N; e += NT) {
        const int q = e / N, m = e - q * N;
        const int line = l0 + q;
        double kx, ky, kz;
        if (p.dim == 2) {
            kx = wavenum(line, p.n[0], p.L[0]);
            ky = wavenum(m, p.n[1], p.L[1]);
            kz = 0.0;
        } else {
            kx = wavenum(line % p.n[0], p.n[0], p.L[0]);
            ky = wavenum(line / p.n[0], p.n[1], p.L[1]);
            kz = wavenum(m, p.n[2], p.L[2]);
        }
        const double K = 0.5 * (kx * kx + ky * ky + kz * kz);
        cpx<R>* x0 = X + (0 * LPB + q) * PITCH + m;
        cpx<R>* x1 = X + (1 * LPB + q) * PITCH + m;
        cpx<R>* x2 = X + (2 * LPB + q) * PITCH + m;
        if (HL) {
            const cpx<double> v0 = wid(*x0), v1 = wid(*x1), v2 = wid(*x2);
            const cpx<double> s0 = cmk(-kx, ky), s1 = cmk(-kx, -ky);
            const cpx<double> S0 = cmul(s0, v1);
            const cpx<double> S1 = cmul(s1, v0) + cmul(s0, v2);
            const cpx<double> S2 = cmul(s1, v1);
            if (X2) {
                const cpx<double> v[3] = {v0, v1, v2};
                for (int cc = 0; cc < 3; ++cc) {
                    const cpx<double> z = wid(Z[(cc * LPB + q) * PITCH + m]);
                    acc[3 * cc] += K * cabs2(z);
                    acc[3 * cc + 1] += K * re_dot(z, v[cc]);
                    acc[3 * cc + 2] += K * cabs2(v[cc]);
                }
            } else {
                acc[0] += K * cabs2(v0);
                acc[1] += K * cabs2(v1);
                acc[2] += K * cabs2(v2);
                acc[3] += cmulc(S0, v0).x + cmulc(S1, v1).x + cmulc(S2, v2).x;
            }
            const double gm = p.gamma;
            const cpx<double> a0 = invM * (K * v0 - gm * S0);
            const cpx<double> a1 = invM * (K * v1 - gm * S1);
            const cpx<double> a2 = invM * (K * v2 - gm * S2);
            if (doB) {
                const double fb = ky * invM;
                Y[(0 * LPB + q) * PITCH + m] = cmk((R)(fb * v0.x), (R)(fb * v0.y));
                Y[(1 * LPB + q) * PITCH + m] = cmk((R)(fb * v1.x), (R)(fb * v1.y));
                Y[(2 * LPB + q) * PITCH + m] = cmk((R)(fb * v2.x), (R)(fb * v2.y));
            }
            *x0 = cmk((R)a0.x, (R)a0.y);
            *x1 = cmk((R)a1.x, (R)a1.y);
            *x2 = cmk((R)a2.x, (R)a2.y);
        } else {
            const R d0 = (R)(invM / fmax(al[0] + K, fl));
            const R d1 = (R)(invM / fmax(al[1] + K, fl));
            const R d2 = (R)(invM / fmax(al[2] + K, fl));
            *x0 = d0 * *x0;
            *x1 = d1 * *x1;
            *x2 = d2 * *x2;
        }
    }
    __syncthreads();
    lds_fft<R, N, NLN, PITCH, true>(X, tw);
    if (doB) lds_fft<R, N, NLN, PITCH, true>(Y, tw);
    const bool rot2d = HL && rot && p.dim == 2;
    for (int e = threadIdx.x; e < NLN * N; e += NT) {
        const int L = e / N, m = e - L * N;
        const int c = L / LPB, q = L - c * LPB;
        const long long go = c * cs + (long long)(l0 + q) * N + m;
        cpx<R> v = X[L * PITCH + m];
        if (rot2d) {
            const double kx = wavenum(l0 + q, p.n[0], p.L[0]);
            const double y = -p.L[1] + m * p.h[1];
            v = v + (R)(p.omega * y * kx / p.n[0]) * in[go];
        }
        outA[go] = v;
        if (doB) outB[go] = Y[L * PITCH + m];
    }
    if (HL) block_row<(X2 ? NS_KIN : 4)>(acc, red, RED_MID_STRIDE);
}

// ---------------------------------------------------------------------------
// launch configuration (tiles sized so that small grids still give >= ~200
// blocks and each block's LDS stays near or under 64 KB)
// ---------------------------------------------------------------------------
template <typename R> constexpr int tile_fwd(int N) {
    return sizeof(R) == 8 ? (N >= 1024 ? 2 : 4) : (N >= 1024 ? 4 : 8);
}
template <typename R> constexpr int tile_inv(int N) {
    return sizeof(R) == 8 ? (N >= 512 ? 2 : 4) : (N >= 512 ? 4 : 8);
}
constexpr int lpb_mid(int N) { return N >= 256 ? 1 : (N >= 128 ? 2 : (N >= 64 ? 4 : 8)); }

int mid_blocks(int N, int nlines) { return nlines / lpb_mid(N); }
template <typename R> int invT_pre_blocks(int N, int B, int Cc) { return 3 * B * (Cc / tile_inv<R>(N)); }
template int invT_pre_blocks<double>(int, int, int);
template int invT_pre_blocks<float>(int, int, int);

template <typename R, int N>
static hipError_t fwdT_n(int pro, int dual, const Slot<R>* slots, int nslots, int in, int out, int aux0, int aux1,
                         int A, int B, int ncomp, const cpx<R>* tw, hipStream_t s) {
    constexpr int TILE = tile_fwd<R>(N);
    if (B % TILE) return hipErrorInvalidValue;
    if (dual && pro != PRO_DIR) return hipErrorInvalidValue;
    const size_t lds = (size_t)TILE * (N + 1) * sizeof(cpx<R>);
    dim3 grid((unsigned)((long long)(dual ? 6 : ncomp) * A * (B / TILE)), (unsigned)nslots);
    if (dual) {
        GS_LAUNCH((k_fwdT<R, N, TILE, PRO_DIR, true>), grid, dim3(NT), lds, s, slots, in, out, aux0, aux1, A, B, tw);
        return hipGetLastError();
    }
    switch (pro) {
    case PRO_PLAIN:
        GS_LAUNCH((k_fwdT<R, N, TILE, PRO_PLAIN, false>), grid, dim3(NT), lds, s, slots, in, out, aux0, aux1, A, B, tw);
        break;
    case PRO_UPDATE:
        GS_LAUNCH((k_fwdT<R, N, TILE, PRO_UPDATE, false>), grid, dim3(NT), lds, s, slots, in, out, aux0, aux1, A, B, tw);
        break;
    case PRO_DIR:
        GS_LAUNCH((k_fwdT<R, N, TILE, PRO_DIR, false>), grid, dim3(NT), lds, s, slots, in, out, aux0, aux1, A, B, tw);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R, int N>
static hipError_t invT_n(int epi, const Slot<R>* slots, int nslots, int in, int in2, int out, int out2, int uin,
                         int B, int Cc, double scale, int use_invnP, int rot_any, const cpx<R>* tw, hipStream_t s) {
    constexpr int TILE = tile_inv<R>(N);
    if (Cc % TILE) return hipErrorInvalidValue;
    const size_t lds = (size_t)(epi == EPI_SCALE ? 1 : 2) * TILE * (N + 1) * sizeof(cpx<R>);
    dim3 grid((unsigned)(3LL * B * (Cc / TILE)), (unsigned)nslots);
    switch (epi) {
    case EPI_SCALE:
        GS_LAUNCH((k_invT<R, N, TILE, EPI_SCALE>), grid, dim3(NT), lds, s, slots, in, in2, out, out2, uin, B, Cc, scale, use_invnP, rot_any, tw);
        break;
    case EPI_HL:
        GS_LAUNCH((k_invT<R, N, TILE, EPI_HL>), grid, dim3(NT), lds, s, slots, in, in2, out, out2, uin, B, Cc, scale, use_invnP, rot_any, tw);
        break;
    case EPI_ROTX:
        GS_LAUNCH((k_invT<R, N, TILE, EPI_ROTX>), grid, dim3(NT), lds, s, slots, in, in2, out, out2, uin, B, Cc, scale, use_invnP, rot_any, tw);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R, int N>
static hipError_t invT_pre_n(const Slot<R>* slots, int nslots, int in, int out, int B, int Cc, int dir,
                             const cpx<R>* tw, hipStream_t s) {
    constexpr int TILE = tile_inv<R>(N);
    if (Cc % TILE) return hipErrorInvalidValue;
    const size_t lds = (size_t)TILE * (N + 1) * sizeof(cpx<R>);
    dim3 grid((unsigned)(3LL * B * (Cc / TILE)), (unsigned)nslots);
    static_assert(NS_DIR <= RED_DIR_STRIDE, "partial-sum row");
    GS_LAUNCH((k_invT_pre<R, N, TILE>), grid, dim3(NT), lds, s, slots, in, out, B, Cc, dir, tw);
    return hipGetLastError();
}

template <typename R, int N>
static hipError_t mid_n(int op, const Slot<R>* slots, int nslots, int in, int outA, int outB, int nlines,
                        int rot_any, const cpx<R>* tw, hipStream_t s) {
    constexpr int LPB = lpb_mid(N);
    if (nlines % LPB) return hipErrorInvalidValue;
    const int nB = ((op == MID_HL || op == MID_HLX) && rot_any) ? 1 : 0;
    const int nX = op == MID_HLX ? 2 : 1;
    const size_t lds = (size_t)(nB + nX) * 3 * LPB * (N + 1) * sizeof(cpx<R>);
    dim3 grid((unsigned)(nlines / LPB), (unsigned)nslots);
    if (op == MID_HL)
        GS_LAUNCH((k_mid<R, N, LPB, MID_HL>), grid, dim3(NT), lds, s, slots, in, outA, outB, nlines, rot_any, tw);
    else if (op == MID_HLX)
        GS_LAUNCH((k_mid<R, N, LPB, MID_HLX>), grid, dim3(NT), lds, s, slots, in, outA, outB, nlines, rot_any, tw);
    else
        GS_LAUNCH((k_mid<R, N, LPB, MID_PRE>), grid, dim3(NT), lds, s, slots, in, outA, outB, nlines, 0, tw);
    return hipGetLastError();
}

#define GS_SWITCH_N(CALL)                        \
    switch (N) {                                 \
    case 16: return CALL(16);                    \
    case 32: return CALL(32);                    \
    case 64: return CALL(64);                    \
    case 128: return CALL(128);                  \
    case 256: return CALL(256);                  \
    case 512: return CALL(512);                  \
    case 1024: return CALL(1024);                \
    default: return hipErrorInvalidValue;        \
    }

template <typename R>
hipError_t launch_fwdT(int N, int pro, int dual, const Slot<R>* slots, int nslots, int in, int out, int aux0,
                       int aux1, int A, int B, int ncomp, const cpx<R>* tw, hipStream_t s) {
#define CALL(n) fwdT_n<R, n>(pro, dual, slots, nslots, in, out, aux0, aux1, A, B, ncomp, tw, s)
    GS_SWITCH_N(CALL)
#undef CALL
}

template <typename R>
hipError_t launch_invT(int N, int epi, const Slot<R>* slots, int nslots, int in, int in2, int out, int out2,
                       int uin, int B, int Cc, double scale, int use_invnP, int rot_any, const cpx<R>* tw,
                       hipStream_t s) {
#define CALL(n) invT_n<R, n>(epi, slots, nslots, in, in2, out, out2, uin, B, Cc, scale, use_invnP, rot_any, tw, s)
    GS_SWITCH_N(CALL)
#undef CALL
}

template <typename R>
hipError_t launch_invT_pre(int N, const Slot<R>* slots, int nslots, int in, int out, int B, int Cc, int dir,
                           const cpx<R>* tw, hipStream_t s) {
#define CALL(n) invT_pre_n<R, n>(slots, nslots, in, out, B, Cc, dir, tw, s)
    GS_SWITCH_N(CALL)
#undef CALL
}

template <typename R>
hipError_t launch_mid(int N, int op, const Slot<R>* slots, int nslots, int in, int outA, int outB, int nlines,
                      int rot_any, const cpx<R>* tw, hipStream_t s) {
#define CALL(n) mid_n<R, n>(op, slots, nslots, in, outA, outB, nlines, rot_any, tw, s)
    GS_SWITCH_N(CALL)
#undef CALL
}

#define GS_INST_FFT(R)                                                                                           \
    template hipError_t launch_fwdT<R>(int, int, int, const Slot<R>*, int, int, int, int, int, int, int, int,     \
                                       const cpx<R>*, hipStream_t);                                              \
    template hipError_t launch_invT<R>(int, int, const Slot<R>*, int, int, int, int, int, int, int, int, double,  \
                                       int, int, const cpx<R>*, hipStream_t);                                    \
    template hipError_t launch_invT_pre<R>(int, const Slot<R>*, int, int, int, int, int, int, const cpx<R>*,      \
                                           hipStream_t);                                                         \
    template hipError_t launch_mid<R>(int, int, const Slot<R>*, int, int, int, int, int, int, const cpx<R>*,      \
                                      hipStream_t);
GS_INST_FFT(double)
GS_INST_FFT(float)

}  // namespace gs
