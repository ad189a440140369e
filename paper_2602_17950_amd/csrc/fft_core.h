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
#pragma once
#include "device_common.h"
#include "control.h"

namespace gs {

// threads per block: a template parameter NT of each kernel (whole waves)

// LDS layout of a line of N complex values: element e at e + e/16 (one pad
// slot per 16), lines PITCH apart (odd). Radix-16 passes write with stride 16
// and the transposed global accesses read columns; both then fall on distinct
// banks.
template <int N> struct Lay {
    static constexpr int P = (N + N / 16) | 1;
};
__device__ __forceinline__ int lx(int e) { return e + (e >> 4); }
__host__ __device__ constexpr int lxc(int e) { return e + (e >> 4); }

// Whether the LDS offsets of the RAD values of a Stockham butterfly (see
// fft_pass) from its first value are the same for every butterfly j: the
// reads at j + r N/RAD (RD), the writes at db + r NS, db = (j - k) RAD + k,
// k = j mod NS (WR). Checked at compile time over every j.
template <int N, int RAD, int NS> struct PassIdx {
    static constexpr int NB = N / RAD;
    static constexpr bool rd() {
        for (int j = 0; j < NB; ++j)
            for (int r = 1; r < RAD; ++r)
                if (lxc(j + r * NB) - lxc(j) != lxc(r * NB)) return false;
        return true;
    }
    static constexpr bool wr() {
        for (int j = 0; j < NB; ++j) {
            const int k = j % NS, db = (j - k) * RAD + k;
            for (int r = 1; r < RAD; ++r)
                if (lxc(db + r * NS) - lxc(db) != lxc(r * NS)) return false;
        }
        return true;
    }
    static constexpr bool RD = rd(), WR = wr();
};

// Workgroups are dispatched to the 8 XCDs in turn, and each XCD has its own
// L2. The transposed passes read tiles of TILE values per line position, 32
// or 64 bytes: two neighbouring tiles share every 128-byte line. This map
// hands each XCD a contiguous range of tiles in order (when the grid width is
// a multiple of 8), so the two halves of a line are read by blocks of one XCD
// at about the same time instead of being fetched once by each of two XCDs.
__device__ __forceinline__ int xcd_block(int b, int G) {
    return (G & 7) ? b : (b & 7) * (G >> 3) + (b >> 3);
}

template <typename R, bool INV>
__device__ __forceinline__ cpx<R> twid(const cpx<R>* __restrict__ tw, int m) {
    cpx<R> w = tw[m];
    if (INV) w.y = -w.y;
    return w;
}

// exp(-2 pi i m / 16) (cos, -sin), m = 0..15
__host__ __device__ constexpr double w16c(int m) {
    switch (m & 15) {
    case 0: return 1.0;
    case 1: return 0.923879532511286756128;
    case 2: return 0.707106781186547524401;
    case 3: return 0.382683432365089771728;
    case 4: return 0.0;
    case 5: return -0.382683432365089771728;
    case 6: return -0.707106781186547524401;
    case 7: return -0.923879532511286756128;
    case 8: return -1.0;
    case 9: return -0.923879532511286756128;
    case 10: return -0.707106781186547524401;
    case 11: return -0.382683432365089771728;
    case 12: return 0.0;
    case 13: return 0.382683432365089771728;
    case 14: return 0.707106781186547524401;
    default: return 0.923879532511286756128;
    }
}
__host__ __device__ constexpr double w16s(int m) { return -w16c((m & 15) + 12); }   // -sin = cos(. + 3/4 turn)

// v * exp(-+2 pi i m / 16) for a compile-time m (after unrolling)
template <typename R, bool INV>
__device__ __forceinline__ cpx<R> rot16(cpx<R> v, int m) {
    m &= 15;
    if (m == 0) return v;
    if (m == 8) return cmk(-v.x, -v.y);
    if (m == 4) return INV ? cmk(-v.y, v.x) : cmk(v.y, -v.x);     // * (+-i)
    if (m == 12) return INV ? cmk(v.y, -v.x) : cmk(-v.y, v.x);
    const R c = (R)w16c(m), sn = (R)(INV ? -w16s(m) : w16s(m));
    return cmk(v.x * c - v.y * sn, v.x * sn + v.y * c);
}

// in-place DFT of RAD values in registers, kernel exp(-+2 pi i r q / RAD)
template <typename R, bool INV>
__device__ __forceinline__ void dft2(cpx<R>& a, cpx<R>& b) {
    const cpx<R> t = a - b;
    a = a + b;
    b = t;
}
template <typename R, bool INV>
__device__ __forceinline__ void dft4(cpx<R>& v0, cpx<R>& v1, cpx<R>& v2, cpx<R>& v3) {
    const cpx<R> a = v0 + v2, b = v0 - v2, c = v1 + v3, d = v1 - v3;
    const cpx<R> id = cmuli(d);
    v0 = a + c;
    v2 = a - c;
    if (INV) { v1 = b + id; v3 = b - id; }
    else     { v1 = b - id; v3 = b + id; }
}
// RAD = A * B with r = r1 + A r2, q = q2 + B q1: DFT_B over r2, twiddle
// exp(-+2 pi i r1 q2 / RAD), DFT_A over r1.
template <typename R, int RAD, bool INV>
__device__ __forceinline__ void dftr(cpx<R> (&v)[RAD]) {
    if constexpr (RAD == 2) {
        dft2<R, INV>(v[0], v[1]);
    } else if constexpr (RAD == 3) {
        // y_q = sum_r v_r w^{rq}, w = exp(-+2 pi i / 3) = -1/2 -+ i sqrt(3)/2
        const R h = (R)0.866025403784438646763723170752936183;   // sqrt(3)/2
        const cpx<R> s = v[1] + v[2], d = v[1] - v[2];
        const cpx<R> m = v[0] - (R)0.5 * s;
        const cpx<R> id = cmk(-h * d.y, h * d.x);   // i sqrt(3)/2 (v1 - v2)
        v[0] = v[0] + s;
        if (INV) { v[1] = m + id; v[2] = m - id; }
        else     { v[1] = m - id; v[2] = m + id; }
    } else if constexpr (RAD == 4) {
        dft4<R, INV>(v[0], v[1], v[2], v[3]);
    } else if constexpr (RAD == 5) {
        // y_q = sum_r v_r w^{rq}, w = exp(-+2 pi i / 5): with t1 = v1 + v4,
        // t2 = v2 + v3, t3 = v1 - v4, t4 = v2 - v3, the cosines and sines of
        // 2 pi / 5 and 4 pi / 5 give y1,4 = v0 + c1 t1 + c2 t2 -+ i (s1 t3 + s2 t4)
        // and y2,3 = v0 + c2 t1 + c1 t2 -+ i (s2 t3 - s1 t4) (upper signs forward)
        const R c1 = (R)0.309016994374947424102293417182819059, c2 = (R)-0.809016994374947424102293417182819059;
        const R s1 = (R)0.951056516295153572116439333379382143, s2 = (R)0.587785252292473129168705954639072769;
        const cpx<R> t1 = v[1] + v[4], t2 = v[2] + v[3], t3 = v[1] - v[4], t4 = v[2] - v[3];
        const cpx<R> a1 = v[0] + c1 * t1 + c2 * t2, a2 = v[0] + c2 * t1 + c1 * t2;
        const cpx<R> b1 = s1 * t3 + s2 * t4, b2 = s2 * t3 - s1 * t4;
        const cpx<R> ib1 = cmuli(b1), ib2 = cmuli(b2);   // i b1, i b2
        v[0] = v[0] + t1 + t2;
        if (INV) { v[1] = a1 + ib1; v[4] = a1 - ib1; v[2] = a2 + ib2; v[3] = a2 - ib2; }
        else     { v[1] = a1 - ib1; v[4] = a1 + ib1; v[2] = a2 - ib2; v[3] = a2 + ib2; }
    } else if constexpr (RAD == 8) {
        // A = 2, B = 4
        cpx<R> y[2][4];
#pragma unroll
        for (int r1 = 0; r1 < 2; ++r1) {
            y[r1][0] = v[r1]; y[r1][1] = v[r1 + 2]; y[r1][2] = v[r1 + 4]; y[r1][3] = v[r1 + 6];
            dft4<R, INV>(y[r1][0], y[r1][1], y[r1][2], y[r1][3]);
        }
#pragma unroll
        for (int q2 = 1; q2 < 4; ++q2) y[1][q2] = rot16<R, INV>(y[1][q2], 2 * q2);
#pragma unroll
        for (int q2 = 0; q2 < 4; ++q2) {
            dft2<R, INV>(y[0][q2], y[1][q2]);
            v[q2] = y[0][q2];
            v[q2 + 4] = y[1][q2];
        }
    } else {
        static_assert(RAD == 16, "radix 2, 3, 4, 5, 8 or 16");
        // A = 4, B = 4
        cpx<R> y[4][4];
#pragma unroll
        for (int r1 = 0; r1 < 4; ++r1) {
            y[r1][0] = v[r1]; y[r1][1] = v[r1 + 4]; y[r1][2] = v[r1 + 8]; y[r1][3] = v[r1 + 12];
            dft4<R, INV>(y[r1][0], y[r1][1], y[r1][2], y[r1][3]);
        }
#pragma unroll
        for (int r1 = 1; r1 < 4; ++r1)
#pragma unroll
            for (int q2 = 1; q2 < 4; ++q2) y[r1][q2] = rot16<R, INV>(y[r1][q2], r1 * q2);
#pragma unroll
        for (int q2 = 0; q2 < 4; ++q2) {
            dft4<R, INV>(y[0][q2], y[1][q2], y[2][q2], y[3][q2]);
#pragma unroll
            for (int q1 = 0; q1 < 4; ++q1) v[q2 + 4 * q1] = y[q1][q2];
        }
    }
}

// One Stockham pass of radix RAD on NL lines of N values (in LDS, layout Lay):
// butterfly j of a line reads x[j + r N/RAD], applies the twiddles of the
// pass, transforms, and writes to (j - k) RAD + k + r NS with k = j mod NS
// (NS = product of the radices of the earlier passes). tw[m] = exp(-2 pi i m / N).
// When the LDS offsets of a butterfly's RAD reads (or writes) from its first
// one are the same for every butterfly, they are compile-time constants.
template <typename R, int N, int NL, int NT, int RAD, int NS, bool INV>
__device__ __forceinline__ void fft_pass(cpx<R>* buf, const cpx<R>* __restrict__ tw) {
    using PI = PassIdx<N, RAD, NS>;
    constexpr int NB = N / RAD;
    constexpr int TOT = NL * NB;
    constexpr int BPT = (TOT + NT - 1) / NT;
    constexpr int P = Lay<N>::P;
    constexpr int TWS = N / (NS * RAD);
    cpx<R> v[BPT][RAD];
    int lb[BPT], db[BPT];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int b = threadIdx.x + i * NT;
        lb[i] = -1;
        if (TOT % NT == 0 || b < TOT) {
            const int l = b / NB, j = b - l * NB;
            const int k = j % NS;
            const cpx<R>* src = buf + l * P;
            if constexpr (PI::RD) {
                const cpx<R>* s0 = src + lx(j);
#pragma unroll
                for (int r = 0; r < RAD; ++r) v[i][r] = s0[lxc(r * NB)];
            } else {
#pragma unroll
                for (int r = 0; r < RAD; ++r) v[i][r] = src[lx(j + r * NB)];
            }
            if constexpr (NS > 1) {
                // (forming the powers costs less than loading each from the
                // table: measured)
                if constexpr (sizeof(R) == 4) {
                    // float: the running product in double from the double table
                    // that follows the float one (N entries on), each power
                    // rounded once: correctly rounded twiddles from one load
                    const cpx<double>* twd = reinterpret_cast<const cpx<double>*>(tw + N);
                    const cpx<double> w1 = twid<double, INV>(twd, k * TWS);
                    cpx<double> w = w1;
#pragma unroll
                    for (int r = 1; r < RAD; ++r) {
                        v[i][r] = cmul(v[i][r], cmk((R)w.x, (R)w.y));
                        if (r + 1 < RAD) w = cmul(w, w1);
                    }
                } else {
                    // double: w^r as a running product of one table value (at most
                    // 7 products, ~1e-15 relative)
                    const cpx<R> w1 = twid<R, INV>(tw, k * TWS);
                    cpx<R> w = w1;
#pragma unroll
                    for (int r = 1; r < RAD; ++r) {
                        v[i][r] = cmul(v[i][r], w);
                        if (r + 1 < RAD) w = cmul(w, w1);
                    }
                }
            }
            dftr<R, RAD, INV>(v[i]);
            lb[i] = l * P;
            db[i] = (j - k) * RAD + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        if (lb[i] >= 0) {
            if constexpr (PI::WR) {
                cpx<R>* d0 = buf + lb[i] + lx(db[i]);
#pragma unroll
                for (int r = 0; r < RAD; ++r) d0[lxc(r * NS)] = v[i][r];
            } else {
#pragma unroll
                for (int r = 0; r < RAD; ++r) buf[lb[i] + lx(db[i] + r * NS)] = v[i][r];
            }
        }
    }
    __syncthreads();
}

// For N divisible by 3 one radix-3 pass first (NS = 1: no twiddles), then a
// radix-5 pass for every factor 5, then passes of radix RMAX while it divides
// the rest, then one pass of the remaining power of two (NS = product of the
// radices done so far).
template <typename R, int N, int NL, int NT, int RMAX, int NS, bool INV>
__device__ __forceinline__ void fft_passes(cpx<R>* buf, const cpx<R>* __restrict__ tw) {
    constexpr int REST = N / NS;
    if constexpr (NS == 1 && N % 3 == 0) {
        fft_pass<R, N, NL, NT, 3, 1, INV>(buf, tw);
        fft_passes<R, N, NL, NT, RMAX, 3, INV>(buf, tw);
    } else if constexpr (REST % 5 == 0) {
        fft_pass<R, N, NL, NT, 5, NS, INV>(buf, tw);
        fft_passes<R, N, NL, NT, RMAX, NS * 5, INV>(buf, tw);
    } else if constexpr (REST >= RMAX) {
        fft_pass<R, N, NL, NT, RMAX, NS, INV>(buf, tw);
        fft_passes<R, N, NL, NT, RMAX, NS * RMAX, INV>(buf, tw);
    } else if constexpr (REST > 1) {
        fft_pass<R, N, NL, NT, REST, NS, INV>(buf, tw);
    }
}

// N = 2^a 3^b 5^c with b <= 1 and c <= 2 (the factors the passes handle)
template <int N> struct Pow2Part {
    static constexpr int odd = (N % 3 == 0 ? 3 : 1) * (N % 25 == 0 ? 25 : (N % 5 == 0 ? 5 : 1));
    static constexpr int p2 = N / odd;
    static constexpr bool odd_ok = N % odd == 0 && (p2 & (p2 - 1)) == 0 && p2 >= 2;
};

// Largest radix per pass: 16 in float; 8 in double, which halves the
// registers a butterfly holds and so keeps more waves resident.
template <typename R> constexpr int rmax() { return sizeof(R) == 8 ? 8 : 16; }

// Transform NL lines of length N held in LDS (layout Lay<N>, line l at
// buf + l * Lay<N>::P; natural order in and out, unnormalised). The
// radices, and so the bits of the result, do not depend on NT.
template <typename R, int N, int NL, int NT, bool INV>
__device__ __forceinline__ void lds_fft(cpx<R>* buf, const cpx<R>* __restrict__ tw) {
    static_assert(N >= 16 && N <= 2400 && Pow2Part<N>::odd_ok, "N = 2^a 3^b 5^c, b <= 1, c <= 2");
    fft_passes<R, N, NL, NT, rmax<R>(), 1, INV>(buf, tw);
}

// one complex value as a single vector access (keeps register arrays of
// complex values out of private memory)
template <typename R> using vec2 = R __attribute__((ext_vector_type(2)));
template <typename R> __device__ __forceinline__ void ld2(cpx<R>& d, const cpx<R>* p) {
    const vec2<R> v = *reinterpret_cast<const vec2<R>*>(p);
    d.x = v.x;
    d.y = v.y;
}
template <typename R> __device__ __forceinline__ void st2(cpx<R>* p, const cpx<R>& a) {
    vec2<R> v;
    v.x = a.x;
    v.y = a.y;
    *reinterpret_cast<vec2<R>*>(p) = v;
}

// Transposed passes (invT, invT_pre): a unit is one tile of TILE lines of one
// component. A block takes units b, b + G, ... (b in the XCD order); when
// the prefetch of the next unit's input takes at most 32 registers, the
// next unit is loaded while the current one is transformed and the twiddle
// tables are read from a copy in LDS.
template <typename R, int N, int TILE, int NT> struct TilePlan {
    static constexpr int EPT = (TILE * N + NT - 1) / NT;
    static constexpr bool PIPE = 2 * EPT * (int)sizeof(cpx<R>) <= 128;
    static constexpr size_t TW_BYTES =
        PIPE ? (size_t)N * sizeof(cpx<R>) + (sizeof(R) == 4 ? (size_t)N * 16 : 0) : 0;
    __host__ __device__ static constexpr size_t tw_offset(int nbuf) {
        return ((size_t)nbuf * TILE * Lay<N>::P * sizeof(cpx<R>) + 15) & ~(size_t)15;
    }
};

template <typename R, int N, int TILE, int NT>
__device__ __forceinline__ void tile_fetch(const cpx<R>* __restrict__ in, const cpx<R>* __restrict__ in2, int nin,
                                           long long base, int B, int Cc,
                                           cpx<R> (&a)[TilePlan<R, N, TILE, NT>::EPT],
                                           cpx<R> (&b)[TilePlan<R, N, TILE, NT>::EPT]) {
#pragma unroll
    for (int i = 0; i < TilePlan<R, N, TILE, NT>::EPT; ++i) {
        const int e = threadIdx.x + i * NT;
        if (TILE * N % NT == 0 || e < TILE * N) {
            const int l = e % TILE, m = e / TILE;
            const long long gi = base + (long long)m * B * Cc + l;
            ld2(a[i], in + gi);
            if (nin == 2) ld2(b[i], in2 + gi);
        }
    }
}
// unit u -> component c, position bb and first line c0 of its tile
__device__ __forceinline__ void tile_unit(int u, int tiles, int B, int TILE_, int& c, int& bb, int& c0) {
    const int ct = u % tiles;
    const int blk = u / tiles;
    bb = blk % B;
    c = blk / B;
    c0 = ct * TILE_;
}
// copy of the twiddle table(s) into LDS (16-byte chunks)
template <typename R, int N>
__device__ __forceinline__ void tw_to_lds(cpx<R>* dst, const cpx<R>* __restrict__ tw, size_t bytes, int nt) {
    for (int e = threadIdx.x; e < (int)(bytes / 16); e += nt)
        reinterpret_cast<vec2<double>*>(dst)[e] = reinterpret_cast<const vec2<double>*>(tw)[e];
}

// ---------------------------------------------------------------------------
// forward pass with transposed store
// ---------------------------------------------------------------------------
// DUAL (with PRO_DIR): components 3..5 of the output are the plain transform
// of aux1 (Phi), so that the middle pass sees both spectra.
template <typename R, typename RX, int N, int TILE, int PRO, bool DUAL, int NT>
__global__ __launch_bounds__(NT) void k_fwdT(const Slot* __restrict__ slots, int iin, int iout, int iaux0,
                                             int iaux1, int A, int B, const cpx<R>* __restrict__ tw) {
    const Slot& S = slots[blockIdx.y];
    const SolveState* st = as_global(S.st);
    if (st->done) return;
    cpx<R>* inp = fld<R>(S, iin);
    cpx<R>* __restrict__ out = fld<R>(S, iout);
    // PRO_DIR: aux0 = P_C r (type R), aux1 = Phi (type RX)
    const cpx<R>* __restrict__ auxR = (PRO == PRO_DIR && iaux0 >= 0) ? fld<R>(S, iaux0) : nullptr;
    const cpx<RX>* __restrict__ aux1 = iaux1 >= 0 ? fld<RX>(S, iaux1) : nullptr;
    constexpr int PITCH = Lay<N>::P;
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

    // the prologue combinations are formed in double and rounded once
    int mode = second ? PRO_PLAIN : PRO;
    double k0 = 1, k1 = 0, k2 = 1;
    if (PRO == PRO_DIR) {
        k0 = st->beta;
        k1 = st->dphi;
        k2 = st->invnP;
    }
    // the thread's points in batches of EB: every load of a batch is issued
    // before its stores (a store to inp would otherwise hold back the loads of
    // the next point, which the compiler must assume it may alias)
    constexpr int EPT = TilePlan<R, N, TILE, NT>::EPT;
    constexpr int EB = EPT < 4 ? EPT : 4;
#pragma unroll
    for (int i0 = 0; i0 < EPT; i0 += EB) {
        cpx<R> vi[EB], va[EB];
        cpx<RX> vx[EB];
#pragma unroll
        for (int j = 0; j < EB; ++j) {
            if (i0 + j >= EPT) continue;   // EPT need not be a multiple of EB
            const int e = threadIdx.x + (i0 + j) * NT;
            if (TILE * N % NT != 0 && e >= TILE * N) continue;
            const int l = e / N, m = e - l * N;
            const long long gi = base + (long long)l * N + m;
            if (second) {
                vx[j] = aux1[gi];
            } else {
                vi[j] = inp[gi];
                if (mode == PRO_DIR) {
                    va[j] = auxR[gi];
                    vx[j] = aux1[gi];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < EB; ++j) {
            if (i0 + j >= EPT) continue;   // EPT need not be a multiple of EB
            const int e = threadIdx.x + (i0 + j) * NT;
            if (TILE * N % NT != 0 && e >= TILE * N) continue;
            const int l = e / N, m = e - l * N;
            cpx<R> v;
            if (second) {
                v = cvt<R>(vx[j]);
            } else {
                v = vi[j];
                if (mode == PRO_DIR) {
                    // D = -P r + beta P^{n-1};  P^n = D - Re<D,Phi> Phi  (stored), transform P^n / |P^n|
                    const cpx<double> d = k0 * wid(v) - wid(va[j]) - k1 * wid(vx[j]);
                    v = cvt<R>(d);
                    inp[base + (long long)l * N + m] = v;
                    v = (R)k2 * v;
                }
            }
            lds[l * PITCH + lx(m)] = v;
        }
    }
    __syncthreads();
    lds_fft<R, N, TILE, NT, false>(lds, tw);
    for (int e = threadIdx.x; e < TILE * N; e += NT) {
        const int l = e % TILE, m = e / TILE;
        out[(((long long)c * N + m) * A + a) * B + b0 + l] = lds[l * PITCH + lx(m)];
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
template <typename R, int N, int TILE, int EPI, int NT>
__global__ __launch_bounds__(NT) void k_invT(const Slot* __restrict__ slots, int iin, int iin2, int iout,
                                             int iout2, int iuin, int B, int Cc, double scale, int use_invnP,
                                             int rot_any, const cpx<R>* __restrict__ tw) {
    const Slot& S = slots[blockIdx.y];
    const SolveState* st = as_global(S.st);
    if (st->done) return;
    const Phys p = S.p;
    // the rotation input/output pair exists for rotating slots of the H_L chain
    const int nin = (EPI != EPI_SCALE && rot_any && p.omega != 0.0) ? 2 : 1;
    const cpx<R>* __restrict__ in = fld<R>(S, iin);
    const cpx<R>* __restrict__ in2 = nin == 2 ? fld<R>(S, iin2) : nullptr;
    cpx<R>* __restrict__ out = fld<R>(S, iout);
    cpx<R>* __restrict__ out2 = (nin == 2 && iout2 >= 0) ? fld<R>(S, iout2) : nullptr;
    const cpx<R>* __restrict__ uin = iuin >= 0 ? fld<R>(S, iuin) : nullptr;
    using TP = TilePlan<R, N, TILE, NT>;
    constexpr int PITCH = Lay<N>::P;
    constexpr int EPT = TP::EPT;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    cpx<R>* lds2 = lds + TILE * PITCH;
    const cpx<R>* twl = tw;
    if constexpr (TP::PIPE) {
        cpx<R>* t = reinterpret_cast<cpx<R>*>(smem_raw + TP::tw_offset(EPI == EPI_SCALE ? 1 : 2));
        tw_to_lds<R, N>(t, tw, TP::TW_BYTES, NT);
        twl = t;
    }
    const int tiles = Cc / TILE;
    const int units = 3 * B * tiles;
    const R uscale = (EPI == EPI_HL && use_invnP) ? (R)st->invnP : (R)1;
    cpx<R> pa[TP::PIPE ? EPT : 1], pb[TP::PIPE ? EPT : 1];
    int u = xcd_block(blockIdx.x, gridDim.x);
    int c, bb, c0;
    if constexpr (TP::PIPE) {
        if (u < units) {
            tile_unit(u, tiles, B, TILE, c, bb, c0);
            tile_fetch<R, N, TILE, NT>(in, in2, nin, (((long long)c * N) * B + bb) * Cc + c0, B, Cc, pa, pb);
        }
    }
    // a loop over units only when pipelined (otherwise one unit per block)
    if (u < units) do {
    tile_unit(u, tiles, B, TILE, c, bb, c0);
    if constexpr (TP::PIPE) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = threadIdx.x + i * NT;
            if (TILE * N % NT == 0 || e < TILE * N) {
                const int l = e % TILE, m = e / TILE;
                st2(lds + l * PITCH + lx(m), pa[i]);
                if (nin == 2) st2(lds2 + l * PITCH + lx(m), pb[i]);
            }
        }
    } else {
        for (int e = threadIdx.x; e < TILE * N; e += NT) {
            const int l = e % TILE, m = e / TILE;
            const long long gi = (((long long)c * N + m) * B + bb) * Cc + c0 + l;
            lds[l * PITCH + lx(m)] = in[gi];
            if (nin == 2) lds2[l * PITCH + lx(m)] = in2[gi];
        }
    }
    __syncthreads();
    if constexpr (TP::PIPE) {
        if (u + (int)gridDim.x < units) {
            int cn, bn, c0n;
            tile_unit(u + gridDim.x, tiles, B, TILE, cn, bn, c0n);
            tile_fetch<R, N, TILE, NT>(in, in2, nin, (((long long)cn * N) * B + bn) * Cc + c0n, B, Cc, pa, pb);
        }
    }
    lds_fft<R, N, TILE, NT, true>(lds, twl);
    if (nin == 2) lds_fft<R, N, TILE, NT, true>(lds2, twl);
    // in batches of EB points, the loads of uin (and of a tabulated potential)
    // issued before the batch's stores (see the forward pass)
    constexpr int EB = EPT < 4 ? EPT : 4;
#pragma unroll
    for (int i0 = 0; i0 < EPT; i0 += EB) {
        cpx<R> vu[EB];
        double vV[EB];
#pragma unroll
        for (int j = 0; j < EB; ++j) {
            if (i0 + j >= EPT) continue;   // EPT need not be a multiple of EB
            const int e = threadIdx.x + (i0 + j) * NT;
            if (TILE * N % NT != 0 && e >= TILE * N) continue;
            const int l = e / N, m = e - l * N;
            const long long go = (((long long)c * B + bb) * Cc + c0 + l) * N + m;
            if (EPI == EPI_HL) {
                vu[j] = uin[go];
                const double x = -p.L[0] + m * p.h[0];
                const double y = -p.L[1] + (c0 + l) * p.h[1];
                const double z = p.dim == 3 ? -p.L[2] + bb * p.h[2] : 0.0;
                double V2, V4;
                trap_at(p, go - (long long)c * p.M, x, y, z, V2, V4);
                vV[j] = V2 + V4;
            } else if (EPI == EPI_ROTX && nin == 2) {
                vu[j] = uin[go];
            }
        }
#pragma unroll
        for (int j = 0; j < EB; ++j) {
            if (i0 + j >= EPT) continue;   // EPT need not be a multiple of EB
            const int e = threadIdx.x + (i0 + j) * NT;
            if (TILE * N % NT != 0 && e >= TILE * N) continue;
            const int l = e / N, m = e - l * N;
            const long long go = (((long long)c * B + bb) * Cc + c0 + l) * N + m;
            cpx<R> v = lds[l * PITCH + lx(m)];
            if (EPI == EPI_SCALE) {
                out[go] = (R)scale * v;
            } else if (EPI == EPI_HL) {
                const double x = -p.L[0] + m * p.h[0];
                v = v + (R)vV[j] * (uscale * vu[j]);
                if (nin == 2) v = v - (R)(p.omega * x) * lds2[l * PITCH + lx(m)];
                out[go] = v;
            } else if (EPI == EPI_ROTX) {
                if (nin == 2) {
                    const double kx = wavenum_odd(bb, p.n[0], p.L[0], p.nyq_zero);
                    const double y = -p.L[1] + m * p.h[1];
                    v = v + (R)(p.omega * y * kx / p.n[0]) * vu[j];
                    out2[go] = lds2[l * PITCH + lx(m)];
                }
                out[go] = v;
            }
        }
    }
    if constexpr (TP::PIPE) __syncthreads();   // lds and lds2 are refilled by the next unit
    } while (TP::PIPE && (u += gridDim.x) < units);
}

// ---------------------------------------------------------------------------
// last pass of the preconditioner: P r = P_V^{1/2} (inverse transform), with the
// partial sums of the direction reductions of the next step fused in
// (Re<r,Pr>, Re<r_prev,Pr>, Re<phi,Pr>, |Pr|^2, Re<Pr,P^{n-1}>).
// ---------------------------------------------------------------------------
template <typename R, typename RS, int N, int TILE, int NT>
__global__ __launch_bounds__(NT) void k_invT_pre(const Slot* __restrict__ slots, int iin, int iout, int B,
                                                 int Cc, int dir, const cpx<R>* __restrict__ tw) {
    const Slot& S = slots[blockIdx.y];
    SolveState* st = as_global(S.st);
    if (st->done) return;
    const cpx<R>* __restrict__ in = fld<R>(S, iin);
    cpx<R>* __restrict__ out = fld<R>(S, iout);
    const R* __restrict__ pv = pvf<R>(S);
    using TP = TilePlan<R, N, TILE, NT>;
    constexpr int PITCH = Lay<N>::P;
    constexpr int EPT = TP::EPT;
    static_assert(NT % 64 == 0, "whole waves");
    constexpr int NQ = (TILE * N + 63) / 64;   // chunks of 64 points per unit
    __shared__ double chs[NQ][ChunkSums<NS_DIR>::P];
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    const cpx<R>* twl = tw;
    if constexpr (TP::PIPE) {
        cpx<R>* t = reinterpret_cast<cpx<R>*>(smem_raw + TP::tw_offset(1));
        tw_to_lds<R, N>(t, tw, TP::TW_BYTES, NT);
        twl = t;
    }
    const cpx<R>* r = dir ? fld<R>(S, B_R0 + st->cur) : nullptr;
    const cpx<R>* rp = dir ? fld<R>(S, B_R0 + (st->cur ^ 1)) : nullptr;
    const cpx<RS>* phi = fld<RS>(S, B_PHI);
    const cpx<R>* Pprev = fld<R>(S, B_P);
    const int tiles = Cc / TILE;
    const int units = 3 * B * tiles;
    cpx<R> pa[TP::PIPE ? EPT : 1], pb[TP::PIPE ? EPT : 1];
    int u = xcd_block(blockIdx.x, gridDim.x);
    int c, bb, c0;
    if constexpr (TP::PIPE) {
        if (u < units) {
            tile_unit(u, tiles, B, TILE, c, bb, c0);
            tile_fetch<R, N, TILE, NT>(in, nullptr, 1, (((long long)c * N) * B + bb) * Cc + c0, B, Cc, pa, pb);
        }
    }
    // a loop over units only when pipelined (otherwise one unit per block)
    if (u < units) do {
    tile_unit(u, tiles, B, TILE, c, bb, c0);
    if constexpr (TP::PIPE) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = threadIdx.x + i * NT;
            if (TILE * N % NT == 0 || e < TILE * N) {
                const int l = e % TILE, m = e / TILE;
                st2(lds + l * PITCH + lx(m), pa[i]);
            }
        }
    } else {
        for (int e = threadIdx.x; e < TILE * N; e += NT) {
            const int l = e % TILE, m = e / TILE;
            lds[l * PITCH + lx(m)] = in[(((long long)c * N + m) * B + bb) * Cc + c0 + l];
        }
    }
    __syncthreads();
    if constexpr (TP::PIPE) {
        if (u + (int)gridDim.x < units) {
            int cn, bn, c0n;
            tile_unit(u + gridDim.x, tiles, B, TILE, cn, bn, c0n);
            tile_fetch<R, N, TILE, NT>(in, nullptr, 1, (((long long)cn * N) * B + bn) * Cc + c0n, B, Cc, pa, pb);
        }
    }
    lds_fft<R, N, TILE, NT, true>(lds, twl);
    // one loop over the points in wave-uniform chunks of 64 (batching its loads
    // as the other passes do raised the register count and lost occupancy:
    // measured slower); the partial sums of a chunk are reduced by its wave,
    // so the unit's row does not depend on NT
    // (two points per lane before the wave's tree, as in the middle pass, was
    // measured slower here: 103 -> 110 us for the float pass at 32 slots of 256^2)
    for (int base = threadIdx.x & ~63; base < TILE * N; base += NT) {
        const int e = base + (threadIdx.x & 63);
        double acc[NS_DIR] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (e < TILE * N) {
            const int l = e / N, m = e - l * N;
            const long long go = (((long long)c * B + bb) * Cc + c0 + l) * N + m;
            const cpx<R> v = pv[go] * lds[l * PITCH + lx(m)];
            out[go] = v;
            if (dir) {
                const cpx<double> w = wid(v);
                acc[0] = re_dot(wid(r[go]), w);
                acc[1] = re_dot(wid(rp[go]), w);
                acc[2] = re_dot(wid(phi[go]), w);
                acc[3] = cabs2(w);
                acc[4] = re_dot(wid(Pprev[go]), w);
            }
        }
        if (dir) chunk_add<NS_DIR>(acc, chs, base >> 6);
    }
    // one partial-sum row per unit, whichever block took it
    if (dir) {
        __syncthreads();
        chunk_row<NS_DIR>(chs, NQ, as_global(S.red_dir), RED_DIR_STRIDE, u);
    }
    if constexpr (TP::PIPE) __syncthreads();   // lds and the chunk sums are refilled by the next unit
    } while (TP::PIPE && (u += gridDim.x) < units);
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
// Symbols at the wavenumber of middle-pass line `line` (the flattened
// positions of the axes transformed before) and position m on the middle
// axis: the kinetic symbol 1/2 |k|^2 from the wavenumbers, and k_x, k_y of
// the odd operators (SOC, rotation) in their odd-operator reading.
struct SpecK {
    double K, kx, ky;
};
__device__ __forceinline__ SpecK spec_k(const Phys& p, int line, int m) {
    int jx, jy, jz;
    if (p.dim == 2) {
        jx = line; jy = m; jz = 0;
    } else {
        jx = line % p.n[0]; jy = line / p.n[0]; jz = m;
    }
    const double wx = wavenum(jx, p.n[0], p.L[0]), wy = wavenum(jy, p.n[1], p.L[1]);
    const double wz = p.dim == 3 ? wavenum(jz, p.n[2], p.L[2]) : 0.0;
    return SpecK{0.5 * (wx * wx + wy * wy + wz * wz), wavenum_odd(jx, p.n[0], p.L[0], p.nyq_zero),
                 wavenum_odd(jy, p.n[1], p.L[1], p.nyq_zero)};
}
// 1/x for a positive, finite, normal x: the hardware estimate refined by two
// Newton steps r <- r + r (1 - x r), each of which squares the relative
// error (to below 1 ulp, from the estimate's ~2^-26)
__device__ __forceinline__ double recip_pos(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// H_L's spectral part at one wavenumber for the three components v (the
// spectra, unnormalised): a = (1/2 |k|^2 v - gamma S(k) v) / M with
// S(k) = [[0, s0, 0], [s1, 0, s0], [0, s1, 0]], s0 = -k_x + i k_y (L0),
// s1 = -k_x - i k_y (L1); the point's partial sums: 1/2 |k|^2 |v_l|^2 and
// Re v^dag S v, or with the spectrum z of Phi (X2) 1/2 |k|^2 |z_l|^2,
// 1/2 |k|^2 Re z_l conj(v_l) and 1/2 |k|^2 |v_l|^2.
template <bool X2>
__device__ __forceinline__ void hl_point(const SpecK& k, double gamma, double invM, const cpx<double> (&v)[3],
                                         const cpx<double> (&z)[3], cpx<double> (&a)[3], double (&acc)[X2 ? 9 : 4]) {
    const cpx<double> s0 = cmk(-k.kx, k.ky), s1 = cmk(-k.kx, -k.ky);
    const cpx<double> S0 = cmul(s0, v[1]);
    const cpx<double> S1 = cmul(s1, v[0]) + cmul(s0, v[2]);
    const cpx<double> S2 = cmul(s1, v[1]);
    if constexpr (X2) {
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            acc[3 * cc] = k.K * cabs2(z[cc]);
            acc[3 * cc + 1] = k.K * re_dot(z[cc], v[cc]);
            acc[3 * cc + 2] = k.K * cabs2(v[cc]);
        }
    } else {
        acc[0] = k.K * cabs2(v[0]);
        acc[1] = k.K * cabs2(v[1]);
        acc[2] = k.K * cabs2(v[2]);
        acc[3] = cmulc(S0, v[0]).x + cmulc(S1, v[1]).x + cmulc(S2, v[2]).x;
    }
    a[0] = invM * (k.K * v[0] - gamma * S0);
    a[1] = invM * (k.K * v[1] - gamma * S1);
    a[2] = invM * (k.K * v[2] - gamma * S2);
}

// The spectral operator of a middle pass at point e of a line group (line
// l0 + e / N, position e mod N of the middle axis), on the group's spectra in
// LDS: X (three components, line c LPB + q at X + (c LPB + q) PITCH), for
// MID_HLX Z (Phi's spectrum, same layout), for a rotating slot the output Y
// (the k_y part, same layout; Y may take Z's place: the point's Z values are
// read before its Y values are written). acc: the point's partial sums.
template <typename R, int N, int LPB, int OP>
__device__ __forceinline__ void mid_point(const Phys& p, int l0, int e, cpx<R>* X, const cpx<R>* Z, cpx<R>* Y,
                                          bool doB, double invM, bool unit, const double (&al)[3], double fl,
                                          double (&acc)[OP == MID_HLX ? NS_KIN : 4]) {
    constexpr int PITCH = Lay<N>::P;
    constexpr bool HL = OP == MID_HL || OP == MID_HLX;
    constexpr bool X2 = OP == MID_HLX;
    const int q = e / N, m = e - q * N;
    const SpecK sk = spec_k(p, l0 + q, m);
    cpx<R>* x0 = X + (0 * LPB + q) * PITCH + lx(m);
    cpx<R>* x1 = X + (1 * LPB + q) * PITCH + lx(m);
    cpx<R>* x2 = X + (2 * LPB + q) * PITCH + lx(m);
    if constexpr (HL) {
        const cpx<double> v[3] = {wid(*x0), wid(*x1), wid(*x2)};
        cpx<double> z[3] = {};
        if constexpr (X2)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) z[cc] = wid(Z[(cc * LPB + q) * PITCH + lx(m)]);
        cpx<double> a[3];
        hl_point<X2>(sk, p.gamma, invM, v, z, a, acc);
        if (doB) {
            const double fb = sk.ky * invM;
            Y[(0 * LPB + q) * PITCH + lx(m)] = cmk((R)(fb * v[0].x), (R)(fb * v[0].y));
            Y[(1 * LPB + q) * PITCH + lx(m)] = cmk((R)(fb * v[1].x), (R)(fb * v[1].y));
            Y[(2 * LPB + q) * PITCH + lx(m)] = cmk((R)(fb * v[2].x), (R)(fb * v[2].y));
        }
        *x0 = cmk((R)a[0].x, (R)a[0].y);
        *x1 = cmk((R)a[1].x, (R)a[1].y);
        *x2 = cmk((R)a[2].x, (R)a[2].y);
    } else {
        const R d0 = (R)(unit ? invM : invM * recip_pos(fmax(al[0] + sk.K, fl)));
        const R d1 = (R)(unit ? invM : invM * recip_pos(fmax(al[1] + sk.K, fl)));
        const R d2 = (R)(unit ? invM : invM * recip_pos(fmax(al[2] + sk.K, fl)));
        *x0 = d0 * *x0;
        *x1 = d1 * *x1;
        *x2 = d2 * *x2;
    }
}

// Values per thread of a middle pass over NLN lines, and whether the block
// pipelines its line groups: the next group's input is loaded into registers
// while the current one is transformed (when that takes at most 6 values).
template <typename R, int N, int LPB, int OP, int NT> struct MidPlan {
    static constexpr int NLN = 3 * LPB;
    static constexpr int EPT = (NLN * N + NT - 1) / NT;
    static constexpr bool PIPE = EPT * (OP == MID_HLX ? 2 : 1) <= 6;
    // LDS copy of the input for the 2D rotation term when three line groups fit in 64 KB
    static constexpr bool CLDS = 3 * NLN * Lay<N>::P * (int)sizeof(cpx<R>) <= 65536;
    // line buffers of the block (X; Z or Y; the input copy) and the byte offset
    // of the block's copy of the twiddle table after them
    __host__ __device__ static constexpr int nbuf(bool rot_any) {
        return OP == MID_PRE ? 1 : (rot_any ? 2 + (CLDS ? 1 : 0) : (OP == MID_HLX ? 2 : 1));
    }
    __host__ __device__ static constexpr size_t tw_offset(bool rot_any) {
        return ((size_t)nbuf(rot_any) * NLN * Lay<N>::P * sizeof(cpx<R>) + 15) & ~(size_t)15;
    }
    // the table of exp(-2 pi i m / N), and for float the double table after it;
    // copied into LDS by a pipelined block, which reuses it for many groups
    static constexpr size_t TW_BYTES =
        PIPE ? (size_t)N * sizeof(cpx<R>) + (sizeof(R) == 4 ? (size_t)N * 16 : 0) : 0;
};

template <typename R, int N, int LPB, int OP, int NT>
__device__ __forceinline__ void mid_fetch(const cpx<R>* __restrict__ in, const cpx<R>* __restrict__ in2,
                                          long long cs, int l0, cpx<R> (&a)[MidPlan<R, N, LPB, OP, NT>::EPT],
                                          cpx<R> (&b)[MidPlan<R, N, LPB, OP, NT>::EPT]) {
    using MP = MidPlan<R, N, LPB, OP, NT>;
#pragma unroll
    for (int i = 0; i < MP::EPT; ++i) {
        const int e = threadIdx.x + i * NT;
        if (MP::NLN * N % NT == 0 || e < MP::NLN * N) {
            const int L = e / N, m = e - L * N;
            const int c = L / LPB, q = L - c * LPB;
            const long long gi = c * cs + (long long)(l0 + q) * N + m;
            ld2(a[i], in + gi);
            if (OP == MID_HLX) ld2(b[i], in2 + gi);
        }
    }
}

// Middle pass: FFT along the contiguous axis of NLN = 3 LPB lines (the three
// components of LPB line positions), the spectral operator, inverse FFT.
// Block b of a slot takes line groups b, b + gridDim.x, ...; every group
// writes its own partial-sum row, so the sums do not depend on the grid.
template <typename R, int N, int LPB, int OP, int NT>
__global__ __launch_bounds__(NT) void k_mid(const Slot* __restrict__ slots, int iin, int ioutA, int ioutB,
                                            int nlines, int rot_any, const cpx<R>* __restrict__ tw) {
    using MP = MidPlan<R, N, LPB, OP, NT>;
    const Slot& S = slots[blockIdx.y];
    const SolveState* st = as_global(S.st);
    if (st->done) return;
    const Phys p = S.p;
    const int rot = rot_any && p.omega != 0.0;
    const cpx<R>* __restrict__ in = fld<R>(S, iin);
    const cpx<R>* __restrict__ in2 = (OP == MID_HLX) ? in + 3 * p.M : nullptr;
    cpx<R>* __restrict__ outA = fld<R>(S, ioutA);
    cpx<R>* __restrict__ outB = ioutB >= 0 ? fld<R>(S, ioutB) : nullptr;
    double* __restrict__ red = as_global(S.red_mid);
    constexpr int PITCH = Lay<N>::P;
    constexpr int NLN = MP::NLN;
    constexpr int EPT = MP::EPT;
    constexpr bool HL = OP == MID_HL || OP == MID_HLX;
    constexpr bool X2 = OP == MID_HLX;
    constexpr int NVM = X2 ? NS_KIN : 4;   // partial sums per line group
    static_assert(NT % 64 == 0, "whole waves");
    // the group's points in chunks of 64 KP points: lane l of the wave that takes a
    // chunk adds the sums of points l, l + 64, ..., l + 64 (KP - 1) of it in that
    // order before the wave's halving tree, which then runs once per KP points
    // (at 32 slots of 256^2, KP = 2 took hl_mid from 63 to 60 us in float; four
    // points per lane, one chunk and one busy wave per group, 69 us)
    constexpr int KP = LPB * N >= 512 ? 4 : (LPB * N >= 256 ? 2 : 1);
    constexpr int NQ = (LPB * N + 64 * KP - 1) / (64 * KP);
    __shared__ double chs[HL ? NQ : 1][ChunkSums<NVM>::P];
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cpx<R>* X = reinterpret_cast<cpx<R>*>(smem_raw);
    cpx<R>* Z = X + NLN * PITCH;                       // spectrum of Phi (MID_HLX)
    // rotation output B; with MID_HLX it takes Z's place (each point's Z values
    // are read by the thread that then writes its B values)
    cpx<R>* Y = X + NLN * PITCH;
    cpx<R>* Cp = X + 2 * NLN * PITCH;                  // input copy for the 2D rotation term
    // a pipelined block copies the twiddle tables once into LDS: every transform
    // stage of every line group then reads them there instead of from global
    // memory (visible after the first barrier of the group loop)
    const cpx<R>* twl = tw;
    if constexpr (MP::PIPE) {
        cpx<R>* t = reinterpret_cast<cpx<R>*>(smem_raw + MP::tw_offset(rot_any != 0));
        for (int e = threadIdx.x; e < (int)(MP::TW_BYTES / 16); e += NT)
            reinterpret_cast<vec2<double>*>(t)[e] = reinterpret_cast<const vec2<double>*>(tw)[e];
        twl = t;
    }
    const bool doB = HL && rot;
    const bool rot2d = doB && p.dim == 2;
    const long long cs = (long long)nlines * N;
    const int ngroups = nlines / LPB;
    // transforms of two line groups at once when a thread then holds at most
    // 8 (double) or 16 (float) values
    constexpr bool JOINT = 2 * NLN * N <= (sizeof(R) == 8 ? 8 : 16) * NT;
    cpx<R> pa[EPT], pb[EPT];
    int grp = blockIdx.x;
    if (MP::PIPE && grp < ngroups) mid_fetch<R, N, LPB, OP, NT>(in, in2, cs, grp * LPB, pa, pb);
    const double invM = 1.0 / (double)p.M;
    double al[3] = {0.0, 0.0, 0.0}, fl = 0.0;
    // the potential preconditioner (3.14) has no kinetic factor: unit multiplier
    const bool unit = OP == MID_PRE && st->precond == GS_PC_POTENTIAL;
    if (OP == MID_PRE) {
        al[0] = st->alpha[0]; al[1] = st->alpha[1]; al[2] = st->alpha[2];
        fl = 1e-12 * fmax(1.0, fmax(al[0], fmax(al[1], al[2])));
    }
    for (; grp < ngroups; grp += gridDim.x) {
        const int l0 = grp * LPB;
        if (!MP::PIPE) mid_fetch<R, N, LPB, OP, NT>(in, in2, cs, l0, pa, pb);
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = threadIdx.x + i * NT;
            if (NLN * N % NT == 0 || e < NLN * N) {
                const int L = e / N, m = e - L * N;
                st2(X + L * PITCH + lx(m), pa[i]);
                if (X2) st2(Z + L * PITCH + lx(m), pb[i]);
                if (MP::CLDS && rot2d) st2(Cp + L * PITCH + lx(m), pa[i]);
            }
        }
        __syncthreads();
        if (MP::PIPE && grp + (int)gridDim.x < ngroups)
            mid_fetch<R, N, LPB, OP, NT>(in, in2, cs, (grp + gridDim.x) * LPB, pa, pb);
        if constexpr (X2 && JOINT) {
            lds_fft<R, N, 2 * NLN, NT, false>(X, twl);   // X and Z are adjacent
        } else {
            lds_fft<R, N, NLN, NT, false>(X, twl);
            if constexpr (X2) lds_fft<R, N, NLN, NT, false>(Z, twl);
        }
        // the partial sums per chunk (one wave's iteration; the lanes past the
        // group's last point add zeros), so the row does not depend on NT
        for (int base = (threadIdx.x & ~63) * KP; base < LPB * N; base += NT * KP) {
            double acc[NVM];
#pragma unroll
            for (int k = 0; k < NVM; ++k) acc[k] = 0.0;
#pragma unroll
            for (int j = 0; j < KP; ++j) {
                const int e = base + 64 * j + (threadIdx.x & 63);
                if (e < LPB * N) {
                    double a1[NVM];
                    mid_point<R, N, LPB, OP>(p, l0, e, X, Z, Y, doB, invM, unit, al, fl, a1);
                    if constexpr (HL)
#pragma unroll
                        for (int k = 0; k < NVM; ++k) acc[k] += a1[k];
                }
            }
            if (HL) chunk_add<NVM>(acc, chs, base / (64 * KP));   // the whole wave
        }
        __syncthreads();
        if constexpr (HL && JOINT) {
            if (doB) lds_fft<R, N, 2 * NLN, NT, true>(X, twl);   // X and Y are adjacent
            else lds_fft<R, N, NLN, NT, true>(X, twl);
        } else {
            lds_fft<R, N, NLN, NT, true>(X, twl);
            if (doB) lds_fft<R, N, NLN, NT, true>(Y, twl);
        }
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = threadIdx.x + i * NT;
            if (NLN * N % NT == 0 || e < NLN * N) {
                const int L = e / N, m = e - L * N;
                const int c = L / LPB, q = L - c * LPB;
                const long long go = c * cs + (long long)(l0 + q) * N + m;
                cpx<R> v = X[L * PITCH + lx(m)];
                if (rot2d) {
                    const double kx = wavenum_odd(l0 + q, p.n[0], p.L[0], p.nyq_zero);
                    const double y = -p.L[1] + m * p.h[1];
                    const cpx<R> x = MP::CLDS ? Cp[L * PITCH + lx(m)] : in[go];
                    v = v + (R)(p.omega * y * kx / p.n[0]) * x;
                }
                outA[go] = v;
                if (doB) outB[go] = Y[L * PITCH + lx(m)];
            }
        }
        if (HL) chunk_row<NVM>(chs, NQ, red, RED_MID_STRIDE, grp);
        __syncthreads();   // X, Z, Y, the copy and the chunk sums are refilled by the next group
    }
}

// ---------------------------------------------------------------------------
// middle pass for lines longer than 1024 (2D, the y axis): the three
// component lines of one position no longer fit in LDS together, so the pass
// runs as three kernels: the forward transforms line by line (k_lfft), the
// spectral operator on the whole spectrum with every component of a
// wavenumber at hand (k_lspec, with the partial sums of the kinetic
// coefficients in rows of a fixed pointwise grid), and the inverse
// transforms line by line, which add the rotation term.
// ---------------------------------------------------------------------------
// One line of N contiguous values per block: forward (unscaled) or inverse
// transform of the [ncomp][nlines][N] field iin into iout (in place when they
// are equal: a block reads its whole line before it writes), blocks
// [0, ncomp nlines) of a slot; with iin2 >= 0 the next 3 nlines blocks
// transform the three components of iin2 into iout2, for rotating slots
// only. With irot >= 0 (the inverse of the H_L output of a rotating slot) the
// 2D rotation term is added to iout: Omega y k_x C / Nx, C the x-transformed
// input of the chain at irot.
template <typename R, int N, bool INV, int NT>
__global__ __launch_bounds__(NT) void k_lfft(const Slot* __restrict__ slots, int iin, int iout, int ncomp,
                                             int nlines, int irot, int iin2, int iout2,
                                             const cpx<R>* __restrict__ tw) {
    const Slot& S = slots[blockIdx.y];
    const SolveState* st = as_global(S.st);
    if (st->done) return;
    const Phys p = S.p;
    const bool second = (int)blockIdx.x >= ncomp * nlines;
    if (second && p.omega == 0.0) return;
    const int b = second ? (int)blockIdx.x - ncomp * nlines : (int)blockIdx.x;
    const int c = b / nlines, l = b - c * nlines;
    const long long off = (long long)c * nlines * N + (long long)l * N;
    const cpx<R>* in = fld<R>(S, second ? iin2 : iin) + off;
    cpx<R>* out = fld<R>(S, second ? iout2 : iout) + off;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cpx<R>* lds = reinterpret_cast<cpx<R>*>(smem_raw);
    for (int m = threadIdx.x; m < N; m += NT) {
        cpx<R> v;
        ld2(v, in + m);
        lds[lx(m)] = v;
    }
    __syncthreads();
    lds_fft<R, N, 1, NT, INV>(lds, tw);
    const bool rot = !second && irot >= 0 && p.omega != 0.0;
    const cpx<R>* __restrict__ C = rot ? fld<R>(S, irot) + off : nullptr;
    const double kx = rot ? wavenum_odd(l, p.n[0], p.L[0], p.nyq_zero) : 0.0;
    for (int m = threadIdx.x; m < N; m += NT) {
        cpx<R> v = lds[lx(m)];
        if (rot) {
            const double y = -p.L[1] + m * p.h[1];
            v = v + (R)(p.omega * y * kx / p.n[0]) * C[m];
        }
        st2(out + m, v);
    }
}

// Spectral operator of the middle pass on the whole spectrum in[c][line][m]
// (components 3..5: the spectrum of Phi, for MID_HLX), one point per thread
// in a grid-stride loop over the M points; outputs as in k_mid. The partial
// sums of a block form row blockIdx.x of red_mid (gridDim.x rows, a function
// of M only).
template <typename R, int OP>
__global__ __launch_bounds__(PT) void k_lspec(const Slot* __restrict__ slots, int iin, int ioutA, int ioutB,
                                              int N, int rot_any) {
    const Slot& S = slots[blockIdx.y];
    const SolveState* st = as_global(S.st);
    if (st->done) return;
    const Phys p = S.p;
    const long long M = p.M;
    constexpr bool HL = OP == MID_HL || OP == MID_HLX;
    constexpr bool X2 = OP == MID_HLX;
    constexpr int NVM = X2 ? NS_KIN : 4;
    const cpx<R>* __restrict__ in = fld<R>(S, iin);
    cpx<R>* __restrict__ outA = fld<R>(S, ioutA);
    const bool doB = HL && rot_any && p.omega != 0.0;
    cpx<R>* __restrict__ outB = doB ? fld<R>(S, ioutB) : nullptr;
    const double invM = 1.0 / (double)M;
    double al[3] = {0.0, 0.0, 0.0}, fl = 0.0;
    const bool unit = OP == MID_PRE && st->precond == GS_PC_POTENTIAL;
    if (OP == MID_PRE) {
        al[0] = st->alpha[0]; al[1] = st->alpha[1]; al[2] = st->alpha[2];
        fl = 1e-12 * fmax(1.0, fmax(al[0], fmax(al[1], al[2])));
    }
    double tot[NVM];
#pragma unroll
    for (int k = 0; k < NVM; ++k) tot[k] = 0.0;
    for (long long i = (long long)blockIdx.x * PT + threadIdx.x; i < M; i += (long long)gridDim.x * PT) {
        const int line = (int)(i / N), m = (int)(i - (long long)line * N);
        const SpecK sk = spec_k(p, line, m);
        if (HL) {
            const cpx<double> v[3] = {wid(in[i]), wid(in[M + i]), wid(in[2 * M + i])};
            cpx<double> z[3] = {};
            if (X2) {
                z[0] = wid(in[3 * M + i]);
                z[1] = wid(in[4 * M + i]);
                z[2] = wid(in[5 * M + i]);
            }
            cpx<double> a[3];
            double acc[NVM];
            hl_point<X2>(sk, p.gamma, invM, v, z, a, acc);
#pragma unroll
            for (int k = 0; k < NVM; ++k) tot[k] += acc[k];
#pragma unroll
            for (int c = 0; c < 3; ++c) outA[c * M + i] = cmk((R)a[c].x, (R)a[c].y);
            if (doB) {
                const double fb = sk.ky * invM;
#pragma unroll
                for (int c = 0; c < 3; ++c) outB[c * M + i] = cmk((R)(fb * v[c].x), (R)(fb * v[c].y));
            }
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const R d = (R)(unit ? invM : invM * recip_pos(fmax(al[c] + sk.K, fl)));
                outA[c * M + i] = d * in[c * M + i];
            }
        }
    }
    if (HL) block_row<NVM>(tot, as_global(S.red_mid), RED_MID_STRIDE);
}

}  // namespace gs
