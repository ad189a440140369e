// Device helpers shared by the kernel translation units: deterministic block
// reductions into per-block rows, the fixed-order gather of those rows, grid
// coordinates, and the pointwise spin-1 algebra of the Hamiltonian (Sec. 1 of
// the paper).
#pragma once
#include "gs_internal.h"

namespace gs {

constexpr int PT = 256;   // threads per block of every kernel

// block maximum; thread 0 ends with it
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

template <int N> struct Pow2Ceil { static constexpr int v = 2 * Pow2Ceil<(N + 1) / 2>::v; };
template <> struct Pow2Ceil<1> { static constexpr int v = 1; };
template <int N> struct ILog2 { static constexpr int v = 1 + ILog2<N / 2>::v; };
template <> struct ILog2<1> { static constexpr int v = 0; };

// One reduce-scatter step across lanes `O` apart: each lane keeps the half of
// its H*2 partials selected by its lane bit O and adds the partner's copy of
// that half.
template <int H, int O>
__device__ __forceinline__ void halve_step(double* v, int lane) {
    const bool b = (lane & O) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const double keep = b ? v[H + i] : v[i];
        const double send = b ? v[i] : v[H + i];
        v[i] = keep + __shfl_xor(send, O, 64);
    }
}
template <int P, int O>
__device__ __forceinline__ void halve_all(double* v, int lane) {
    if constexpr (P > 1) {
        halve_step<P / 2, O>(v, lane);
        halve_all<P / 2, O / 2>(v, lane);
    } else if constexpr (O >= 1) {
        v[0] += __shfl_xor(v[0], O, 64);
        halve_all<1, O / 2>(v, lane);
    }
}

// Block sums of NV doubles written as this block's row: a recursive-halving
// reduce-scatter inside each wave (about P shuffles for P = NV rounded up to a
// power of two, instead of 6 NV), the four wave totals of each value added in
// a fixed order, and the row stored by NV threads at once.
template <int NV, int NTB = PT>
__device__ __forceinline__ void block_row(const double (&acc)[NV], double* rows, int stride, int row) {
    constexpr int P = Pow2Ceil<NV>::v;
    static_assert(P <= 64, "at most 64 sums per row");
    static_assert(NTB % 64 == 0 && NTB <= 1024, "whole waves");
    constexpr int SH = 6 - ILog2<P>::v;   // lanes 2^SH apart hold the same value index
    __shared__ double sh[NTB / 64][P];
    double v[P];
#pragma unroll
    for (int k = 0; k < P; ++k) v[k] = k < NV ? acc[k] : 0.0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    halve_all<P, 32>(v, lane);
    if ((lane & ((1 << SH) - 1)) == 0) sh[wv][lane >> SH] = v[0];
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = sh[0][threadIdx.x];
        for (int w = 1; w < NTB / 64; ++w) t += sh[w][threadIdx.x];
        rows[(long long)row * stride + threadIdx.x] = t;
    }
}
template <int NV, int NTB = PT>
__device__ __forceinline__ void block_row(const double (&acc)[NV], double* rows, int stride) {
    block_row<NV, NTB>(acc, rows, stride, (int)blockIdx.x);
}

// Sums over the points of a work unit whose order does not depend on the
// number of threads: the unit's points are visited as e = threadIdx.x + i NT
// (NT a multiple of 64, the point count a multiple of 64), so every chunk of
// 64 consecutive points is one wave's iteration. chunk_add reduces the wave's
// per-point values of one chunk by the fixed halving tree and keeps the
// chunk's totals in LDS (chunk q at ch[q]); chunk_row adds the chunks of the
// unit in chunk order and stores the unit's row. A launch configuration can
// then change the thread count without changing a bit of the sums.
template <int NV> struct ChunkSums {
    static constexpr int P = Pow2Ceil<NV>::v;
    static constexpr int SH = 6 - ILog2<P>::v;
};
template <int NV>
__device__ __forceinline__ void chunk_add(const double (&val)[NV], double (*ch)[ChunkSums<NV>::P], int q) {
    constexpr int P = ChunkSums<NV>::P, SH = ChunkSums<NV>::SH;
    double v[P];
#pragma unroll
    for (int k = 0; k < P; ++k) v[k] = k < NV ? val[k] : 0.0;
    const int lane = threadIdx.x & 63;
    halve_all<P, 32>(v, lane);
    if ((lane & ((1 << SH) - 1)) == 0) ch[q][lane >> SH] = v[0];
}
// after a barrier that follows the unit's last chunk_add
template <int NV>
__device__ __forceinline__ void chunk_row(double (*ch)[ChunkSums<NV>::P], int nq, double* rows, int stride, int row) {
    if (threadIdx.x < NV) {
        double t = ch[0][threadIdx.x];
        for (int q = 1; q < nq; ++q) t += ch[q][threadIdx.x];
        rows[(long long)row * stride + threadIdx.x] = t;
    }
}

// Totals over nrows rows (fixed order) of NV values at the given stride, on
// thread 0 of a block of PT threads. Entries k < 32 with (maxmask >> k) & 1 are
// maxima (of non-negative values).
template <int NV>
__device__ __forceinline__ void gather(double (&tot)[NV], const double* rows, int nrows, int stride,
                                       unsigned maxmask = 0u) {
    // each thread adds its rows (all NV loads of a row in flight at once), then
    // the sums are reduce-scattered inside each wave (recursive halving) and
    // thread k adds the four wave partials of value k; maxima by block max
    constexpr int P = Pow2Ceil<NV>::v;
    static_assert(P <= 64, "at most 64 values per row");
    constexpr int SH = 6 - ILog2<P>::v;   // lanes 2^SH apart hold the same value index
    __shared__ double sh[PT / 64][P];
    __shared__ double st[NV];
    double v[P];
#pragma unroll
    for (int k = 0; k < P; ++k) v[k] = 0.0;
    for (int b = threadIdx.x; b < nrows; b += PT)
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const double x = rows[(long long)b * stride + k];
            v[k] = (k < 32 && ((maxmask >> k) & 1u)) ? fmax(v[k], x) : v[k] + x;
        }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double m[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const bool mx = k < 32 && ((maxmask >> k) & 1u);
        m[k] = mx ? bmax(v[k]) : 0.0;   // maxmask is uniform: the block max is taken by all threads
        if (mx) v[k] = 0.0;
    }
    halve_all<P, 32>(v, lane);
    if ((lane & ((1 << SH) - 1)) == 0) sh[wv][lane >> SH] = v[0];
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = sh[0][threadIdx.x];
        for (int w = 1; w < PT / 64; ++w) t += sh[w][threadIdx.x];
        st[threadIdx.x] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) tot[k] = (k < 32 && ((maxmask >> k) & 1u)) ? m[k] : st[k];
    __syncthreads();   // sh and st are reused by the next gather of this size
}

// grid coordinates x_m = -L + m h of point index i ([Nz][Ny][Nx], x fastest)
__device__ __forceinline__ void coords(const Phys& p, long long i, double& x, double& y, double& z) {
    const unsigned nx = (unsigned)p.n[0], ny = (unsigned)p.n[1];
    const unsigned ii = (unsigned)i;   // M < 2^32 for every admissible grid
    const unsigned ix = ii % nx, iyz = ii / nx, iy = iyz % ny, iz = iyz / ny;
    x = -p.L[0] + ix * p.h[0];
    y = -p.L[1] + iy * p.h[1];
    z = p.dim == 3 ? -p.L[2] + iz * p.h[2] : 0.0;
}

// Spin densities of Phi (Sec. 1): rho_l = |phi_l|^2, F_z = rho_1 - rho_-1,
// G = conj(phi_1) phi_0 + conj(phi_0) phi_-1, so that F_+/sqrt2 = G and
// |F|^2 = 2 |G|^2 + F_z^2.
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

// Nonlinear part of H(Phi) (Euler-Lagrange equations (2.6)-(2.8)) applied to u
// in the compact form c0 rho u + c1 (F.f) u,
//   (F.f)u = (F_z u1 + conj(G) u0, G u1 + conj(G) u-1, G u0 - F_z u-1).
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
template <typename R>
__device__ __forceinline__ void store3(cpx<R>* f, long long i, long long M, const cpx<double> (&v)[3]) {
    f[i] = cmk((R)v[0].x, (R)v[0].y);
    f[M + i] = cmk((R)v[1].x, (R)v[1].y);
    f[2 * M + i] = cmk((R)v[2].x, (R)v[2].y);
}

__device__ __forceinline__ double re_dot(const cpx<double>& a, const cpx<double>& b) { return a.x * b.x + a.y * b.y; }

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

}  // namespace gs
