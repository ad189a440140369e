// Launch configuration of the FFT passes: the fixed table of tiles and block
// sizes, the candidate schedules the autotuner chooses from, and the grid
// sizing of the persistent passes. Included by the launcher translation units
// (fft_fwd.hip, fft_inv.hip, fft_mid.hip).
#pragma once
#include <algorithm>

#include "fft_core.h"

namespace gs {

// ---------------------------------------------------------------------------
// fixed table (tiles sized so that small grids still give >= ~200 blocks and
// each block's LDS stays near or under 64 KB)
// ---------------------------------------------------------------------------
// Lines per block of the transposing passes. In double, 8 lines give 128-byte
// runs in the transposed stores of the forward passes; the H_L inverse pass,
// which holds two transforms in LDS, keeps 4, and so does the preconditioner's
// last pass: its next tile then fits in registers (pipelined), and a lone
// solve gets twice the blocks (measured at 256^2: same batch time, 10 instead
// of 14 us per launch for one solve).
// Lines longer than 1024 (1200, 2400) keep the LDS of a block near 82 KB.
template <typename R> constexpr int tile_fwd(int N) {
    return sizeof(R) == 8 ? (N >= 1024 ? 2 : (N >= 512 ? 4 : 8)) : (N > 1200 ? 2 : (N >= 1024 ? 4 : 8));
}
template <typename R> constexpr int tile_pre(int N) { return sizeof(R) == 8 ? (N >= 1024 ? 2 : 4) : tile_fwd<R>(N); }
template <typename R> constexpr int tile_inv(int N) {
    return sizeof(R) == 8 ? (N > 1200 ? 1 : (N >= 512 ? 2 : 4)) : (N > 1200 ? 2 : (N >= 512 ? 4 : 8));
}
// Line positions per block of the middle pass (its partial-sum rows are one
// per group of lpb_mid lines: a function of the grid only).
constexpr int lpb_mid(int N) { return N >= 256 ? 1 : (N >= 128 ? 2 : (N >= 64 ? 4 : 8)); }
// threads per block of the fixed table (whole waves)
constexpr int nt_tile0(int N) { return 256; }
constexpr int nt_mid0(int N) { return N >= 1024 ? 512 : 256; }

// ---------------------------------------------------------------------------
// candidate schedules. Candidate 0 is the fixed table. Every candidate of a
// pass computes the same bits: a line's transform does not depend on which
// thread holds which butterfly, the pointwise work is per point, and the
// reducing passes sum in wave chunks of 64 points (chunk_add), independent of
// the block size; their line grouping (lpb_mid, tile_pre) is not a candidate.
// ---------------------------------------------------------------------------
// forward transposing pass: (tile, 256), (tile, 128), (tile / 2, 128)
template <typename R> constexpr Cand fwd_cand(int N, int c) {
    const int t = tile_fwd<R>(N);
    return c == 0 ? Cand{t, nt_tile0(N)} : c == 1 ? Cand{t, 128} : Cand{t > 1 ? t / 2 : t, 128};
}
// inverse transposing pass: (tile, 256), (tile, 128), (tile / 2, 128)
template <typename R> constexpr Cand inv_cand(int N, int c) {
    const int t = tile_inv<R>(N);
    return c == 0 ? Cand{t, nt_tile0(N)} : c == 1 ? Cand{t, 128} : Cand{t > 1 ? t / 2 : t, 128};
}
// last pass of the preconditioner: the tile is fixed; 256, 128 or 512 threads
template <typename R> constexpr Cand pre_cand(int N, int c) {
    const int t = tile_pre<R>(N);
    return c == 0 ? Cand{t, nt_tile0(N)} : c == 1 ? Cand{t, 128} : Cand{t, 512};
}
// middle pass: the fixed block size, half and a quarter of it (at least 64)
constexpr Cand mid_cand(int N, int c) {
    const int nt = nt_mid0(N) >> c;
    return Cand{lpb_mid(N), nt < 64 ? 64 : nt};
}
// at most this many values of a line set per thread (register budget)
constexpr int CAND_MAX_EPT = 24;
template <typename R> constexpr bool fwd_cand_fits(int N, int c) {
    return fwd_cand<R>(N, c).tile * N <= CAND_MAX_EPT * fwd_cand<R>(N, c).nt;
}
template <typename R> constexpr bool inv_cand_fits(int N, int c) {
    return inv_cand<R>(N, c).tile * N <= CAND_MAX_EPT * inv_cand<R>(N, c).nt;
}
template <typename R> constexpr bool pre_cand_fits(int N, int c) {
    return pre_cand<R>(N, c).tile * N <= CAND_MAX_EPT * pre_cand<R>(N, c).nt &&
           pre_cand<R>(N, c).tile * N >= pre_cand<R>(N, c).nt / 4;
}
// (lines longer than 1024 take the split middle pass: k_lfft, k_lspec)
constexpr bool mid_cand_fits(int N, int c) {
    return N <= 1024 && (c == 0 || nt_mid0(N) >> c >= 64) && 3 * lpb_mid(N) * N <= CAND_MAX_EPT * mid_cand(N, c).nt;
}

inline int cu_count() {
    static int n = 0;
    if (!n) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        n = v;
    }
    return n;
}

// Blocks per slot of a transposed pass: one per unit, or, for a pipelined
// kernel, as many as fill the device once, in multiples of 8 (the XCD tile
// order); the occupancy is queried once per kernel.
template <auto KERNEL, bool PIPE, typename... Args>
static hipError_t tile_go(int units, int nslots, int ntb, size_t lds, hipStream_t s, Args... args) {
    int G = units;
    if (PIPE) {
        static int per_cu = -1;
        if (per_cu < 0) {
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, KERNEL, ntb, lds) != hipSuccess || nb <= 0) nb = 1;
            per_cu = nb;
        }
        const long long resident = (long long)per_cu * cu_count();
        const long long g = std::max<long long>(1, (resident + nslots - 1) / nslots);
        if (g < units) G = (int)std::min<long long>(units, std::max<long long>(8, g & ~7LL));
    }
    GS_LAUNCH(KERNEL, dim3((unsigned)G, (unsigned)nslots), dim3(ntb), lds, s, args...);
    return hipGetLastError();
}

// Blocks per slot of a middle pass: one per line group, or, for a pipelined
// kernel, as many as fill the device once (every resident block then loops
// over several groups; the occupancy is queried once per kernel).
template <auto KERNEL, typename MP, typename... Args>
static hipError_t mid_go(int ngroups, int nslots, int ntb, size_t lds, hipStream_t s, Args... args) {
    int G = ngroups;
    if (MP::PIPE) {
        static int per_cu = -1;
        if (per_cu < 0) {
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, KERNEL, ntb, lds) != hipSuccess || nb <= 0) nb = 1;
            per_cu = nb;
        }
        const long long resident = (long long)per_cu * cu_count();
        G = (int)std::min<long long>(ngroups, std::max<long long>(1, (resident + nslots - 1) / nslots));
    }
    GS_LAUNCH(KERNEL, dim3((unsigned)G, (unsigned)nslots), dim3(ntb), lds, s, args...);
    return hipGetLastError();
}

// the supported line lengths: 2^a (16..1024), 3 2^a (24..768), and the
// lengths with factors of 5 of the paper's largest grids and their halvings
#define GS_SWITCH_N(CALL)                        \
    switch (N) {                                 \
    case 16: return CALL(16);                    \
    case 24: return CALL(24);                    \
    case 48: return CALL(48);                    \
    case 96: return CALL(96);                    \
    case 192: return CALL(192);                  \
    case 384: return CALL(384);                  \
    case 768: return CALL(768);                  \
    case 32: return CALL(32);                    \
    case 64: return CALL(64);                    \
    case 128: return CALL(128);                  \
    case 256: return CALL(256);                  \
    case 512: return CALL(512);                  \
    case 1024: return CALL(1024);                \
    case 80: return CALL(80);                    \
    case 160: return CALL(160);                  \
    case 600: return CALL(600);                  \
    case 1200: return CALL(1200);                \
    case 2400: return CALL(2400);                \
    default: return hipErrorInvalidValue;        \
    }

#define GS_SWITCH_CAND(CALL)                     \
    switch (cand) {                              \
    case 0: return CALL(0);                      \
    case 1: return CALL(1);                      \
    case 2: return CALL(2);                      \
    default: return hipErrorInvalidValue;        \
    }

}  // namespace gs
