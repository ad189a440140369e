// Launchers of the middle pass (k_mid), one kernel per line length, schedule
// candidate and spectral operator.
#include <cstdint>

#include "fft_launch.h"

namespace gs {

template <typename R, int N, int C>
static hipError_t mid_nc(int op, const Slot* slots, int nslots, int in, int outA, int outB, int nlines,
                         int rot_any, const cpx<R>* tw, hipStream_t s) {
    if constexpr (!mid_cand_fits(N, C)) {
        return hipErrorInvalidValue;
    } else {
        constexpr int LPB = mid_cand(N, C).tile;
        constexpr int NTB = mid_cand(N, C).nt;
        if (nlines % LPB) return hipErrorInvalidValue;
        const int ngroups = nlines / LPB;
        using HL = MidPlan<R, N, LPB, MID_HL, NTB>;
        using HX = MidPlan<R, N, LPB, MID_HLX, NTB>;
        using PR = MidPlan<R, N, LPB, MID_PRE, NTB>;
        const bool ra = rot_any != 0;
        if (op == MID_HL)
            return mid_go<k_mid<R, N, LPB, MID_HL, NTB>, HL>(ngroups, nslots, NTB, HL::tw_offset(ra) + HL::TW_BYTES,
                                                             s, slots, in, outA, outB, nlines, rot_any, tw);
        if (op == MID_HLX)
            return mid_go<k_mid<R, N, LPB, MID_HLX, NTB>, HX>(ngroups, nslots, NTB, HX::tw_offset(ra) + HX::TW_BYTES,
                                                              s, slots, in, outA, outB, nlines, rot_any, tw);
        return mid_go<k_mid<R, N, LPB, MID_PRE, NTB>, PR>(ngroups, nslots, NTB, PR::tw_offset(false) + PR::TW_BYTES,
                                                          s, slots, in, outA, outB, nlines, 0, tw);
    }
}

template <typename R>
hipError_t launch_mid(int N, int op, const Slot* slots, int nslots, int in, int outA, int outB, int nlines,
                      int rot_any, const cpx<R>* tw, int cand, hipStream_t s) {
#define CALLC(c) mid_nc<R, NN, c>(op, slots, nslots, in, outA, outB, nlines, rot_any, tw, s)
#define CALL(n)                                                                                                 \
    [&]() -> hipError_t {                                                                                       \
        constexpr int NN = n;                                                                                   \
        GS_SWITCH_CAND(CALLC)                                                                                   \
    }()
    GS_SWITCH_N(CALL)
#undef CALL
#undef CALLC
}

// k_lfft: one line per block of 256 threads; lines longer than 1024 only
template <typename R, int N, bool INV>
static hipError_t lfft_n(const Slot* slots, int nslots, int iin, int iout, int ncomp, int nlines, int irot,
                         int iin2, int iout2, const cpx<R>* tw, hipStream_t s) {
    constexpr int NT = 256;
    const long long blocks = (long long)(ncomp + (iin2 >= 0 ? 3 : 0)) * nlines;
    if (blocks <= 0 || blocks > INT32_MAX) return hipErrorInvalidValue;
    GS_LAUNCH((k_lfft<R, N, INV, NT>), dim3((unsigned)blocks, (unsigned)nslots), dim3(NT),
              (size_t)Lay<N>::P * sizeof(cpx<R>), s, slots, iin, iout, ncomp, nlines, irot, iin2, iout2, tw);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_lfft(int N, int inv, const Slot* slots, int nslots, int iin, int iout, int ncomp, int nlines,
                       int irot, int iin2, int iout2, const cpx<R>* tw, hipStream_t s) {
#define LF(n) (inv ? lfft_n<R, n, true>(slots, nslots, iin, iout, ncomp, nlines, irot, iin2, iout2, tw, s) \
                   : lfft_n<R, n, false>(slots, nslots, iin, iout, ncomp, nlines, irot, iin2, iout2, tw, s))
    switch (N) {
    case 1200: return LF(1200);
    case 2400: return LF(2400);
    default: return hipErrorInvalidValue;
    }
#undef LF
}

template <typename R>
hipError_t launch_lspec(int op, const Slot* slots, int nslots, int in, int outA, int outB, int N, int nlines,
                        int rot_any, hipStream_t s) {
    const dim3 grid((unsigned)pw_blocks((long long)N * nlines), (unsigned)nslots);
    switch (op) {
    case MID_HL: GS_LAUNCH((k_lspec<R, MID_HL>), grid, dim3(PT), 0, s, slots, in, outA, outB, N, rot_any); break;
    case MID_HLX: GS_LAUNCH((k_lspec<R, MID_HLX>), grid, dim3(PT), 0, s, slots, in, outA, outB, N, rot_any); break;
    case MID_PRE: GS_LAUNCH((k_lspec<R, MID_PRE>), grid, dim3(PT), 0, s, slots, in, outA, outB, N, 0); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// partial-sum rows of the middle pass: one per line group, or, for the split
// pass of long lines, one per block of its pointwise grid
int mid_blocks(int N, int nlines) { return N > 1024 ? pw_blocks((long long)N * nlines) : nlines / lpb_mid(N); }
bool mid_cand_ok(int N, int c) { return c >= 0 && c < NCAND && mid_cand_fits(N, c); }
Cand mid_cand_of(int N, int c) { return mid_cand(N, c); }

template hipError_t launch_mid<double>(int, int, const Slot*, int, int, int, int, int, int, const cpx<double>*, int,
                                       hipStream_t);
template hipError_t launch_mid<float>(int, int, const Slot*, int, int, int, int, int, int, const cpx<float>*, int,
                                      hipStream_t);
template hipError_t launch_lfft<double>(int, int, const Slot*, int, int, int, int, int, int, int, int,
                                        const cpx<double>*, hipStream_t);
template hipError_t launch_lfft<float>(int, int, const Slot*, int, int, int, int, int, int, int, int,
                                       const cpx<float>*, hipStream_t);
template hipError_t launch_lspec<double>(int, const Slot*, int, int, int, int, int, int, int, hipStream_t);
template hipError_t launch_lspec<float>(int, const Slot*, int, int, int, int, int, int, int, hipStream_t);

}  // namespace gs
