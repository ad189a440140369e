// Launchers of the middle pass (k_mid), one kernel per line length, schedule
// candidate and spectral operator.
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

int mid_blocks(int N, int nlines) { return nlines / lpb_mid(N); }
bool mid_cand_ok(int N, int c) { return c >= 0 && c < NCAND && mid_cand_fits(N, c); }
Cand mid_cand_of(int N, int c) { return mid_cand(N, c); }

template hipError_t launch_mid<double>(int, int, const Slot*, int, int, int, int, int, int, const cpx<double>*, int,
                                       hipStream_t);
template hipError_t launch_mid<float>(int, int, const Slot*, int, int, int, int, int, int, const cpx<float>*, int,
                                      hipStream_t);

}  // namespace gs
