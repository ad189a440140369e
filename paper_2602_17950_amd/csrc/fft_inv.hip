// Launchers of the inverse transposing passes (k_invT, and k_invT_pre, the
// preconditioner's last pass), one kernel per line length, schedule candidate
// and epilogue.
#include "fft_launch.h"

namespace gs {

template <typename R, int N, int C>
static hipError_t invT_nc(int epi, const Slot* slots, int nslots, int in, int in2, int out, int out2, int uin,
                          int B, int Cc, double scale, int use_invnP, int rot_any, const cpx<R>* tw, hipStream_t s) {
    if constexpr (!inv_cand_fits<R>(N, C)) {
        return hipErrorInvalidValue;
    } else {
        constexpr int TILE = inv_cand<R>(N, C).tile;
        constexpr int NTB = inv_cand<R>(N, C).nt;
        using TP = TilePlan<R, N, TILE, NTB>;
        if (Cc % TILE) return hipErrorInvalidValue;
        const int units = 3 * B * (Cc / TILE);
        const size_t lds = TP::tw_offset(epi == EPI_SCALE ? 1 : 2) + TP::TW_BYTES;
        switch (epi) {
        case EPI_SCALE:
            return tile_go<k_invT<R, N, TILE, EPI_SCALE, NTB>, TP::PIPE>(units, nslots, NTB, lds, s, slots, in, in2,
                                                                          out, out2, uin, B, Cc, scale, use_invnP,
                                                                          rot_any, tw);
        case EPI_HL:
            return tile_go<k_invT<R, N, TILE, EPI_HL, NTB>, TP::PIPE>(units, nslots, NTB, lds, s, slots, in, in2,
                                                                       out, out2, uin, B, Cc, scale, use_invnP,
                                                                       rot_any, tw);
        case EPI_ROTX:
            return tile_go<k_invT<R, N, TILE, EPI_ROTX, NTB>, TP::PIPE>(units, nslots, NTB, lds, s, slots, in, in2,
                                                                         out, out2, uin, B, Cc, scale, use_invnP,
                                                                         rot_any, tw);
        default:
            return hipErrorInvalidValue;
        }
    }
}

template <typename R>
hipError_t launch_invT(int N, int epi, const Slot* slots, int nslots, int in, int in2, int out, int out2,
                       int uin, int B, int Cc, double scale, int use_invnP, int rot_any, const cpx<R>* tw, int cand,
                       hipStream_t s) {
#define CALLC(c) invT_nc<R, NN, c>(epi, slots, nslots, in, in2, out, out2, uin, B, Cc, scale, use_invnP, rot_any, tw, s)
#define CALL(n)                                                                                                 \
    [&]() -> hipError_t {                                                                                       \
        constexpr int NN = n;                                                                                   \
        GS_SWITCH_CAND(CALLC)                                                                                   \
    }()
    GS_SWITCH_N(CALL)
#undef CALL
#undef CALLC
}

template <typename R, typename RS, int N, int C>
static hipError_t invT_pre_nc(const Slot* slots, int nslots, int in, int out, int B, int Cc, int dir,
                              const cpx<R>* tw, hipStream_t s) {
    if constexpr (!pre_cand_fits<R>(N, C)) {
        return hipErrorInvalidValue;
    } else {
        constexpr int TILE = pre_cand<R>(N, C).tile;
        constexpr int NTB = pre_cand<R>(N, C).nt;
        using TP = TilePlan<R, N, TILE, NTB>;
        if (Cc % TILE) return hipErrorInvalidValue;
        static_assert(NS_DIR <= RED_DIR_STRIDE, "partial-sum row");
        return tile_go<k_invT_pre<R, RS, N, TILE, NTB>, TP::PIPE>(3 * B * (Cc / TILE), nslots, NTB,
                                                                   TP::tw_offset(1) + TP::TW_BYTES, s, slots, in,
                                                                   out, B, Cc, dir, tw);
    }
}

template <typename R, typename RS>
hipError_t launch_invT_pre(int N, const Slot* slots, int nslots, int in, int out, int B, int Cc, int dir,
                           const cpx<R>* tw, int cand, hipStream_t s) {
#define CALLC(c) invT_pre_nc<R, RS, NN, c>(slots, nslots, in, out, B, Cc, dir, tw, s)
#define CALL(n)                                                                                                 \
    [&]() -> hipError_t {                                                                                       \
        constexpr int NN = n;                                                                                   \
        GS_SWITCH_CAND(CALLC)                                                                                   \
    }()
    GS_SWITCH_N(CALL)
#undef CALL
#undef CALLC
}

// blocks (= partial-sum rows) of launch_invT_pre for these sizes (the tile is
// the same for every candidate)
template <typename R> int invT_pre_blocks(int N, int B, int Cc) { return 3 * B * (Cc / tile_pre<R>(N)); }

template <typename R> bool invT_cand_ok(int N, int c, int Cc) {
    return c >= 0 && c < NCAND && inv_cand_fits<R>(N, c) && Cc % inv_cand<R>(N, c).tile == 0;
}
template <typename R> bool invT_pre_cand_ok(int N, int c) { return c >= 0 && c < NCAND && pre_cand_fits<R>(N, c); }
template <typename R> Cand invT_cand_of(int N, int c) { return inv_cand<R>(N, c); }
template <typename R> Cand invT_pre_cand_of(int N, int c) { return pre_cand<R>(N, c); }

template hipError_t launch_invT<double>(int, int, const Slot*, int, int, int, int, int, int, int, int, double, int,
                                        int, const cpx<double>*, int, hipStream_t);
template hipError_t launch_invT<float>(int, int, const Slot*, int, int, int, int, int, int, int, int, double, int,
                                       int, const cpx<float>*, int, hipStream_t);
template hipError_t launch_invT_pre<double, double>(int, const Slot*, int, int, int, int, int, int,
                                                    const cpx<double>*, int, hipStream_t);
template hipError_t launch_invT_pre<float, float>(int, const Slot*, int, int, int, int, int, int, const cpx<float>*,
                                                  int, hipStream_t);
template hipError_t launch_invT_pre<float, double>(int, const Slot*, int, int, int, int, int, int,
                                                   const cpx<float>*, int, hipStream_t);
template int invT_pre_blocks<double>(int, int, int);
template int invT_pre_blocks<float>(int, int, int);
template bool invT_cand_ok<double>(int, int, int);
template bool invT_cand_ok<float>(int, int, int);
template bool invT_pre_cand_ok<double>(int, int);
template bool invT_pre_cand_ok<float>(int, int);
template Cand invT_cand_of<double>(int, int);
template Cand invT_cand_of<float>(int, int);
template Cand invT_pre_cand_of<double>(int, int);
template Cand invT_pre_cand_of<float>(int, int);

}  // namespace gs
