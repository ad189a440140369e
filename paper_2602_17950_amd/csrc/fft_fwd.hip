// Launchers of the forward transposing pass (k_fwdT), one kernel per line
// length, schedule candidate and prologue.
#include "fft_launch.h"

namespace gs {

template <typename R, typename RX, int N, int C>
static hipError_t fwdT_nc(int pro, int dual, const Slot* slots, int nslots, int in, int out, int aux0, int aux1,
                          int A, int B, int ncomp, const cpx<R>* tw, hipStream_t s) {
    if constexpr (!fwd_cand_fits<R>(N, C)) {
        return hipErrorInvalidValue;
    } else {
        constexpr int TILE = fwd_cand<R>(N, C).tile;
        constexpr int NTB = fwd_cand<R>(N, C).nt;
        if (B % TILE) return hipErrorInvalidValue;
        const size_t lds = (size_t)TILE * Lay<N>::P * sizeof(cpx<R>);
        dim3 grid((unsigned)((long long)(dual ? 6 : ncomp) * A * (B / TILE)), (unsigned)nslots);
        if (dual && pro == PRO_DIR) {
            GS_LAUNCH((k_fwdT<R, RX, N, TILE, PRO_DIR, true, NTB>), grid, dim3(NTB), lds, s, slots, in, out, aux0,
                      aux1, A, B, tw);
        } else if (!dual && pro == PRO_PLAIN) {
            // the plain transform reads no operand of the other type
            GS_LAUNCH((k_fwdT<R, R, N, TILE, PRO_PLAIN, false, NTB>), grid, dim3(NTB), lds, s, slots, in, out, aux0,
                      -1, A, B, tw);
        } else {
            return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
}

template <typename R, typename RX>
hipError_t launch_fwdT(int N, int pro, int dual, const Slot* slots, int nslots, int in, int out, int aux0,
                       int aux1, int A, int B, int ncomp, const cpx<R>* tw, int cand, hipStream_t s) {
#define CALLC(c) fwdT_nc<R, RX, NN, c>(pro, dual, slots, nslots, in, out, aux0, aux1, A, B, ncomp, tw, s)
#define CALL(n)                                                                                                 \
    [&]() -> hipError_t {                                                                                       \
        constexpr int NN = n;                                                                                   \
        GS_SWITCH_CAND(CALLC)                                                                                   \
    }()
    GS_SWITCH_N(CALL)
#undef CALL
#undef CALLC
}

// candidate c of the pass for lines of length N, with B (a multiple of the tile) lines
template <typename R> bool fwdT_cand_ok(int N, int c, int B) {
    return c >= 0 && c < NCAND && fwd_cand_fits<R>(N, c) && B % fwd_cand<R>(N, c).tile == 0;
}
template <typename R> Cand fwdT_cand_of(int N, int c) { return fwd_cand<R>(N, c); }

template hipError_t launch_fwdT<double, double>(int, int, int, const Slot*, int, int, int, int, int, int, int, int,
                                                const cpx<double>*, int, hipStream_t);
template hipError_t launch_fwdT<float, float>(int, int, int, const Slot*, int, int, int, int, int, int, int, int,
                                              const cpx<float>*, int, hipStream_t);
template hipError_t launch_fwdT<float, double>(int, int, int, const Slot*, int, int, int, int, int, int, int, int,
                                               const cpx<float>*, int, hipStream_t);
template hipError_t launch_fwdT<double, float>(int, int, int, const Slot*, int, int, int, int, int, int, int, int,
                                               const cpx<double>*, int, hipStream_t);
template bool fwdT_cand_ok<double>(int, int, int);
template bool fwdT_cand_ok<float>(int, int, int);
template Cand fwdT_cand_of<double>(int, int);
template Cand fwdT_cand_of<float>(int, int);

}  // namespace gs
