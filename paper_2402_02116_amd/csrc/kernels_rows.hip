// Row-transform launchers: every (size, points-per-thread) variant with the
// forward store and all inverse epilogues.
#include "fft_kernels.h"

FW_BEGIN
// (size, points per thread) pairs built: the default and the alternative of
// each size (the default only in the complex128 build); the 5 * 2^k lengths
// are x axes of 3-D grids.
#ifdef FW_C128
#define FW_ROW_VARIANTS(X)                                                                           \
    X(16, 16) X(24, 12) X(32, 16) X(48, 12) X(64, 16) X(96, 12) X(128, 16) X(192, 12) X(256, 16)     \
    X(384, 12) X(512, 16) X(768, 12) X(1024, 16) X(1536, 12) X(2048, 16) X(20, 10) X(40, 10) X(80, 10)  \
    X(160, 10)
#else
#define FW_ROW_VARIANTS(X)                                                                          \
    X(16, 16) X(16, 8) X(24, 12) X(24, 24) X(32, 16) X(32, 8) X(48, 12) X(48, 24) X(64, 16) X(64, 8) \
    X(96, 12) X(96, 24) X(128, 16) X(128, 8) X(192, 12) X(192, 24) X(256, 16) X(256, 8) X(384, 12)  \
    X(384, 24) X(512, 16) X(512, 8) X(768, 12) X(768, 24) X(1024, 16) X(1024, 8) X(1536, 12)         \
    X(1536, 24) X(2048, 16) X(2048, 8) X(512, 32) X(1024, 32) X(20, 10) X(40, 10) X(80, 10) X(80, 20)       \
    X(160, 10) X(160, 20)
#endif

hipError_t launch_rows_fwd(int n, int P, const cplx* in, cplx* out, int nrows, int rps, SpecLayout lay,
                           const SysState* st, const cplx* tw, hipStream_t s) {
    if (!row_points_ok(n, P)) return hipErrorInvalidValue;
    const cplx* t = tw + twiddle_offset(n);
#define FW_CASE(N, PP) \
    if (n == N && P == PP) \
        return rows_launch<N, PP, false, EPI_STORE>(in, out, nullptr, nullptr, nullptr, nrows, rps, lay, st, t, s);
    FW_ROW_VARIANTS(FW_CASE)
#undef FW_CASE
    return hipErrorInvalidValue;
}

template <int N, int P>
static hipError_t rows_inv_np(int epi, const cplx* in, const cplx* u, const cplx* aux, cplx* out,
                              double* part, int nrows, int rps, SpecLayout lay, const SysState* st,
                              const cplx* tw, hipStream_t s, const GmEpi* ge) {
    if ((epi == EPI_ARNOLDI || epi == EPI_GMRES_R0) && (!ge || !ge->part))
        return hipErrorInvalidValue;
    if (epi == EPI_ARNOLDI && (!ge->V || ge->nv < 1 || ge->nv > kGmMax + 1)) return hipErrorInvalidValue;
    switch (epi) {
#define FW_EPI(E) \
    case E: return rows_launch<N, P, true, E>(in, out, u, aux, part, nrows, rps, lay, st, tw, s, ge);
        FW_EPI(EPI_STORE) FW_EPI(EPI_APPLY) FW_EPI(EPI_BICG_V) FW_EPI(EPI_BICG_T) FW_EPI(EPI_TRUERES)
        FW_EPI(EPI_ARNOLDI) FW_EPI(EPI_GMRES_R0)
#undef FW_EPI
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_rows_inv(int n, int P, int epi, const cplx* in, const cplx* u, const cplx* aux,
                           cplx* out, double* part, int nrows, int rps, SpecLayout lay, const SysState* st,
                           const cplx* tw, hipStream_t s, const GmEpi* ge) {
    if (!row_points_ok(n, P)) return hipErrorInvalidValue;
    const cplx* t = tw + twiddle_offset(n);
#define FW_CASE(N, PP) \
    if (n == N && P == PP) return rows_inv_np<N, PP>(epi, in, u, aux, out, part, nrows, rps, lay, st, t, s, ge);
    FW_ROW_VARIANTS(FW_CASE)
#undef FW_CASE
    return hipErrorInvalidValue;
}

FW_END