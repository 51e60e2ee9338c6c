// Column-pass launchers: the Green-multiply pass in every (size, points per
// thread, LDS sharing or component split, block-size bound, twiddles in
// LDS) variant; the plain forward / inverse column transforms (2-D FFT
// entry point) in the default variant.
#include "fft_kernels.h"

FW_BEGIN
#ifdef FW_C128
constexpr bool kWideCols = false;   // the 1024-thread pass is complex64 only
constexpr bool kTwCols = false;   // so is the LDS-twiddle pass
#define FW_COL_VARIANTS(X)                                                                         \
    X(16, 8) X(24, 12) X(32, 8) X(48, 12) X(64, 8) X(96, 12) X(128, 8) X(192, 12) X(256, 8)        \
    X(384, 12) X(512, 8) X(768, 12) X(1024, 8) X(1536, 12) X(2048, 8)
#else
constexpr bool kWideCols = true;
constexpr bool kTwCols = true;
#define FW_COL_VARIANTS(X)                                                                        \
    X(16, 8) X(16, 16) X(16, 4) X(24, 12) X(24, 24) X(32, 8) X(32, 16) X(32, 4) X(48, 12) X(48, 24)  \
    X(64, 8) X(64, 16) X(64, 4) X(96, 12) X(96, 24) X(128, 8) X(128, 16) X(128, 4) X(192, 12)        \
    X(192, 24) X(256, 8) X(256, 16) X(256, 4) X(384, 12) X(384, 24) X(512, 8) X(512, 16) X(768, 12)  \
    X(768, 24) X(1024, 8) X(1024, 16) X(1536, 12) X(1536, 24) X(2048, 8) X(2048, 16)
#endif

hipError_t launch_cols(int mode, const ColCfg& c, cplx* data, const ProbDev& pd, const SysState* st,
                       const cplx* tw, hipStream_t s) {
    const int n = pd.nz;
    if (!col_cfg_ok(n, pd.nx, c)) return hipErrorInvalidValue;
    if (mode != COL_GREEN && !(c.P == col_default(n, pd.nx).P && c.seq == 1)) return hipErrorInvalidValue;
    const cplx* t = tw + twiddle_offset(n);
#define FW_CASE(N, PP)                                                                          \
    if (n == N && c.P == PP) {                                                                  \
        if (mode == COL_GREEN) {                                                                \
            if constexpr (kWideCols && N >= 512 && N % 3 != 0 && PP == 8)                                    \
                if (c.seq == 3) return cols_launch<N, PP, COL_GREEN, true, 1024>(data, pd, c.W, st, t, s); \
            if constexpr (PP < 24)                                                              \
                if (c.seq == 2) return cols_split_launch<N, PP>(data, pd, c.W, st, t, s);     \
            if constexpr (kTwCols && N % 3 != 0 && (PP == 4 || PP == 8))                     \
                if (c.seq == 4) return cols_tw_launch<N, PP>(data, pd, c.W, st, t, s);        \
            return c.seq == 1 ? cols_launch<N, PP, COL_GREEN, true>(data, pd, c.W, st, t, s)    \
                              : cols_launch<N, PP, COL_GREEN, false>(data, pd, c.W, st, t, s);  \
        }                                                                                       \
        if constexpr (PP == ((N % 3 == 0) ? 12 : 8)) {                                         \
            if (mode == COL_FWD) return cols_launch<N, PP, COL_FWD, true>(data, pd, c.W, st, t, s); \
            if (mode == COL_INV) return cols_launch<N, PP, COL_INV, true>(data, pd, c.W, st, t, s); \
        }                                                                                       \
        return hipErrorInvalidValue;                                                            \
    }
    FW_COL_VARIANTS(FW_CASE)
#undef FW_CASE
    return hipErrorInvalidValue;
}

FW_END