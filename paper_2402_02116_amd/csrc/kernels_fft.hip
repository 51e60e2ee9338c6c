// Host side of the FFT passes: supported sizes, the twiddle table, launch
// geometry and the kernel variants (points per thread, columns per block,
// LDS sharing) that the autotuner chooses from.
#include <algorithm>
#include <numeric>

#include "fft.h"
#include "launch.h"

FW_BEGIN
// ------------------------------------------------------------ sizes ------
#define FW_FOR_EACH_SIZE(X) \
    X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(1536) X(2048)

static const int kSizes[] = {16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048};
// Twiddle tables: the 2-D sizes, then the 5 * 2^k axis lengths of 3-D grids.
static const int kTwSizes[] = {16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048,
                               20, 40, 80, 160};

// Default points per thread.  Row passes: 16 for powers of two (radix-16
// passes), 12 for 3 * 2^k.  Column passes hold both field components per
// thread, so they default to 8 (radix 8) to keep registers low and the
// thread count high.  Each size also has one alternative per pass kind.
// The complex128 build has the default variants only.
int row_points_default(int n) { return (n % 5 == 0) ? 10 : (n % 3 == 0) ? 12 : 16; }
static int col_points_default(int n) { return (n % 3 == 0) ? 12 : 8; }
#ifdef FW_C128
static int row_points_alt(int n) { return row_points_default(n); }
static int col_points_alt(int n) { return col_points_default(n); }
static int col_points_small(int) { return 0; }
static int points_radix32(int) { return 0; }
#else
// A third column-pass variant for power-of-two columns up to 256 points: 4
// points per thread (radix-4 passes), four times the threads of the 16-point
// variant, for small batches where a block per CU leaves the pass latency-bound.
static int col_points_small(int n) { return (n % 3 != 0 && n % 5 != 0 && n <= 256) ? 4 : 0; }
static int row_points_alt(int n) { return (n % 5 == 0) ? (n > 40 ? 20 : 10) : (n % 3 == 0) ? 24 : 8; }
static int col_points_alt(int n) { return (n % 3 == 0) ? 24 : 16; }
// A third row-pass variant for 512- and 1024-point rows: 32 points per
// thread, radix-32 passes (32 x 32 at 1024 points: one LDS exchange per
// direction instead of two).  Column passes hold both field components (or
// twice the threads) and spill at 32 points, so they have none.
static int points_radix32(int n) { return (n == 512 || n == 1024) ? 32 : 0; }
#endif

// The 1024-thread shared-buffer column pass exists for long power-of-two
// columns with 8 points per thread only (complex64): more points per thread
// exceed the 128 registers of a 1024-thread block and spill.
static bool cols_wide_built(int n, int P) {
#ifdef FW_C128
    (void)n;
    (void)P;
    return false;
#else
    return n >= 512 && n % 3 != 0 && P == 8;
#endif
}

// The column pass with the twiddle table in LDS (seq 4) exists for
// power-of-two columns with 4 or 8 points per thread and tiles of 4, 8 or 16
// columns (complex64).
static bool cols_tw_built(int n, int P) {
#ifdef FW_C128
    (void)n;
    (void)P;
    return false;
#else
    return n % 3 != 0 && n % 5 != 0 && (P == 4 || P == 8);
#endif
}

bool fft_size_supported(int n) {
    for (int s : kSizes)
        if (s == n) return true;
    return false;
}

size_t twiddle_table_elems() {
    size_t t = 0;
    for (int s : kTwSizes) t += (size_t)s;
    return t;
}

size_t twiddle_offset(int n) {
    size_t t = 0;
    for (int s : kTwSizes) {
        if (s == n) return t;
        t += (size_t)s;
    }
    return (size_t)-1;
}

void twiddle_table_fill(cplx* host) {
    size_t off = 0;
    for (int s : kTwSizes) {
        for (int m = 0; m < s; ++m) {
            // exp(-2 pi i m / s); angle reduced in double
            const double a = -2.0 * 3.14159265358979323846 * (double)m / (double)s;
            host[off + m] = mkc((real)cos(a), (real)sin(a));
        }
        off += (size_t)s;
    }
}

bool row_points_ok(int n, int P) {
    return (fft_size_supported(n) || axis3_size_supported(n)) && n % P == 0 &&
           (P == row_points_default(n) || P == row_points_alt(n) || P == points_radix32(n));
}

int row_candidates(int n, int* out) {
    int k = 0;
    out[k++] = row_points_default(n);
    if (row_points_alt(n) != out[0] && n % row_points_alt(n) == 0) out[k++] = row_points_alt(n);
    if (points_radix32(n)) out[k++] = points_radix32(n);
    return k;
}

RowGeom row_geom(int n, int P, int rows_per_sys) {
    const int T = n / P;
    int F = std::gcd(256 / T, rows_per_sys);
    RowGeom g;
    g.F = F;
    g.threads = ((F * T + 63) / 64) * 64;
    g.blocks_per_sys = rows_per_sys / F;
    return g;
}

static int padded_len(int n) { return n + n / 16 + 1; }

// Column blocks: W columns x T threads per column, at most 512 threads.  With
// W = 16 every 16-lane LDS access group is one contiguous 128-byte row segment
// (no bank conflicts) and every global access a full 128-byte line.
ColGeom col_geom(int nz, int nx, const ColCfg& c) {
    (void)nx;
    const int T = nz / c.P;
    ColGeom g;
    if (c.seq == 4) {   // the LDS-twiddle pass: two column buffers and the twiddle table
        g.threads = c.W * T;
        g.slots = c.W;
        g.lds = ((size_t)padded_len(nz) * c.W * 2 + nz) * sizeof(cplx);
        return g;
    }
    // seq 3: the shared-buffer pass (seq 1) in blocks of up to 1024 threads
    if (c.seq == 2) {   // both components' columns in LDS, no idle threads
        g.threads = 2 * c.W * T;
        g.slots = c.W;
        g.lds = (size_t)padded_len(nz) * c.W * 2 * sizeof(cplx);
        return g;
    }
    g.threads = ((c.W * T + 63) / 64) * 64;
    g.slots = c.W + (g.threads > c.W * T ? 1 : 0);   // idle threads need a private dummy slot
    g.lds = (size_t)padded_len(nz) * g.slots * (c.seq ? 1 : 2) * sizeof(cplx);
    return g;
}

bool col_cfg_ok(int nz, int nx, const ColCfg& c) {
    if (!fft_size_supported(nz) || c.P <= 0 || nz % c.P != 0) return false;
    if (c.P != col_points_default(nz) && c.P != col_points_alt(nz) && c.P != col_points_small(nz)) return false;
    if (c.seq < 0 || c.seq > 4) return false;
    if (c.W < 1 || c.W > 64 || nx % c.W != 0 || (c.W & (c.W - 1)) != 0) return false;
    const ColGeom g = col_geom(nz, nx, c);
    // the component-split pass at 24 points per thread spills registers
    if (c.seq == 2) return c.P < 24 && g.threads % 64 == 0 && g.threads <= 512 && g.lds <= kMaxLds;
    if (c.seq == 3) return cols_wide_built(nz, c.P) && g.threads > 512 && g.threads <= 1024 && g.lds <= kMaxLds;
    if (c.seq == 4)
        return cols_tw_built(nz, c.P) && c.W >= 4 && c.W <= 16 && g.threads % 64 == 0 && g.threads <= 512 &&
               g.lds <= kMaxLds;
    return g.threads <= 512 && g.lds <= kMaxLds;
}

ColCfg col_default(int nz, int nx) {
    ColCfg c{col_points_default(nz), 1, 1};
    const int T = nz / c.P;
    int W = std::max(1, std::min(16, 512 / T));
    while (W > 1 && nx % W != 0) W /= 2;
    c.W = W;
    return c;
}

int col_candidates(int nz, int nx, ColCfg* out, int cap) {
    int k = 0;
    const int ps[3] = {col_points_default(nz), col_points_alt(nz), col_points_small(nz)};
    for (int i = 0; i < 3; ++i) {
        const int P = ps[i];
        if (P == 0 || (i > 0 && P == ps[0]) || (i > 1 && P == ps[1])) continue;
        for (int seq = 4; seq >= 0; --seq)
            for (int W = 4; W <= 32; W *= 2) {
                const ColCfg c{P, W, seq};
                if (col_cfg_ok(nz, nx, c) && k < cap) out[k++] = c;
            }
    }
    return k;
}
FW_END