// Stockham complex FFT for one workgroup, staged through LDS (gfx950).
//
// A length-N transform is done by T = N / P threads; thread t holds the P
// points at positions t + T*m (m = 0..P-1) in registers.  Every radix-R pass
// reads exactly those positions: butterfly j = t + T*b (b < P/R) takes the
// points j + r*N/R = t + T*(b + r*P/R).  It writes its R outputs to the
// autosort positions (j / Ns) * Ns * R + j % Ns + r * Ns, where Ns is the
// product of the radices already applied; after the last pass (Ns * R = N)
// those positions are again t + T*m, so the result stays in registers.  Data
// is therefore loaded from and stored to global memory in coalesced
// t-fastest order, and only the passes in between go through LDS.
//
// The radix sequence is chosen at compile time from {32, 16, 8, 4, 2, 3, 5};
// every radix must divide P.  Twiddles come from a length-N table
// tw[m] = exp(-2 pi i m / N) (double-rounded on the host); the inverse uses
// conjugates.  No normalisation is applied in either direction.
#pragma once

#include "common.h"

FW_BEGIN
struct RadixPlan {
    int np;
    int r[16];
};

constexpr RadixPlan radix_plan(int N, int P) {
    RadixPlan pl{0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
    const int cand[7] = {32, 16, 8, 4, 2, 3, 5};
    int rem = N;
    while (rem > 1) {
        int pick = 0;
        for (int i = 0; i < 7; ++i) {
            if (P % cand[i] == 0 && rem % cand[i] == 0) { pick = cand[i]; break; }
        }
        if (pick == 0 || pl.np == 16) { pl.np = -1; return pl; }
        pl.r[pl.np++] = pick;
        rem /= pick;
    }
    return pl;
}

template <int N, int P>
struct FftShape {
    static_assert(N % P == 0, "P must divide N");
    static constexpr int T = N / P;
    static constexpr RadixPlan plan = radix_plan(N, P);
    static_assert(plan.np > 0, "no radix sequence for (N, P)");
    static constexpr int NP = plan.np;
    static constexpr int ns_before(int i) {
        int s = 1;
        for (int k = 0; k < i; ++k) s *= plan.r[k];
        return s;
    }
};

// Padded LDS index: one spare slot every 16 elements keeps the stride-R
// autosort writes of the first passes off a single bank.
__device__ __forceinline__ int lds_pad(int pos) { return pos + (pos >> 4); }
template <int N>
struct PaddedLen { static constexpr int value = N + N / 16 + 1; };

// The padding is linear over the positions one thread touches in one step:
// pad(b + d) = pad(b) + pad_step(d) whenever (b mod 16) + (d mod 16) < 16.
// The checks below confirm it at compile time, over every thread, for the
// R outputs a radix-R butterfly writes (b = its autosort base, d = r NS)
// and for the P points a thread reads back (b = t, d = T m); those accesses
// then take one padded base per thread plus compile-time offsets, which LDS
// instructions carry as immediates.  LDS accessors provide padded(f, pp),
// the element at an already padded position pp.
constexpr int pad_step(int d) { return d + d / 16; }
constexpr bool pad_linear_writes(int N, int NS, int R) {
    for (int q = 0; q < N; q += NS * R)
        for (int k = 0; k < NS; ++k)
            for (int r = 0; r < R; ++r) {
                const int b = q + k, p = b + r * NS;
                if (p + p / 16 != b + b / 16 + pad_step(r * NS)) return false;
            }
    return true;
}
constexpr bool pad_linear_reads(int N, int P) {
    const int T = N / P;
    for (int t = 0; t < T; ++t)
        for (int m = 0; m < P; ++m) {
            const int p = t + T * m;
            if (p + p / 16 != t + t / 16 + pad_step(T * m)) return false;
        }
    return true;
}

// --------------------------------------------------------- small DFTs -----
template <bool INV>
__device__ __forceinline__ void dft2(cplx& a, cplx& b) {
    const cplx t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(cplx& x0, cplx& x1, cplx& x2, cplx& x3) {
    const cplx a = cadd(x0, x2), b = csub(x0, x2);
    const cplx c = cadd(x1, x3), d = mul_mi<INV>(csub(x1, x3));
    x0 = cadd(a, c);
    x2 = csub(a, c);
    x1 = cadd(b, d);
    x3 = csub(b, d);
}

// multiply by W_M^e = exp(-+ 2 pi i e / M) for compile-time e, M in {8, 16}
template <bool INV, int M, int E>
__device__ __forceinline__ cplx twc(cplx z) {
    constexpr int e = ((E % M) + M) % M;
    constexpr int e16 = e * (16 / M);
    if constexpr (e16 == 0) return z;
    else if constexpr (e16 == 4) return mul_mi<INV>(z);
    else if constexpr (e16 == 8) return mkc(-z.x, -z.y);
    else if constexpr (e16 == 12) return mul_mi<!INV>(z);
    else {
        constexpr double C[16] = {1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508978,
                                  0.0, -0.38268343236508978, -0.70710678118654752, -0.92387953251128674,
                                  -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508978,
                                  0.0, 0.38268343236508978, 0.70710678118654752, 0.92387953251128674};
        constexpr double S[16] = {0.0, 0.38268343236508978, 0.70710678118654752, 0.92387953251128674,
                                  1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508978,
                                  0.0, -0.38268343236508978, -0.70710678118654752, -0.92387953251128674,
                                  -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508978};
        constexpr real c = (real)C[e16];
        constexpr real s = INV ? (real)S[e16] : -(real)S[e16];   // W = c + i s
        return mkc(z.x * c - z.y * s, z.x * s + z.y * c);
    }
}

template <bool INV>
__device__ __forceinline__ void dft8(cplx (&x)[8]) {
    // even / odd halves, then combine with W_8^k
    dft4<INV>(x[0], x[2], x[4], x[6]);
    dft4<INV>(x[1], x[3], x[5], x[7]);
    cplx y[8];
    y[0] = cadd(x[0], x[1]);
    y[4] = csub(x[0], x[1]);
    const cplx o1 = twc<INV, 8, 1>(x[3]);
    y[1] = cadd(x[2], o1);
    y[5] = csub(x[2], o1);
    const cplx o2 = twc<INV, 8, 2>(x[5]);
    y[2] = cadd(x[4], o2);
    y[6] = csub(x[4], o2);
    const cplx o3 = twc<INV, 8, 3>(x[7]);
    y[3] = cadd(x[6], o3);
    y[7] = csub(x[6], o3);
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = y[k];
}

template <bool INV>
__device__ __forceinline__ void dft16(cplx (&x)[16]) {
    // n = n1 + 4 n2: DFT4 over n2, twiddle W16^(n1 k1), DFT4 over n1; out k1 + 4 k2
    dft4<INV>(x[0], x[4], x[8], x[12]);
    dft4<INV>(x[1], x[5], x[9], x[13]);
    dft4<INV>(x[2], x[6], x[10], x[14]);
    dft4<INV>(x[3], x[7], x[11], x[15]);
    // x[n1 + 4 k1] now holds Z_{n1}[k1]
    x[5] = twc<INV, 16, 1>(x[5]);
    x[9] = twc<INV, 16, 2>(x[9]);
    x[13] = twc<INV, 16, 3>(x[13]);
    x[6] = twc<INV, 16, 2>(x[6]);
    x[10] = twc<INV, 16, 4>(x[10]);
    x[14] = twc<INV, 16, 6>(x[14]);
    x[7] = twc<INV, 16, 3>(x[7]);
    x[11] = twc<INV, 16, 6>(x[11]);
    x[15] = twc<INV, 16, 9>(x[15]);
    cplx y[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cplx a = x[4 * k1 + 0], b = x[4 * k1 + 1], c = x[4 * k1 + 2], d = x[4 * k1 + 3];
        dft4<INV>(a, b, c, d);
        y[k1 + 0] = a;
        y[k1 + 4] = b;
        y[k1 + 8] = c;
        y[k1 + 12] = d;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = y[k];
}

// multiply by W_32^e for compile-time e (odd e from cos(k pi / 16), k = 1..7)
template <bool INV, int E>
__device__ __forceinline__ cplx twc32(cplx z) {
    constexpr int e = ((E % 32) + 32) % 32;
    if constexpr (e % 2 == 0) {
        return twc<INV, 16, e / 2>(z);
    } else {
        // cos(2 pi q / 32) for q = 0..8
        constexpr double K[9] = {1.0, 0.980785280403230449126, 0.923879532511286756128,
                                 0.831469612302545237079, 0.707106781186547524401, 0.555570233019602224743,
                                 0.382683432365089771729, 0.195090322016128267848, 0.0};
        // cos and sin of 2 pi e / 32 from the first octant by symmetry
        constexpr int q = e % 8, o = e / 8;   // e = 8 o + q, 0 < q < 8
        constexpr double c0 = K[q], s0 = K[8 - q];
        constexpr double cc = o == 0 ? c0 : o == 1 ? -s0 : o == 2 ? -c0 : s0;
        constexpr double ss = o == 0 ? s0 : o == 1 ? c0 : o == 2 ? -s0 : -c0;
        constexpr real c = (real)cc;
        constexpr real sn = INV ? (real)ss : -(real)ss;   // W = c + i sn
        return mkc(z.x * c - z.y * sn, z.x * sn + z.y * c);
    }
}

template <int K, bool INV>
__device__ __forceinline__ void dft32_combine(cplx (&x)[32], const cplx (&e)[16], const cplx (&o)[16]) {
    if constexpr (K < 16) {
        const cplx t = twc32<INV, K>(o[K]);
        x[K] = cadd(e[K], t);
        x[K + 16] = csub(e[K], t);
        dft32_combine<K + 1, INV>(x, e, o);
    }
}

template <bool INV>
__device__ __forceinline__ void dft32(cplx (&x)[32]) {
    // even / odd 16-point halves, then X[k] = E[k] +- W32^k O[k]
    cplx e[16], o[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        e[i] = x[2 * i];
        o[i] = x[2 * i + 1];
    }
    dft16<INV>(e);
    dft16<INV>(o);
    dft32_combine<0, INV>(x, e, o);
}

template <bool INV>
__device__ __forceinline__ void dft3(cplx& x0, cplx& x1, cplx& x2) {
    const real h = (real)0.86602540378443864676;   // sqrt(3) / 2
    const cplx t1 = cadd(x1, x2);
    const cplx m = mkc(x0.x - 0.5f * t1.x, x0.y - 0.5f * t1.y);
    const cplx d = mul_mi<INV>(cscale(csub(x1, x2), h));
    x0 = cadd(x0, t1);
    x1 = cadd(m, d);
    x2 = csub(m, d);
}

// 5-point DFT from the even / odd sums of the conjugate pairs (1, 4) and
// (2, 3): X_1,4 = x0 + c1 t1 + c2 t2 -+ i (s1 d1 + s2 d2) and
// X_2,3 = x0 + c2 t1 + c1 t2 -+ i (s2 d1 - s1 d2) for the forward sign, with
// c_k = cos(2 pi k / 5), s_k = sin(2 pi k / 5), t = sums, d = differences.
template <bool INV>
__device__ __forceinline__ void dft5(cplx& x0, cplx& x1, cplx& x2, cplx& x3, cplx& x4) {
    const real c1 = (real)0.30901699437494742410, c2 = (real)-0.80901699437494742410;
    const real s1 = (real)0.95105651629515357212, s2 = (real)0.58778525229247312917;
    const cplx t1 = cadd(x1, x4), t2 = cadd(x2, x3);
    const cplx d1 = csub(x1, x4), d2 = csub(x2, x3);
    const cplx a1 = mkc(x0.x + c1 * t1.x + c2 * t2.x, x0.y + c1 * t1.y + c2 * t2.y);
    const cplx a2 = mkc(x0.x + c2 * t1.x + c1 * t2.x, x0.y + c2 * t1.y + c1 * t2.y);
    const cplx b1 = mul_mi<INV>(mkc(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y));
    const cplx b2 = mul_mi<INV>(mkc(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y));
    x0 = cadd(x0, cadd(t1, t2));
    x1 = cadd(a1, b1);
    x4 = csub(a1, b1);
    x2 = cadd(a2, b2);
    x3 = csub(a2, b2);
}

template <int R, bool INV>
__device__ __forceinline__ void dft(cplx (&x)[R]) {
    if constexpr (R == 2) dft2<INV>(x[0], x[1]);
    else if constexpr (R == 3) dft3<INV>(x[0], x[1], x[2]);
    else if constexpr (R == 5) dft5<INV>(x[0], x[1], x[2], x[3], x[4]);
    else if constexpr (R == 4) dft4<INV>(x[0], x[1], x[2], x[3]);
    else if constexpr (R == 8) dft8<INV>(x);
    else if constexpr (R == 16) dft16<INV>(x);
    else if constexpr (R == 32) dft32<INV>(x);
    else static_assert(R == 2, "unsupported radix");
}

// --------------------------------------------------------------- twiddles --
// w[r] = W^(r e) for r = 1..R-1, where W^e = tw[e] (forward; conjugated for
// the inverse).  Only W^e, for R >= 8 W^(4e) and for R = 32 W^(16e) are read
// from the table; the other powers are products of at most five factors (a
// few ulp).
template <int R, bool INV>
__device__ __forceinline__ void twiddles(cplx (&w)[R], const cplx* __restrict__ tw, int e) {
    cplx w1 = tw[e];
    if (INV) w1 = cconj(w1);
    w[1] = w1;
    if constexpr (R >= 3) w[2] = cmul(w1, w1);
    if constexpr (R >= 4) w[3] = cmul(w[2], w1);
    if constexpr (R == 5) w[4] = cmul(w[3], w1);
    if constexpr (R >= 8) {
        cplx w4 = tw[4 * e];
        if (INV) w4 = cconj(w4);
        w[4] = w4;
#pragma unroll
        for (int r = 5; r < 8; ++r) w[r] = cmul(w4, w[r - 4]);
    }
    if constexpr (R >= 16) {
        const cplx w8 = cmul(w[4], w[4]);
        const cplx w12 = cmul(w8, w[4]);
        w[8] = w8;
        w[12] = w12;
#pragma unroll
        for (int r = 1; r < 4; ++r) {
            w[8 + r] = cmul(w8, w[r]);
            w[12 + r] = cmul(w12, w[r]);
        }
    }
    if constexpr (R == 32) {
        cplx w16 = tw[16 * e];
        if (INV) w16 = cconj(w16);
        w[16] = w16;
#pragma unroll
        for (int r = 1; r < 16; ++r) w[16 + r] = cmul(w16, w[r]);
    }
}

// The R outputs of a butterfly with autosort base `base`: x[r] to position
// base + r NS of transform f.
template <int N, int NS, int R, class Lds>
__device__ __forceinline__ void lds_store_outputs(const Lds& lds, int f, int base, const cplx (&x)[R]) {
    if constexpr (pad_linear_writes(N, NS, R)) {
        const int pb = lds_pad(base);
#pragma unroll
        for (int r = 0; r < R; ++r) lds.padded(f, pb + pad_step(r * NS)) = x[r];
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) lds(f, base + r * NS) = x[r];
    }
}

// A thread's P points t + T m of transform f back from LDS.
template <int N, int P, class Lds>
__device__ __forceinline__ void lds_load_points(const Lds& lds, int f, int t, cplx (&v)[P]) {
    constexpr int T = N / P;
    if constexpr (pad_linear_reads(N, P)) {
        const int pt = lds_pad(t);
#pragma unroll
        for (int m = 0; m < P; ++m) v[m] = lds.padded(f, pt + pad_step(T * m));
    } else {
#pragma unroll
        for (int m = 0; m < P; ++m) v[m] = lds(f, t + T * m);
    }
}

// w[r] = W^(r e) = tw[r e] for r = 1..R-1, each read from the table
// (r e < N: e is a multiple of N / (NS R) below N / R).
template <int R, bool INV>
__device__ __forceinline__ void twiddles_direct(cplx (&w)[R], const cplx* __restrict__ tw, int e) {
#pragma unroll
    for (int r = 1; r < R; ++r) {
        const cplx x = tw[r * e];
        w[r] = INV ? cconj(x) : x;
    }
}

// ----------------------------------------------------------- one pass -----
// Pass I of an N-point transform for NF independent transforms held by this
// thread (v[f][m] at position t + T*m).  Non-final passes write to LDS through
// the accessor `lds(f, pos)`; the final pass leaves its outputs in v.
template <int N, int P, int I, bool INV, int NF, bool TWD, class Lds>
__device__ __forceinline__ void fft_pass(cplx (&v)[NF][P], int t,
                                         const cplx* __restrict__ tw, const Lds& lds) {
    using S = FftShape<N, P>;
    constexpr int R = S::plan.r[I];
    constexpr int NS = S::ns_before(I);
    constexpr int NB = P / R;
    constexpr bool LAST = (I == S::NP - 1);
    constexpr int TWS = N / (NS * R);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + S::T * b;
        const int k = j % NS;
        const int base = (j / NS) * NS * R + k;
        cplx w[R];
        if constexpr (NS > 1) {
            if constexpr (TWD) twiddles_direct<R, INV>(w, tw, k * TWS);
            else twiddles<R, INV>(w, tw, k * TWS);
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            cplx x[R];
#pragma unroll
            for (int r = 0; r < R; ++r) x[r] = v[f][b + r * NB];
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) x[r] = cmul(x[r], w[r]);
            }
            dft<R, INV>(x);
            if constexpr (LAST) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[f][b + r * NB] = x[r];
            } else {
                lds_store_outputs<N, NS, R>(lds, f, base, x);
            }
        }
    }
}

template <int N, int P, bool INV, int NF, int I, bool TWD, class Lds>
__device__ __forceinline__ void fft_from(cplx (&v)[NF][P], int t,
                                         const cplx* __restrict__ tw, const Lds& lds) {
    using S = FftShape<N, P>;
    fft_pass<N, P, I, INV, NF, TWD>(v, t, tw, lds);
    if constexpr (I + 1 < S::NP) {
        __syncthreads();
#pragma unroll
        for (int f = 0; f < NF; ++f) lds_load_points<N, P>(lds, f, t, v[f]);
        __syncthreads();
        fft_from<N, P, INV, NF, I + 1, TWD>(v, t, tw, lds);
    }
}

// Full transform.  Every thread of the workgroup must call this (barriers).
// TWD: read every twiddle of a butterfly from the table (a table in LDS),
// instead of the one to three table reads and the products of `twiddles`.
template <int N, int P, bool INV, int NF, bool TWD = false, class Lds>
__device__ __forceinline__ void fft_run(cplx (&v)[NF][P], int t,
                                        const cplx* __restrict__ tw, const Lds& lds) {
    fft_from<N, P, INV, NF, 0, TWD>(v, t, tw, lds);
}

// ------------------------------------------- sequential LDS exchange -----
// Same transform, but the NF transforms of a thread share ONE LDS buffer: a
// pass finishes transform f (butterflies, LDS write, barrier, LDS read,
// barrier) before it starts transform f + 1.  Half the LDS of fft_run for
// NF = 2, at the price of two more barriers per pass.
template <int N, int P, int I, bool INV, int NF, class Lds>
__device__ __forceinline__ void fft_pass_seq(cplx (&v)[NF][P], int t,
                                             const cplx* __restrict__ tw, const Lds& lds) {
    using S = FftShape<N, P>;
    constexpr int R = S::plan.r[I];
    constexpr int NS = S::ns_before(I);
    constexpr int NB = P / R;
    constexpr bool LAST = (I == S::NP - 1);
    constexpr int TWS = N / (NS * R);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = t + S::T * b;
            const int k = j % NS;
            cplx x[R];
#pragma unroll
            for (int r = 0; r < R; ++r) x[r] = v[f][b + r * NB];
            if constexpr (NS > 1) {
                cplx w[R];
                twiddles<R, INV>(w, tw, k * TWS);
#pragma unroll
                for (int r = 1; r < R; ++r) x[r] = cmul(x[r], w[r]);
            }
            dft<R, INV>(x);
            if constexpr (LAST) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[f][b + r * NB] = x[r];
            } else {
                lds_store_outputs<N, NS, R>(lds, 0, (j / NS) * NS * R + k, x);
            }
        }
        if constexpr (!LAST) {
            __syncthreads();
            lds_load_points<N, P>(lds, 0, t, v[f]);
            __syncthreads();
        }
    }
}

template <int N, int P, bool INV, int NF, int I, class Lds>
__device__ __forceinline__ void fft_from_seq(cplx (&v)[NF][P], int t,
                                             const cplx* __restrict__ tw, const Lds& lds) {
    fft_pass_seq<N, P, I, INV, NF>(v, t, tw, lds);
    if constexpr (I + 1 < FftShape<N, P>::NP) fft_from_seq<N, P, INV, NF, I + 1>(v, t, tw, lds);
}

// Full transform with one shared LDS buffer; every thread must call it.  The
// caller must make sure no thread still reads the buffer from earlier use.
template <int N, int P, bool INV, int NF, class Lds>
__device__ __forceinline__ void fft_run_seq(cplx (&v)[NF][P], int t,
                                            const cplx* __restrict__ tw, const Lds& lds) {
    fft_from_seq<N, P, INV, NF, 0>(v, t, tw, lds);
}


FW_END