// LDS-resident tile FFT engine for gfx950 (wave64).
//
// A tile holds W real pencils ("columns") of one transform axis.  Columns
// 2s and 2s+1 form complex sequence s (real part / imaginary part), so one
// complex FFT of length N = 2M transforms two real pencils at once.  The tile
// lives in LDS as a real array buf[row * rs + col] (rows 0..N-1, rs = W + 1:
// the odd padding keeps row-wise and column-wise accesses nearly free of
// bank conflicts); complex element (n, s) is (buf[n*rs + 2s], buf[n*rs + 2s+1]).
//
// Transform kinds built on the length-N complex FFT (M = N/2):
//   forward, zero padded : f_1..f_{M-1} at positions 1..M-1, zeros elsewhere;
//                          C[k] = sum_j f_j cos(pi k j/M), k = 0..M
//                          S[k] = sum_j f_j sin(pi k j/M), k = 1..M-1
//                          "slot" layout: row k = C[k], row M+k = S[k]
//                          (S alone is the raw DST-I)
//   forward, even        : f_0..f_M mirrored to length N; the spectrum is real,
//                          F[k] = f_0 + (-1)^k f_M + 2 sum_{j=1}^{M-1} f_j cos(pi k j/M)
//   inverse, hermitian   : from slots C, S: y_j = sum_{k=0}^{N-1} F_k e^{+i pi k j/M}
//                          with F_k = C_k - i S_k and F_{N-k} = conj(F_k), i.e.
//                          y_j = C_0 + (-1)^j C_M + 2 sum_{k=1}^{M-1}(C_k cos + S_k sin)
//
// The FFT itself is a Stockham autosort transform with radix-2/3/4/5/7/8
// butterflies held in registers and a direct (output-by-output) stage for
// any other prime factor.  Twiddles come from a table w[t] = exp(-2 pi i t/N)
// computed on the host in extended precision.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ips {

template <typename T>
struct cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }

template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }

// multiply by -i (forward) or +i (inverse); the direction is a template
// argument throughout the engine, so no per-element selects are emitted
template <typename T, bool INV>
__device__ __forceinline__ cx<T> rot90(cx<T> a)
{
    if constexpr (INV)
        return cx<T>{-a.y, a.x};
    else
        return cx<T>{a.y, -a.x};
}

constexpr int kMaxStages = 16;

struct FftDesc {
    int N;   // transform length (even)
    int M;   // N / 2
    int nst; // number of Stockham stages
    int rad[kMaxStages];
    int ns[kMaxStages];          // product of the radices before the stage
    unsigned nsmag[kMaxStages];  // ceil(2^32 / ns) for ns not a power of two, else 0
    int nslg[kMaxStages];        // log2(ns) when ns is a power of two
};

// j mod ns for j < 2^16 (exact with the precomputed reciprocal)
__device__ __forceinline__ int fmod_ns(int j, int ns, unsigned mag, int lg)
{
    if (mag == 0) return j & (ns - 1);
    const int q = (int)__umulhi((unsigned)j, mag);
    return j - q * ns;
}

template <typename T>
__device__ __forceinline__ cx<T> lds_c(const T *buf, int rs, int n, int s)
{
    const T *p = buf + n * rs + 2 * s;
    return {p[0], p[1]};
}

template <typename T>
__device__ __forceinline__ void lds_cs(T *buf, int rs, int n, int s, cx<T> v)
{
    T *p = buf + n * rs + 2 * s;
    p[0] = v.x;
    p[1] = v.y;
}

template <typename T, bool INV>
__device__ __forceinline__ cx<T> twid(const cx<T> *tw, int t)
{
    cx<T> w = tw[t];
    if constexpr (INV) w.y = -w.y;
    return w;
}

// Last step of a length-8 DFT from the length-4 DFTs e of the even and o of
// the odd inputs: a[k] = e[k] + w8^k o[k], a[k+4] = e[k] - w8^k o[k].
template <typename T, bool INV>
__device__ __forceinline__ void dft8_combine(cx<T> *a, const cx<T> *e, const cx<T> *o)
{
    const T r = (T)0.70710678118654752440084436210484903928;
    cx<T> o1, o3;
    if constexpr (INV) {
        o1 = cx<T>{r * (o[1].x - o[1].y), r * (o[1].x + o[1].y)};
        o3 = cx<T>{-r * (o[3].x + o[3].y), r * (o[3].x - o[3].y)};
    } else {
        o1 = cx<T>{r * (o[1].x + o[1].y), r * (o[1].y - o[1].x)};
        o3 = cx<T>{r * (o[3].y - o[3].x), -r * (o[3].x + o[3].y)};
    }
    const cx<T> o2 = rot90<T, INV>(o[2]);
    a[0] = cadd(e[0], o[0]);
    a[4] = csub(e[0], o[0]);
    a[1] = cadd(e[1], o1);
    a[5] = csub(e[1], o1);
    a[2] = cadd(e[2], o2);
    a[6] = csub(e[2], o2);
    a[3] = cadd(e[3], o3);
    a[7] = csub(e[3], o3);
}

// Length-8 DFT of a[0..3] followed by four zeros: the first stage of a
// transform whose upper half of inputs is zero (zero-padded sequences).
template <typename T, bool INV>
__device__ __forceinline__ void dft8_lower(cx<T> *a)
{
    const cx<T> r2 = rot90<T, INV>(a[2]), r3 = rot90<T, INV>(a[3]);
    const cx<T> e[4] = {cadd(a[0], a[2]), cadd(a[0], r2), csub(a[0], a[2]), csub(a[0], r2)};
    const cx<T> o[4] = {cadd(a[1], a[3]), cadd(a[1], r3), csub(a[1], a[3]), csub(a[1], r3)};
    dft8_combine<T, INV>(a, e, o);
}

// In-register DFT of length R (forward: exp(-2 pi i/R); inverse: conjugate).
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_small(cx<T> *a, const cx<T> *tw, int N)
{
    if constexpr (R == 2) {
        cx<T> t = a[1];
        a[1] = csub(a[0], t);
        a[0] = cadd(a[0], t);
    } else if constexpr (R == 4) {
        cx<T> s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
        cx<T> s13 = cadd(a[1], a[3]), d13 = rot90<T, INV>(csub(a[1], a[3]));
        a[0] = cadd(s02, s13);
        a[2] = csub(s02, s13);
        a[1] = cadd(d02, d13);
        a[3] = csub(d02, d13);
    } else if constexpr (R == 8) {
        cx<T> e[4] = {a[0], a[2], a[4], a[6]};
        cx<T> o[4] = {a[1], a[3], a[5], a[7]};
        dft_small<T, 4, INV>(e, tw, N);
        dft_small<T, 4, INV>(o, tw, N);
        dft8_combine<T, INV>(a, e, o);
    } else if constexpr (R == 3) {
        // w3 = -1/2 -/+ i sqrt(3)/2:  X1,2 = a0 - (a1 + a2)/2 +/- rot90((sqrt(3)/2)(a1 - a2))
        const T h = (T)0.86602540378443864676372317075293618347;
        const cx<T> t1 = cadd(a[1], a[2]);
        const cx<T> t2 = {a[0].x - (T)0.5 * t1.x, a[0].y - (T)0.5 * t1.y};
        const cx<T> t3 = rot90<T, INV>(cx<T>{h * (a[1].x - a[2].x), h * (a[1].y - a[2].y)});
        a[0] = cadd(a[0], t1);
        a[1] = cadd(t2, t3);
        a[2] = csub(t2, t3);
    } else if constexpr (R == 5) {
        // with b1 = a1 + a4, b2 = a2 + a3, d1 = a1 - a4, d2 = a2 - a3 and
        // c_m = cos(2 pi m/5), s_m = sin(2 pi m/5):
        //   X1,4 = a0 + c1 b1 + c2 b2 +/- rot90(s1 d1 + s2 d2)
        //   X2,3 = a0 + c2 b1 + c1 b2 +/- rot90(s2 d1 - s1 d2)
        const T c1 = (T)0.30901699437494742410229341718281905886, c2 = (T)-0.80901699437494742410229341718281905886;
        const T s1 = (T)0.95105651629515357211643933337938214340, s2 = (T)0.58778525229247312916870595463907276860;
        const cx<T> b1 = cadd(a[1], a[4]), b2 = cadd(a[2], a[3]), d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
        const cx<T> t1 = {a[0].x + c1 * b1.x + c2 * b2.x, a[0].y + c1 * b1.y + c2 * b2.y};
        const cx<T> t2 = {a[0].x + c2 * b1.x + c1 * b2.x, a[0].y + c2 * b1.y + c1 * b2.y};
        const cx<T> u1 = rot90<T, INV>(cx<T>{s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y});
        const cx<T> u2 = rot90<T, INV>(cx<T>{s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y});
        a[0] = cadd(a[0], cadd(b1, b2));
        a[1] = cadd(t1, u1);
        a[4] = csub(t1, u1);
        a[2] = cadd(t2, u2);
        a[3] = csub(t2, u2);
    } else {
        // R = 7: direct sum with table roots of unity w_R^m = w_N^(m N/R)
        cx<T> out[R];
        const int step = N / R;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            cx<T> acc = a[0];
#pragma unroll
            for (int r = 1; r < R; ++r) acc = cadd(acc, cmul(a[r], twid<T, INV>(tw, ((r * q) % R) * step)));
            out[q] = acc;
        }
#pragma unroll
        for (int q = 0; q < R; ++q) a[q] = out[q];
    }
}

// One Stockham stage of radix R (R <= 8) over nseq = 2^lgs sequences of
// length N.  MAXE bounds the complex elements a thread holds
// (nseq * N <= MAXE * NT).
template <typename T, int R, int MAXE, int NT, bool INV>
__device__ __forceinline__ void stage_bfly(T *buf, int rs, int lgs, const FftDesc &fd, int st,
                                           const cx<T> *tw, int tid)
{
    constexpr int BPT = (MAXE + R - 1) / R;
    const int N = fd.N, Ns = fd.ns[st];
    const int NR = N / R;
    const int nbf = (NR << lgs);
    const int tstep = N / (Ns * R);
    const int smask = (1 << lgs) - 1;
    cx<T> v[BPT][R];
    int base[BPT];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int b = tid + i * NT;
        if (b < nbf) {
            const int s = b & smask, j = b >> lgs;
            const int jm = fmod_ns(j, Ns, fd.nsmag[st], fd.nslg[st]);
            base[i] = (j - jm) * R + jm;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = lds_c(buf, rs, j + r * NR, s);
            if (jm != 0) {
                const int e = jm * tstep;
#pragma unroll
                for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], twid<T, INV>(tw, e * r));
            }
            dft_small<T, R, INV>(v[i], tw, N);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int b = tid + i * NT;
        if (b < nbf) {
            const int s = b & smask;
#pragma unroll
            for (int r = 0; r < R; ++r) lds_cs(buf, rs, base[i] + r * Ns, s, v[i][r]);
        }
    }
    __syncthreads();
}

// Stockham stage of arbitrary radix R computed output by output.
template <typename T, int MAXE, int NT, bool INV>
__device__ __forceinline__ void stage_direct(T *buf, int rs, int lgs, const FftDesc &fd, int st,
                                             const cx<T> *tw, int tid)
{
    const int N = fd.N, Ns = fd.ns[st], R = fd.rad[st];
    const int NR = N / R;
    const int tot = N << lgs;
    const int tstep = N / (Ns * R);
    const int smask = (1 << lgs) - 1;
    cx<T> out[MAXE];
#pragma unroll
    for (int i = 0; i < MAXE; ++i) {
        const int e = tid + i * NT;
        if (e < tot) {
            const int s = e & smask, o = e >> lgs;
            const int jm = fmod_ns(o, Ns, fd.nsmag[st], fd.nslg[st]);
            const int t = (o - jm) / Ns, q = t % R, jh = t / R;
            const int j = jh * Ns + jm;
            const int E = jm * tstep + q * NR; // exponent per input index r, in units of w_N
            cx<T> acc = lds_c(buf, rs, j, s);
            int ex = 0;
            for (int r = 1; r < R; ++r) {
                ex += E;
                if (ex >= N) ex -= N;
                acc = cadd(acc, cmul(lds_c(buf, rs, j + r * NR, s), twid<T, INV>(tw, ex)));
            }
            out[i] = acc;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXE; ++i) {
        const int e = tid + i * NT;
        if (e < tot) lds_cs(buf, rs, e >> lgs, e & smask, out[i]);
    }
    __syncthreads();
}

// Stockham stage with every size known at compile time: transform length
// N, radix R, product of the earlier radices NS (a power of two), row pitch
// RS and 2^LGS sequences.  Same data movement as stage_bfly; the index and
// twiddle arithmetic folds to shifts and constants.
// Z: the inputs of rows N/2..N-1 are zero (first stage, radix 8, of a
// zero-padded sequence): they are not loaded, and the butterfly skips them.
template <typename T, int R, int NT, int N, int NS, int RS, int LGS, bool INV, bool Z = false>
__device__ __forceinline__ void stage_ct(T *buf, const cx<T> *tw, int tid)
{
    static_assert(!Z || (R == 8 && NS == 1), "the zero upper half applies to a first radix-8 stage");
    constexpr int NR = N / R, NBF = NR << LGS, TSTEP = N / (NS * R), SMASK = (1 << LGS) - 1;
    constexpr int BPT = (NBF + NT - 1) / NT;
    cx<T> v[BPT][R];
    int base[BPT];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int b = tid + i * NT;
        if (NBF % NT == 0 || b < NBF) {
            const int sq = b & SMASK, j = b >> LGS;
            const int jm = j & (NS - 1);
            base[i] = (j - jm) * R + jm;
            if constexpr (Z) {
#pragma unroll
                for (int r = 0; r < R / 2; ++r) v[i][r] = lds_c(buf, RS, j + r * NR, sq);
                dft8_lower<T, INV>(v[i]);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) v[i][r] = lds_c(buf, RS, j + r * NR, sq);
                if (NS > 1 && jm != 0) {
                    const int e = jm * TSTEP;
#pragma unroll
                    for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], twid<T, INV>(tw, e * r));
                }
                dft_small<T, R, INV>(v[i], tw, N);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int b = tid + i * NT;
        if (NBF % NT == 0 || b < NBF) {
            const int sq = b & SMASK;
#pragma unroll
            for (int r = 0; r < R; ++r) lds_cs(buf, RS, base[i] + r * NS, sq, v[i][r]);
        }
    }
    __syncthreads();
}

// Compile-time transforms for the common power-of-two lengths at the
// default tile widths (radix-8 stages first, as factor_fft orders them).
// tid: the thread index (a caller that runs several transforms in a loop
// may pass one the compiler cannot see through, so that the per-thread index
// and twiddle values are recomputed for each transform instead of being held
// in registers across the loop).
// Z: the upper half of the inputs is zero (see stage_ct).
template <typename T, int NT, int N, int RS, int LGS, bool INV, bool Z = false>
__device__ __forceinline__ void fft_ct(T *buf, const cx<T> *tw, int tid)
{
    if constexpr (N == 256) {
        stage_ct<T, 8, NT, N, 1, RS, LGS, INV, Z>(buf, tw, tid);
        stage_ct<T, 8, NT, N, 8, RS, LGS, INV>(buf, tw, tid);
        stage_ct<T, 4, NT, N, 64, RS, LGS, INV>(buf, tw, tid);
    } else if constexpr (N == 512) {
        stage_ct<T, 8, NT, N, 1, RS, LGS, INV, Z>(buf, tw, tid);
        stage_ct<T, 8, NT, N, 8, RS, LGS, INV>(buf, tw, tid);
        stage_ct<T, 8, NT, N, 64, RS, LGS, INV>(buf, tw, tid);
    } else if constexpr (N == 1024) {
        stage_ct<T, 8, NT, N, 1, RS, LGS, INV, Z>(buf, tw, tid);
        stage_ct<T, 8, NT, N, 8, RS, LGS, INV>(buf, tw, tid);
        stage_ct<T, 8, NT, N, 64, RS, LGS, INV>(buf, tw, tid);
        stage_ct<T, 2, NT, N, 512, RS, LGS, INV>(buf, tw, tid);
    }
}

// Element offset r * rsd + c * csd of a tile in 32-bit arithmetic with
// 24-bit multiplies: the launchers check that strides stay below 2^23 and a
// tile spans less than 2^31 elements (true for every supported grid).
__device__ __forceinline__ int toff(int r, int64_t rsd, int c, int64_t csd)
{
    return __mul24(r, (int)rsd) + __mul24(c, (int)csd);
}

// The compile-time transforms split for tiles that are read from or written
// to global memory by the transform itself (default (N, pitch) pairs only,
// where every stage holds one butterfly per thread):
//   forward:  stage_ct_gin (first stage, inputs from global) + fft_ct_tail
//   inverse:  fft_ct_head + stage_ct_gout (last stage, outputs to global)
// The tile never holds the input rows or the output rows in LDS, which saves
// one LDS write and one read of the tile, and a barrier, per transform.
template <int N>
struct CtLast {
    static constexpr int R = N == 256 ? 4 : N == 512 ? 8 : 2; // radix of the last stage
};

// Every stage after the first.
template <typename T, int NT, int N, int RS, int LGS, bool INV>
__device__ __forceinline__ void fft_ct_tail(T *buf, const cx<T> *tw, int tid)
{
    if constexpr (N == 256) {
        stage_ct<T, 8, NT, N, 8, RS, LGS, INV>(buf, tw, tid);
        stage_ct<T, 4, NT, N, 64, RS, LGS, INV>(buf, tw, tid);
    } else if constexpr (N == 512) {
        stage_ct<T, 8, NT, N, 8, RS, LGS, INV>(buf, tw, tid);
        stage_ct<T, 8, NT, N, 64, RS, LGS, INV>(buf, tw, tid);
    } else if constexpr (N == 1024) {
        stage_ct<T, 8, NT, N, 8, RS, LGS, INV>(buf, tw, tid);
        stage_ct<T, 8, NT, N, 64, RS, LGS, INV>(buf, tw, tid);
        stage_ct<T, 2, NT, N, 512, RS, LGS, INV>(buf, tw, tid);
    }
}

// Every stage but the last.
template <typename T, int NT, int N, int RS, int LGS, bool INV>
__device__ __forceinline__ void fft_ct_head(T *buf, const cx<T> *tw, int tid)
{
    stage_ct<T, 8, NT, N, 1, RS, LGS, INV>(buf, tw, tid);
    stage_ct<T, 8, NT, N, 8, RS, LGS, INV>(buf, tw, tid);
    if constexpr (N == 1024) stage_ct<T, 8, NT, N, 64, RS, LGS, INV>(buf, tw, tid);
}

// The inputs of the first forward stage (radix 8) of thread tid, for
// zero-padded sequences read from global memory: v[2r] and v[2r+1] are
// tile row t = j + r N/8 (r < 4) of sequence sq (j = tid >> LGS, sq = its low
// bits), i.e. source row t - 1 of columns 2 sq and 2 sq + 1; row 0, rows past
// nrows (nrows < N/2) and columns >= ncols are zero.  Element (r, c) is
// src[r*rsd + c*csd].  A loop over tiles can hold v while it transforms the
// previous tile.
template <typename TI, int NT, int N, int LGS>
__device__ __forceinline__ void fetch_gin(TI (&v)[8], const TI *src, int nrows, int ncols, int64_t rsd, int64_t csd,
                                          int tid)
{
    constexpr int NR = N / 8, SMASK = (1 << LGS) - 1;
    static_assert((NR << LGS) == NT, "one butterfly per thread");
    const int sq = tid & SMASK, j = tid >> LGS, c = 2 * sq;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int t = j + r * NR;
        const bool ok = t >= 1 && t <= nrows;
        const TI *p = src + toff(ok ? t - 1 : 0, rsd, c, csd);
        v[2 * r] = ok && c < ncols ? p[0] : (TI)0;
        v[2 * r + 1] = ok && c + 1 < ncols ? p[csd] : (TI)0;
    }
}

// First forward stage (radix 8, upper half of the inputs zero) from the
// registers fetch_gin filled; writes every row of the tile.  Ends with a
// barrier.
template <typename T, typename TI, int NT, int N, int RS, int LGS>
__device__ __forceinline__ void stage_ct_rin(T *buf, const TI (&v)[8], int tid)
{
    constexpr int SMASK = (1 << LGS) - 1;
    const int sq = tid & SMASK, j = tid >> LGS;
    cx<T> a[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = cx<T>{(T)v[2 * r], (T)v[2 * r + 1]};
    dft8_lower<T, false>(a);
#pragma unroll
    for (int r = 0; r < 8; ++r) lds_cs(buf, RS, 8 * j + r, sq, a[r]);
    __syncthreads();
}

// The first forward stage straight from global memory (fetch_gin, then
// stage_ct_rin).
template <typename T, typename TI, int NT, int N, int RS, int LGS>
__device__ __forceinline__ void stage_ct_gin(T *buf, const TI *src, int nrows, int ncols, int64_t rsd,
                                             int64_t csd, int tid)
{
    TI v[8];
    fetch_gin<TI, NT, N, LGS>(v, src, nrows, ncols, rsd, csd, tid);
    stage_ct_rin<T, TI, NT, N, RS, LGS>(buf, v, tid);
}

// Last stage (radix CtLast<N>::R) of the inverse transform, written straight
// to global memory: only output rows t < N/2 are formed (the sine synthesis
// of an odd-symmetric spectrum needs no more; the caller checks that the rows
// it keeps lie below N/2), and rows t = row0..row0+nrows-1 of sequence sq go,
// scaled, to row t - row0 of columns 2 sq and 2 sq + 1 of dst (columns >=
// ncols are skipped).  Element (r, c) is dst[r*rsd + c*csd].
template <typename T, typename TO, int NT, int N, int RS, int LGS>
__device__ __forceinline__ void stage_ct_gout(const T *buf, const cx<T> *tw, TO *dst, int row0, int nrows,
                                              int ncols, int64_t rsd, int64_t csd, T scale, int tid)
{
    constexpr int R = CtLast<N>::R, NR = N / R, NBF = NR << LGS, SMASK = (1 << LGS) - 1;
    static_assert(NBF % NT == 0, "whole butterflies per thread");
#pragma unroll
    for (int i = 0; i < NBF / NT; ++i) {
        const int b = tid + i * NT;
        const int sq = b & SMASK, j = b >> LGS, c = 2 * sq;
        cx<T> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = lds_c(buf, RS, j + r * NR, sq);
        if (j != 0) {
#pragma unroll
            for (int r = 1; r < R; ++r) v[r] = cmul(v[r], twid<T, true>(tw, j * r));
        }
        dft_small<T, R, true>(v, tw, N);
#pragma unroll
        for (int r = 0; r < R / 2; ++r) {
            const int t = j + r * NR - row0;
            if (t >= 0 && t < nrows) {
                TO *p = dst + toff(t, rsd, c, csd);
                if (c < ncols) p[0] = (TO)(scale * v[r].x);
                if (c + 1 < ncols) p[csd] = (TO)(scale * v[r].y);
            }
        }
    }
}

// Full length-N complex FFT of 2^lgs sequences held in LDS (in place), in the
// direction INV (false: exp(-2 pi i t/N), true: the conjugate).
// P2: N is a power of two (only radix-2/4/8 stages are compiled in).
// CT = false keeps the generic stages only.  tid: see fft_ct.
// Z: the upper half of the inputs is zero; the compile-time transforms skip
// it in their first stage, the generic ones read the zeros.
template <typename T, int MAXE, int NT, bool P2, bool CT, bool INV, bool Z = false>
__device__ __forceinline__ void fft_tile_dir(T *buf, int rs, int lgs, const FftDesc &fd, const cx<T> *tw, int tid)
{
    if constexpr (P2 && CT && NT == 256) {
        // (N, tile width) pairs of the default tile budget: N * W / 2 = MAXE * NT
        if constexpr (MAXE == 8) {
            if (fd.N == 512 && rs == 9) return fft_ct<T, NT, 512, 9, 2, INV, Z>(buf, tw, tid);
            if (fd.N == 256 && rs == 17) return fft_ct<T, NT, 256, 17, 3, INV, Z>(buf, tw, tid);
            if (fd.N == 1024 && rs == 5) return fft_ct<T, NT, 1024, 5, 1, INV, Z>(buf, tw, tid);
        }
    }
    if constexpr (P2) {
        for (int st = 0; st < fd.nst; ++st) {
            const int R = fd.rad[st];
            if (R == 8)
                stage_bfly<T, 8, MAXE, NT, INV>(buf, rs, lgs, fd, st, tw, tid);
            else if (R == 4)
                stage_bfly<T, 4, MAXE, NT, INV>(buf, rs, lgs, fd, st, tw, tid);
            else
                stage_bfly<T, 2, MAXE, NT, INV>(buf, rs, lgs, fd, st, tw, tid);
        }
        return;
    }
    for (int st = 0; st < fd.nst; ++st) {
        switch (fd.rad[st]) {
        case 2: stage_bfly<T, 2, MAXE, NT, INV>(buf, rs, lgs, fd, st, tw, tid); break;
        case 3: stage_bfly<T, 3, MAXE, NT, INV>(buf, rs, lgs, fd, st, tw, tid); break;
        case 4: stage_bfly<T, 4, MAXE, NT, INV>(buf, rs, lgs, fd, st, tw, tid); break;
        case 5: stage_bfly<T, 5, MAXE, NT, INV>(buf, rs, lgs, fd, st, tw, tid); break;
        case 8: stage_bfly<T, 8, MAXE, NT, INV>(buf, rs, lgs, fd, st, tw, tid); break;
        default: stage_direct<T, MAXE, NT, INV>(buf, rs, lgs, fd, st, tw, tid); break;
        }
    }
}

// fft_tile_dir with the direction as an argument (a constant argument folds
// to one instantiation).  tid: see fft_ct (-1: threadIdx.x).
template <typename T, int MAXE, int NT, bool P2 = false, bool CT = true>
__device__ __forceinline__ void fft_tile(T *buf, int rs, int lgs, const FftDesc &fd, const cx<T> *tw, bool inv,
                                         int tid = -1)
{
    if (tid < 0) tid = threadIdx.x;
    if (inv)
        fft_tile_dir<T, MAXE, NT, P2, CT, true>(buf, rs, lgs, fd, tw, tid);
    else
        fft_tile_dir<T, MAXE, NT, P2, CT, false>(buf, rs, lgs, fd, tw, tid);
}

// Forward transform of zero-padded sequences: rows N/2..N-1 of the tile must
// hold zeros (the generic stages read them); tid: see fft_ct.
template <typename T, int MAXE, int NT, bool P2 = false, bool CT = true>
__device__ __forceinline__ void fft_tile_zpad(T *buf, int rs, int lgs, const FftDesc &fd, const cx<T> *tw,
                                              int tid = -1)
{
    if (tid < 0) tid = threadIdx.x;
    fft_tile_dir<T, MAXE, NT, P2, CT, false, true>(buf, rs, lgs, fd, tw, tid);
}

// After a forward zero-padded FFT: write C and S in slot layout (in place).
template <typename T, int MAXE, int NT>
__device__ __forceinline__ void post_cs(T *buf, int rs, int lgs, int M, int tid = -1)
{
    if (tid < 0) tid = threadIdx.x;
    constexpr int PPT = MAXE / 2 + 1;
    const int N = 2 * M;
    const int tot = (M + 1) << lgs;
    const int smask = (1 << lgs) - 1;
    T ca[PPT], cb[PPT], sa[PPT], sb[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int e = tid + i * NT;
        if (e < tot) {
            const int s = e & smask, k = e >> lgs;
            const cx<T> z1 = lds_c(buf, rs, k, s);
            const cx<T> z2 = lds_c(buf, rs, k == 0 ? 0 : N - k, s);
            ca[i] = (T)0.5 * (z1.x + z2.x);
            cb[i] = (T)0.5 * (z1.y + z2.y);
            sa[i] = (T)0.5 * (z2.y - z1.y);
            sb[i] = (T)0.5 * (z1.x - z2.x);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int e = tid + i * NT;
        if (e < tot) {
            const int s = e & smask, k = e >> lgs;
            buf[k * rs + 2 * s] = ca[i];
            buf[k * rs + 2 * s + 1] = cb[i];
            if (k >= 1 && k < M) {
                buf[(M + k) * rs + 2 * s] = sa[i];
                buf[(M + k) * rs + 2 * s + 1] = sb[i];
            }
        }
    }
    __syncthreads();
}

// Before an inverse FFT: slots (C, S) -> hermitian-packed complex sequences.
template <typename T, int MAXE, int NT>
__device__ __forceinline__ void pre_herm(T *buf, int rs, int lgs, int M, bool c_zero, int tid = -1)
{
    if (tid < 0) tid = threadIdx.x;
    constexpr int PPT = MAXE / 2 + 1;
    const int N = 2 * M;
    const int tot = (M + 1) << lgs;
    const int smask = (1 << lgs) - 1;
    cx<T> z1[PPT], z2[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int e = tid + i * NT;
        if (e < tot) {
            const int s = e & smask, k = e >> lgs;
            T ca = 0, cb = 0, sa = 0, sb = 0;
            if (!c_zero) {
                ca = buf[k * rs + 2 * s];
                cb = buf[k * rs + 2 * s + 1];
            }
            if (k >= 1 && k < M) {
                sa = buf[(M + k) * rs + 2 * s];
                sb = buf[(M + k) * rs + 2 * s + 1];
            }
            z1[i] = {ca + sb, cb - sa};
            z2[i] = {ca - sb, cb + sa};
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int e = tid + i * NT;
        if (e < tot) {
            const int s = e & smask, k = e >> lgs;
            lds_cs(buf, rs, k, s, z1[i]);
            if (k >= 1 && k < M) lds_cs(buf, rs, N - k, s, z2[i]);
        }
    }
    __syncthreads();
}

// Even extension: rows 1..M-1 copied to rows N-1..M+1.
template <typename T, int NT>
__device__ __forceinline__ void pre_even(T *buf, int rs, int lgW, int M, int tid = -1)
{
    if (tid < 0) tid = threadIdx.x;
    const int N = 2 * M;
    const int tot = (M - 1) << lgW;
    for (int e = tid; e < tot; e += NT) {
        const int c = e & ((1 << lgW) - 1), j = 1 + (e >> lgW);
        buf[(N - j) * rs + c] = buf[j * rs + c];
    }
    __syncthreads();
}

template <typename T, int NT>
__device__ __forceinline__ void zero_rows(T *buf, int rs, int lgW, int r0, int r1, int tid = -1)
{
    if (tid < 0) tid = threadIdx.x;
    const int tot = (r1 - r0) << lgW;
    const int cm = (1 << lgW) - 1;
    for (int e = tid; e < tot; e += NT) buf[(r0 + (e >> lgW)) * rs + (e & cm)] = (T)0;
}

template <typename T, int NT>
__device__ __forceinline__ void load_twiddles(cx<T> *dst, const cx<double> *src, int N)
{
    for (int t = threadIdx.x; t < N; t += NT) {
        cx<double> w = src[t];
        dst[t] = {(T)w.x, (T)w.y};
    }
}

// Global -> LDS: rows [0, nrows) x cols [0, W = 2^lgW) of the tile land at
// LDS rows row0.. ; columns >= ncols are zero.  Element (r, c) is
// src[r*rsd + c*csd].  Rows-contiguous sources are read one column per wave.
template <typename T, typename TI, int NT>
__device__ __forceinline__ void tile_load(T *buf, int rs, int row0, const TI *src, int nrows, int ncols,
                                          int64_t rsd, int64_t csd, int lgW, int tid = -1)
{
    if (tid < 0) tid = threadIdx.x;
    const int W = 1 << lgW;
    if (rsd == 1 && csd != 1) {
        const int lane = tid & 63, wave = tid >> 6;
        for (int c = wave; c < W; c += NT / 64) {
            if (c < ncols) {
                const TI *col = src + c * csd;
                for (int r = lane; r < nrows; r += 64) buf[(row0 + r) * rs + c] = (T)col[r];
            } else {
                for (int r = lane; r < nrows; r += 64) buf[(row0 + r) * rs + c] = (T)0;
            }
        }
    } else {
        const int cm = W - 1;
        const int tot = nrows << lgW;
        for (int e = tid; e < tot; e += NT) {
            const int c = e & cm, r = e >> lgW;
            T v = (T)0;
            if (c < ncols) v = (T)src[toff(r, rsd, c, csd)];
            buf[(row0 + r) * rs + c] = v;
        }
    }
}

// Global -> LDS for a tile of two column sets: tile column j < W/2 holds
// source column cA + j (if j < nA), tile column W/2 + j holds source column
// cB - j (if j < nB); every other column is zero.  Element (r, col) is
// src[r*rsd + col*csd].  Rows-contiguous sources are read by whole waves per
// column (several waves per column when the tile has fewer columns than the
// block has waves).
template <typename T, typename TI, int NT>
__device__ void tile_load_pair(T *buf, int rs, int row0, const TI *src, int nrows, int64_t rsd, int64_t csd,
                               int lgW, int cA, int nA, int cB, int nB, int tid = -1)
{
    if (tid < 0) tid = threadIdx.x;
    const int W = 1 << lgW, Wh = W >> 1;
    auto src_col = [&](int c) -> int {
        const int j = c < Wh ? c : c - Wh;
        return c < Wh ? (j < nA ? cA + j : -1) : (j < nB ? cB - j : -1);
    };
    if (rsd == 1 && csd != 1) {
        constexpr int NW = NT / 64;
        const int lane = tid & 63, wave = tid >> 6;
        const int cstep = NW < W ? NW : W;
        const int rstep = (NW / cstep) * 64;
        const int rbeg = (wave / cstep) * 64 + lane;
        for (int c = wave % cstep; c < W; c += cstep) {
            const int sc = src_col(c);
            T *dst = buf + row0 * rs + c;
            if (sc >= 0) {
                const TI *col = src + sc * csd;
                for (int r = rbeg; r < nrows; r += rstep) dst[r * rs] = (T)col[r];
            } else {
                for (int r = rbeg; r < nrows; r += rstep) dst[r * rs] = (T)0;
            }
        }
        return;
    }
    const int cm = W - 1;
    const int tot = nrows << lgW;
    for (int e = tid; e < tot; e += NT) {
        const int c = e & cm, r = e >> lgW;
        const int sc = src_col(c);
        T v = (T)0;
        if (sc >= 0) v = (T)src[toff(r, rsd, sc, csd)];
        buf[(row0 + r) * rs + c] = v;
    }
}

// The element mapping of tile_load_pair for a compile-time width WC, split
// in two halves so that a loop over tiles can fetch the next tile into
// registers (fetch_pair) while it transforms the current one, and write them
// to LDS afterwards (put_pair).  Each thread holds EPT elements; covers()
// tells whether that is enough for nrows rows.
template <int NT, int WC, int EPT>
struct PairMap {
    static constexpr int NW = NT / 64;
    static constexpr int CSTEP = NW < WC ? NW : WC;  // rows-contiguous: columns per sweep of the waves
    static constexpr int CPT = WC / CSTEP;           // columns per thread
    static constexpr int RB = EPT / CPT;             // rows per column per thread
    static constexpr int RSTEP = (NW / CSTEP) * 64;
    __host__ __device__ static bool covers(int nrows, bool rows_contiguous)
    {
        return rows_contiguous ? RB * RSTEP >= nrows : EPT * NT >= nrows * WC;
    }
};

template <int WC>
__device__ __forceinline__ int pair_src_col(int c, int cA, int nA, int cB, int nB)
{
    constexpr int Wh = WC / 2;
    const int j = c < Wh ? c : c - Wh;
    return c < Wh ? (j < nA ? cA + j : -1) : (j < nB ? cB - j : -1);
}

// MIR = false: plain tile, tile column c holds source column cA + c (c < nA).
template <typename TI, int NT, int WC, int EPT, bool MIR = true>
__device__ __forceinline__ void fetch_pair(TI (&v)[EPT], const TI *src, int nrows, int64_t rsd, int64_t csd,
                                           int cA, int nA, int cB, int nB, int tid)
{
    auto src_col = [&](int c) {
        if constexpr (MIR)
            return pair_src_col<WC>(c, cA, nA, cB, nB);
        else
            return c < nA ? cA + c : -1;
    };
    using PM = PairMap<NT, WC, EPT>;
    if (rsd == 1 && csd != 1) {
        const int lane = tid & 63, wave = tid >> 6;
        const int rbeg = (wave / PM::CSTEP) * 64 + lane;
#pragma unroll
        for (int kc = 0; kc < PM::CPT; ++kc) {
            const int sc = src_col(wave % PM::CSTEP + kc * PM::CSTEP);
            const TI *col = src + (int64_t)(sc < 0 ? 0 : sc) * csd;
#pragma unroll
            for (int kr = 0; kr < PM::RB; ++kr) {
                const int r = rbeg + kr * PM::RSTEP;
                v[kc * PM::RB + kr] = (sc >= 0 && r < nrows) ? col[r] : (TI)0;
            }
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int e = tid + k * NT;
        const int c = e & (WC - 1), r = e / WC;
        const int sc = src_col(c);
        v[k] = (sc >= 0 && r < nrows) ? src[toff(r, rsd, sc, csd)] : (TI)0;
    }
}

template <typename T, typename TI, int NT, int WC, int EPT>
__device__ __forceinline__ void put_pair(T *buf, int rs, int row0, const TI (&v)[EPT], int nrows, bool rows_contiguous,
                                         int tid)
{
    using PM = PairMap<NT, WC, EPT>;
    if (rows_contiguous) {
        const int lane = tid & 63, wave = tid >> 6;
        const int rbeg = (wave / PM::CSTEP) * 64 + lane;
#pragma unroll
        for (int kc = 0; kc < PM::CPT; ++kc) {
            const int c = wave % PM::CSTEP + kc * PM::CSTEP;
#pragma unroll
            for (int kr = 0; kr < PM::RB; ++kr) {
                const int r = rbeg + kr * PM::RSTEP;
                if (r < nrows) buf[(row0 + r) * rs + c] = (T)v[kc * PM::RB + kr];
            }
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int e = tid + k * NT;
        const int c = e & (WC - 1), r = e / WC;
        if (r < nrows) buf[(row0 + r) * rs + c] = (T)v[k];
    }
}

// q[0] + q[s] + ... + q[(n-1) s] with four independent partial sums, so that
// four loads are in flight at a time: ((a0 + a1) + (a2 + a3)).
template <typename T, typename TI>
__device__ __forceinline__ T sum_strided(const TI *q, int n, int64_t s)
{
    T a0 = (T)0, a1 = (T)0, a2 = (T)0, a3 = (T)0;
    int k = 0;
    for (; k + 4 <= n; k += 4) {
        a0 += (T)q[k * s];
        a1 += (T)q[(k + 1) * s];
        a2 += (T)q[(k + 2) * s];
        a3 += (T)q[(k + 3) * s];
    }
    for (; k < n; ++k) a0 += (T)q[k * s];
    return (a0 + a1) + (a2 + a3);
}

// As tile_load (columns contiguous or generic), but every element is the sum
// of nsum copies spaced sstride apart (summing partial results on the fly).
template <typename T, typename TI, int NT>
__device__ __forceinline__ void tile_load_sum(T *buf, int rs, int row0, const TI *src, int nrows, int ncols,
                                              int64_t rsd, int64_t csd, int lgW, int nsum, int64_t sstride,
                                              int tid = -1)
{
    if (tid < 0) tid = threadIdx.x;
    const int W = 1 << lgW;
    if (rsd == 1 && csd != 1) {
        const int lane = tid & 63, wave = tid >> 6;
        for (int c = wave; c < W; c += NT / 64) {
            for (int r = lane; r < nrows; r += 64) {
                T v = (T)0;
                if (c < ncols) v = sum_strided<T>(src + c * csd + r, nsum, sstride);
                buf[(row0 + r) * rs + c] = v;
            }
        }
        return;
    }
    const int cm = W - 1;
    const int tot = nrows << lgW;
    for (int e = tid; e < tot; e += NT) {
        const int c = e & cm, r = e >> lgW;
        T v = (T)0;
        if (c < ncols) v = sum_strided<T>(src + toff(r, rsd, c, csd), nsum, sstride);
        buf[(row0 + r) * rs + c] = v;
    }
}

// LDS -> global: LDS rows row0..row0+nrows-1, cols [0, ncols) go to
// dst[r*rsd + c*csd] scaled by `scale`.
template <typename T, typename TO, int NT>
__device__ __forceinline__ void tile_store(const T *buf, int rs, int row0, TO *dst, int nrows, int ncols,
                                           int64_t rsd, int64_t csd, T scale, int lgW, int tid = -1)
{
    if (tid < 0) tid = threadIdx.x;
    if (rsd == 1 && csd != 1) {
        const int lane = tid & 63, wave = tid >> 6;
        for (int c = wave; c < ncols; c += NT / 64) {
            TO *col = dst + c * csd;
            for (int r = lane; r < nrows; r += 64) col[r] = (TO)(scale * buf[(row0 + r) * rs + c]);
        }
    } else {
        const int cm = (1 << lgW) - 1;
        const int tot = nrows << lgW;
        for (int e = tid; e < tot; e += NT) {
            const int c = e & cm, r = e >> lgW;
            if (c < ncols) dst[toff(r, rsd, c, csd)] = (TO)(scale * buf[(row0 + r) * rs + c]);
        }
    }
}

// As tile_store, but the scaled values are added to the destination.
template <typename T, typename TO, int NT>
__device__ __forceinline__ void tile_store_acc(const T *buf, int rs, int row0, TO *dst, int nrows, int ncols,
                                               int64_t rsd, int64_t csd, T scale, int lgW, int tid = -1)
{
    if (tid < 0) tid = threadIdx.x;
    if (rsd == 1 && csd != 1) {
        const int lane = tid & 63, wave = tid >> 6;
        for (int c = wave; c < ncols; c += NT / 64) {
            TO *col = dst + c * csd;
            for (int r = lane; r < nrows; r += 64) col[r] += (TO)(scale * buf[(row0 + r) * rs + c]);
        }
    } else {
        const int cm = (1 << lgW) - 1;
        const int tot = nrows << lgW;
        for (int e = tid; e < tot; e += NT) {
            const int c = e & cm, r = e >> lgW;
            if (c < ncols) dst[toff(r, rsd, c, csd)] += (TO)(scale * buf[(row0 + r) * rs + c]);
        }
    }
}

// Blocks are dealt to the 8 XCDs round-robin; remap so that each XCD works on
// one contiguous range of logical tiles (neighbouring tiles share its L2).
__device__ __forceinline__ int xcd_remap(int bid, int nblocks)
{
    constexpr int kXcd = 8;
    if (nblocks < kXcd || nblocks % kXcd != 0) return bid;
    return (bid % kXcd) * (nblocks / kXcd) + bid / kXcd;
}

} // namespace ips
