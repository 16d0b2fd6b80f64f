// Boundary convolution kernel of the infinite-domain Poisson solver (gfx950):
// boundary values as sums over slices of 2D (3D problems) or 1D (2D problems)
// discrete convolutions, accumulated in Fourier space with the kernel spectra
// (Section 4, eqs. Trap2D, Trap2Dconvolution, convolution).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace ips {

// ---------------------------------------------------------------------------
// Boundary convolution, contraction over the tile columns (3D and 2D)
// ---------------------------------------------------------------------------
// Columns c and ncols-1-c lie at mirrored distances from the two faces: the
// kernel spectrum that weights column c for face 0 weights column ncols-1-c
// for face M, and the other way round.  A tile therefore holds W/2 columns
// c0.. of the first half and their mirrors ncols-1-c0.. (the middle column of
// an odd count only once), so each kernel-spectrum value loaded serves two
// columns, and with the C and S rows of the pencil transform four products
// per face.
template <typename T, typename TI, int MAXE, bool WB, bool P2, int RPT, int NTT, int WHC, int NC>
__global__ __launch_bounds__(NTT) void k_cc(CcArgs a, int nchunk)
{
    constexpr bool BIG = NTT != NT;
    extern __shared__ __align__(16) unsigned char smem[];
    // NC > 0: the transform length, known at compile time (only the
    // compile-time Stockham stages of that length are built in)
    // (only the pairs that have compile-time stages: fdc carries no stage list)
    static_assert(NC == 0 || (P2 && MAXE == 8 && NTT == NT && NC * WHC == 8 * NT), "no compile-time stages");
    FftDesc fdc{};
    if constexpr (NC > 0) {
        fdc.N = NC;
        fdc.M = NC / 2;
    }
    const FftDesc &fd = NC > 0 ? fdc : a.fd;
    // the prefetching variants run one tile width only (their launcher checks it)
    const int N = fd.N, M = fd.M, W = WHC > 0 ? 2 * WHC : a.W, rs = BIG ? W : W + 1;
    const int lgW = 31 - __clz(W), lgs = lgW - 1, Wh = W >> 1;
    const cx<T> *tw = tw_table<T, BIG>(smem, a.tw, a.twf);
    T *buf = reinterpret_cast<T *>(smem + (BIG ? 0 : (size_t)N * sizeof(cx<T>)));
    // Logical order: for each wavenumber k_b of the other axis, its cos slot
    // and its sin slot are neighbours, so the blocks reading the same kernel
    // spectra K[.][k_b][.] run together on one XCD (shared L2).
    const int lb = xcd_remap(blockIdx.x, nchunk * a.nbatch);
    const int ch = lb % nchunk, q = lb / nchunk;
    int bt = q;
    if (a.Mo > 0) {
        // q = 0 -> slot 0; q = 2kb-1 -> slot kb; q = 2kb -> slot Mo+kb (kb < Mo); q = 2Mo-1 -> slot Mo
        if (q == 0)
            bt = 0;
        else if (q == 2 * a.Mo - 1)
            bt = a.Mo;
        else
            bt = (q & 1) ? (q + 1) / 2 : a.Mo + q / 2;
    }
    const int kb = a.Mo > 0 ? (bt <= a.Mo ? bt : bt - a.Mo) : 0;
    const TI *in = static_cast<const TI *>(a.in) + bt * a.ibs;
    T *Bout = static_cast<T *>(a.Bout);
    // Slot rows per thread: t = threadIdx.x + i NTT < M, i < TPT, owns rows t
    // and M + t, i.e. C_t and S_t (which share the kernel spectrum value) for
    // t >= 1, and C_0 and C_M for t = 0.
    constexpr int TPT = RPT / 2;
    double a10[TPT], a11[TPT], a20[TPT], a21[TPT]; // [row 1|2][face 0|M]
#pragma unroll
    for (int i = 0; i < TPT; ++i) a10[i] = a11[i] = a20[i] = a21[i] = 0.0;
    if (!BIG) load_twiddles<T, NTT>(reinterpret_cast<cx<T> *>(smem), a.tw, N);
    const int hc = (a.ncols + 1) >> 1; // first-half columns (the chunked range)
    // tiles of this chunk: a contiguous run of columns, or (interleaved) every
    // nchunk-th tile, so that the blocks of one batch entry, which run side by
    // side, read neighbouring columns at the same time (strided pencils share
    // their cache lines across those blocks instead of re-fetching them)
    const int cbeg = a.interleave ? ch * Wh : ch * a.cols_per_chunk;
    const int cend = a.interleave ? hc : min(hc, cbeg + a.cols_per_chunk);
    const int cstep = a.interleave ? nchunk * Wh : Wh;
    // PF (compile-time width): the next tile is fetched into registers while
    // the current one is transformed and contracted
    constexpr bool PF = WHC > 0;
    constexpr int WCF = PF ? 2 * WHC : 2;
    const bool rcont = a.irs == 1 && a.ics != 1;
    auto n_a = [&](int c) { return min(Wh, cend - c); };
    auto n_b = [&](int c) { return min(n_a(c), max(0, (a.ncols - 2 * c) >> 1)); };
    TI pf[MAXE];
    if constexpr (PF)
        if (cbeg < cend)
            fetch_pair<TI, NTT, WCF, MAXE>(pf, in, a.nrows_in, a.irs, a.ics, cbeg, n_a(cbeg), a.ncols - 1 - cbeg,
                                          n_b(cbeg), threadIdx.x);
    for (int c0 = cbeg; c0 < cend; c0 += cstep) {
        const int nA = n_a(c0);
        const int m0 = a.ncols - 1 - c0; // mirror of c0
        const int nB = n_b(c0);          // mirrors distinct from their column
        // the thread index, opaque to the compiler: per-thread index and
        // twiddle values are recomputed for each tile rather than held in
        // registers across the loop
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        tid &= NTT - 1; // the range (known bits) of the thread index
        zero_rows<T, NTT>(buf, rs, lgW, 0, 1, tid);
        zero_rows<T, NTT>(buf, rs, lgW, 1 + a.nrows_in, N, tid);
        if constexpr (PF) {
            put_pair<T, TI, NTT, WCF, MAXE>(buf, rs, 1, pf, a.nrows_in, rcont, tid);
            const int c1 = c0 + cstep;
            if (c1 < cend)
                fetch_pair<TI, NTT, WCF, MAXE>(pf, in, a.nrows_in, a.irs, a.ics, c1, n_a(c1), a.ncols - 1 - c1,
                                              n_b(c1), tid);
        } else {
            tile_load_pair<T, TI, NTT>(buf, rs, 1, in, a.nrows_in, a.irs, a.ics, lgW, c0, nA, m0, nB, tid);
        }
        __syncthreads();
        // rows 1..nrows_in <= M-1 hold data, rows from M on are zero
        if (a.nrows_in <= M - 1)
            fft_tile_zpad<T, MAXE, NTT, P2>(buf, rs, lgs, fd, tw, tid);
        else
            fft_tile<T, MAXE, NTT, P2>(buf, rs, lgs, fd, tw, false, tid);
        post_cs<T, MAXE, NTT>(buf, rs, lgs, M, tid);
        if (WB && (a.Mo == 0 || bt > a.Mo)) {
            const int64_t bb = a.Mo == 0 ? 0 : (int64_t)(bt - a.Mo - 1) * a.Bbs;
            const int lane = tid & 63, wave = tid >> 6;
            for (int c = wave; c < W; c += NTT / 64) {
                const int j = c < Wh ? c : c - Wh;
                const int col = c < Wh ? (j < nA ? c0 + j : -1) : (j < nB ? m0 - j : -1);
                if (col < 0) continue;
                const int64_t cb = (int64_t)col * a.Bcs + bb;
                for (int r = lane; r < M - 1; r += 64) {
                    const T v = buf[(M + 1 + r) * rs + c];
                    if (a.Bf32)
                        static_cast<float *>(a.Bout)[cb + (int64_t)r * a.Brs] = (float)v;
                    else
                        Bout[cb + (int64_t)r * a.Brs] = v;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < TPT; ++i) {
            const int t = tid + i * NTT;
            if (t < M) {
                const bool two = t > 0; // row M + t is S_t (else C_M, see below)
                const T *r1 = buf + t * rs, *r2 = buf + (M + t) * rs;
                // FP64 kernel spectra and FP64 sums in every mode: an FP32 slot
                // value is widened exactly, so the boundary sums accumulate in FP64
                const double *Kr = static_cast<const double *>(a.K) + (int64_t)kb * a.Ko;
                const double *KA = Kr + t + (int64_t)c0 * a.Kd; // K at column c0 + j
                const double *KB = Kr + t + (int64_t)m0 * a.Kd; // K at column m0 - j
                using TA = double;
                TA s10 = a10[i], s11 = a11[i], s20 = a20[i], s21 = a21[i];
                auto col_pair = [&](int j) {
                    const TA kA = KA[(int64_t)j * a.Kd], kB = KB[-(int64_t)j * a.Kd];
                    const TA ud = (TA)r1[j], um = (TA)r1[Wh + j];
                    const TA vd = two ? (TA)r2[j] : (TA)0, vm = two ? (TA)r2[Wh + j] : (TA)0;
                    s10 = fma(kA, ud, s10);
                    s10 = fma(kB, um, s10);
                    s11 = fma(kB, ud, s11);
                    s11 = fma(kA, um, s11);
                    s20 = fma(kA, vd, s20);
                    s20 = fma(kB, vm, s20);
                    s21 = fma(kB, vd, s21);
                    s21 = fma(kA, vm, s21);
                };
                if (WHC > 0 && nA == WHC) {
#pragma unroll
                    for (int j = 0; j < WHC; ++j) col_pair(j);
                } else {
                    for (int j = 0; j < nA; ++j) col_pair(j);
                }
                if (!two) {
                    // C_M (no sine partner) with its own kernel spectrum
                    const double *MA = Kr + M + (int64_t)c0 * a.Kd, *MB = Kr + M + (int64_t)m0 * a.Kd;
                    for (int j = 0; j < nA; ++j) {
                        const TA kA = MA[(int64_t)j * a.Kd], kB = MB[-(int64_t)j * a.Kd];
                        const TA vd = (TA)r2[j], vm = (TA)r2[Wh + j];
                        s20 = fma(kA, vd, s20);
                        s20 = fma(kB, vm, s20);
                        s21 = fma(kB, vd, s21);
                        s21 = fma(kA, vm, s21);
                    }
                }
                a10[i] = s10;
                a11[i] = s11;
                a20[i] = s20;
                a21[i] = s21;
            }
        }
        __syncthreads();
    }
    // FP64 partials [face][chunk][batch][slot]: slot rows t and M + t
    const int64_t o0 = ((int64_t)ch * a.nbatch + bt) * N, o1 = o0 + (int64_t)nchunk * a.nbatch * N;
    double *pp = static_cast<double *>(a.part);
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
        const int t = threadIdx.x + i * NTT;
        if (t < M) {
            pp[o0 + t] = a10[i];
            pp[o1 + t] = a11[i];
            pp[o0 + M + t] = a20[i];
            pp[o1 + M + t] = a21[i];
        }
    }
}

template <typename T, typename TI, int MAXE, bool WB, bool P2, int RPT, int NTT = NT, int WHC = 0, int NC = 0>
static void launch_cc_k(const CcArgs &a, int nchunk, hipStream_t st)
{
    const size_t lds = tile_lds<T>(a.fd.N, a.W);
    set_lds((const void *)&k_cc<T, TI, MAXE, WB, P2, RPT, NTT, WHC, NC>, lds);
    hipLaunchKernelGGL((k_cc<T, TI, MAXE, WB, P2, RPT, NTT, WHC, NC>), dim3(nchunk * a.nbatch), dim3(NTT), lds,
                       st, a, nchunk);
}

// Compile-time widths (W = 16, 8 for 2M = 256, 512; W = 4 for lengths in
// (512, 1024]) get a fully unrolled contraction and the register prefetch of
// the next tile (shorter lengths other than powers of two measured faster
// without, in batches of small uneven boxes).
template <int WHC, int MAXE, int NTT = NT>
static bool prefetch_fits(const CcArgs &a)
{
    return a.W == 2 * WHC && PairMap<NTT, 2 * WHC, MAXE>::covers(a.nrows_in, a.irs == 1 && a.ics != 1);
}

template <typename T, typename TI, int MAXE, bool WB>
static void launch_cc_m(const CcArgs &a, int nchunk, hipStream_t st)
{
    const bool p2 = is_pow2(a.fd.N);
    if constexpr (MAXE == 8) {
        // the default (length, width) pairs with compile-time Stockham stages
        if (a.fd.N == 512 && prefetch_fits<4, 8>(a))
            return launch_cc_k<T, TI, 8, WB, true, 2, NT, 4, 512>(a, nchunk, st);
        if (a.fd.N == 256 && prefetch_fits<8, 8>(a))
            return launch_cc_k<T, TI, 8, WB, true, 2, NT, 8, 256>(a, nchunk, st);
        if (a.fd.N == 1024 && prefetch_fits<2, 8>(a))
            return launch_cc_k<T, TI, 8, WB, true, 4, NT, 2, 1024>(a, nchunk, st);
    }
    if (a.fd.N <= 2 * NT) {
        if (p2 && prefetch_fits<8, MAXE>(a))
            launch_cc_k<T, TI, MAXE, WB, true, 2, NT, 8>(a, nchunk, st);
        else if (p2 && prefetch_fits<4, MAXE>(a))
            launch_cc_k<T, TI, MAXE, WB, true, 2, NT, 4>(a, nchunk, st);
        else if (p2)
            launch_cc_k<T, TI, MAXE, WB, true, 2>(a, nchunk, st);
        else
            launch_cc_k<T, TI, MAXE, WB, false, 2>(a, nchunk, st);
    } else if (a.fd.N <= 4 * NT) {
        if (p2 && prefetch_fits<2, MAXE>(a))
            launch_cc_k<T, TI, MAXE, WB, true, 4, NT, 2>(a, nchunk, st);
        else if (p2)
            launch_cc_k<T, TI, MAXE, WB, true, 4>(a, nchunk, st);
        else if (prefetch_fits<2, MAXE>(a))
            launch_cc_k<T, TI, MAXE, WB, false, 4, NT, 2>(a, nchunk, st);
        else
            launch_cc_k<T, TI, MAXE, WB, false, 4>(a, nchunk, st);
    } else {
        if (p2)
            launch_cc_k<T, TI, MAXE, WB, true, 8>(a, nchunk, st);
        else
            launch_cc_k<T, TI, MAXE, WB, false, 8>(a, nchunk, st);
    }
}

template <typename T, typename TI, bool WB>
static hipError_t launch_cc_t(const CcArgs &a, int nchunk, hipStream_t st)
{
    const int work = (a.W / 2) * a.fd.N;
    if (big_fft(a.fd.N)) {
        // one complex sequence (a column and its mirror) per tile; rows per thread = N / NTB <= 8
        const bool p2 = is_pow2(a.fd.N);
        if (a.W != 2 || a.fd.N > 8 * NTB) return hipErrorInvalidValue;
        if (a.fd.N <= 4 * NTB) {
            if (p2)
                launch_cc_k<T, TI, 4, WB, true, 4, NTB>(a, nchunk, st);
            else
                launch_cc_k<T, TI, 4, WB, false, 4, NTB>(a, nchunk, st);
        } else {
            if (p2)
                launch_cc_k<T, TI, 8, WB, true, 8, NTB>(a, nchunk, st);
            else
                launch_cc_k<T, TI, 8, WB, false, 8, NTB>(a, nchunk, st);
        }
        return hipGetLastError();
    }
    if (work <= 8 * NT)
        launch_cc_m<T, TI, 8, WB>(a, nchunk, st);
    else
        launch_cc_m<T, TI, 16, WB>(a, nchunk, st);
    return hipGetLastError();
}

hipError_t launch_cc(const CcArgs &a, int nchunk, bool f32, bool in_f32, hipStream_t st)
{
    const int work = (a.W / 2) * a.fd.N;
    if (!big_fft(a.fd.N) && (work > 16 * NT || a.fd.N > 8 * NT)) return hipErrorInvalidValue;
    if (a.W < 2 || a.cols_per_chunk < 1) return hipErrorInvalidValue;
    if (!tile_strides_ok(a.nrows_in, a.irs, a.ncols, a.ics)) return hipErrorInvalidValue;
    const bool wb = a.Bout != nullptr;
    if (!f32) {
        if (in_f32) return hipErrorInvalidValue;
        return wb ? launch_cc_t<double, double, true>(a, nchunk, st)
                  : launch_cc_t<double, double, false>(a, nchunk, st);
    }
    if (in_f32) return wb ? launch_cc_t<float, float, true>(a, nchunk, st)
                          : launch_cc_t<float, float, false>(a, nchunk, st);
    return wb ? launch_cc_t<float, double, true>(a, nchunk, st)
              : launch_cc_t<float, double, false>(a, nchunk, st);
}

} // namespace ips
