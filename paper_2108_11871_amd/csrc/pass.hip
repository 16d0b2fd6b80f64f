// Pencil transforms of the infinite-domain Poisson solver (gfx950): DST-I,
// zero-padded cosine/sine, even (DCT-I) and hermitian-synthesis transforms
// along one axis of a strided 2D/3D array (Sections 3, 4, 5).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace ips {

// Tile lb -> (column block cb, batch entry bt).  Column blocks vary fastest,
// except where the output's batch stride is 1: there neighbouring batch
// entries come first, so that the blocks that run side by side (on one XCD)
// write neighbouring words of the same cache lines (a tile row writes its W
// values at the output's column stride).
__device__ __forceinline__ void tile_of(const PassArgs &a, int ncb, int lb, int &cb, int &bt)
{
    if (a.obs == 1 && a.nbatch > 1) {
        bt = lb % a.nbatch;
        cb = lb / a.nbatch;
    } else {
        cb = lb % ncb;
        bt = lb / ncb;
    }
}

// One tile of a pass: tile lb (column block lb % ncb of batch entry lb / ncb),
// loaded into LDS (rows placed as the input mode needs), transformed along its
// rows and stored.  WT > 0: the tile width, known at compile time (equal to
// a.W, which the launcher checks); NC > 0 likewise the transform length (only
// the compile-time Stockham stages of that length are built in).
template <typename T, typename TI, typename TO, int MAXE, bool P2, int NTT, int WT = 0, int NC = 0>
__device__ __forceinline__ void pass_tile(const PassArgs &a, int lb)
{
    constexpr bool BIG = NTT != NT;
    extern __shared__ __align__(16) unsigned char smem[];
    // (only the pairs that have compile-time stages: fdc carries no stage list)
    static_assert(NC == 0 || (P2 && MAXE == 8 && !BIG && NC * WT == 16 * NT), "no compile-time stages");
    FftDesc fdc{};
    if constexpr (NC > 0) {
        fdc.N = NC;
        fdc.M = NC / 2;
    }
    const FftDesc &fd = NC > 0 ? fdc : a.fd;
    const int N = fd.N, M = fd.M, W = WT > 0 ? WT : a.W, rs = BIG ? W : W + 1;
    const int lgW = 31 - __clz(W), lgs = lgW - 1;
    const cx<T> *tw = tw_table<T, BIG>(smem, a.tw, a.twf);
    T *buf = reinterpret_cast<T *>(smem + (BIG ? 0 : (size_t)N * sizeof(cx<T>)));
    const int ncb = (a.ncols + W - 1) / W;
    int cb, bt;
    tile_of(a, ncb, lb, cb, bt);
    const int c0 = cb * W;
    const int nc = min(W, a.ncols - c0);
    const TI *in = static_cast<const TI *>(a.in) + bt * a.ibs + c0 * a.ics;
    TO *out = static_cast<TO *>(a.out) + bt * a.obs + c0 * a.ocs;
    if (!BIG) load_twiddles<T, NTT>(reinterpret_cast<cx<T> *>(smem), a.tw, N);
    bool inv = false;
    if (a.in_mode == IN_ZPAD) {
        zero_rows<T, NTT>(buf, rs, lgW, 0, 1);
        zero_rows<T, NTT>(buf, rs, lgW, 1 + a.nrows_in, N);
        tile_load<T, TI, NTT>(buf, rs, 1, in, a.nrows_in, nc, a.irs, a.ics, lgW);
        __syncthreads();
    } else if (a.in_mode == IN_ZPAD0) {
        zero_rows<T, NTT>(buf, rs, lgW, a.nrows_in, N);
        tile_load<T, TI, NTT>(buf, rs, 0, in, a.nrows_in, nc, a.irs, a.ics, lgW);
        __syncthreads();
    } else if (a.in_mode == IN_EVEN) {
        tile_load<T, TI, NTT>(buf, rs, 0, in, a.nrows_in, nc, a.irs, a.ics, lgW);
        __syncthreads();
        pre_even<T, NTT>(buf, rs, lgW, M);
    } else if (a.in_mode == IN_HERM) {
        if (a.nsum > 1)
            tile_load_sum<T, TI, NTT>(buf, rs, 0, in, a.nrows_in, nc, a.irs, a.ics, lgW, a.nsum,
                                      a.sstride);
        else
            tile_load<T, TI, NTT>(buf, rs, 0, in, a.nrows_in, nc, a.irs, a.ics, lgW);
        __syncthreads();
        pre_herm<T, MAXE, NTT>(buf, rs, lgs, M, false);
        inv = true;
    } else {
        tile_load<T, TI, NTT>(buf, rs, M + 1, in, a.nrows_in, nc, a.irs, a.ics, lgW);
        __syncthreads();
        pre_herm<T, MAXE, NTT>(buf, rs, lgs, M, true);
        inv = true;
    }
    // zero-padded input (rows 1..nrows_in <= M-1, zeros from row M on):
    // the first stage skips the zero half
    if (a.in_mode == IN_ZPAD && a.nrows_in <= M - 1)
        fft_tile_zpad<T, MAXE, NTT, P2>(buf, rs, lgs, fd, tw);
    else
        fft_tile<T, MAXE, NTT, P2>(buf, rs, lgs, fd, tw, inv);
    if (a.in_mode == IN_ZPAD || a.in_mode == IN_ZPAD0) post_cs<T, MAXE, NTT>(buf, rs, lgs, M);
    if (a.accum)
        tile_store_acc<T, TO, NTT>(buf, rs, a.out_r0, out, a.out_nrows, nc, a.ors, a.ocs, (T)a.scale, lgW);
    else
        tile_store<T, TO, NTT>(buf, rs, a.out_r0, out, a.out_nrows, nc, a.ors, a.ocs, (T)a.scale, lgW);
}

// One pencil pass.  A tile is W consecutive columns of one batch entry; it is
// loaded into LDS (rows placed as the input mode needs), transformed along
// its rows and stored.  Generic widths (WC = 0): one tile per block.  With a
// compile-time width WC and EPT fetch registers per thread, the grid holds as
// many blocks as are resident on the device at once, each block walks the
// tiles with the grid size as stride and fetches the next tile into
// registers while the current one is transformed.  The thread index is made
// opaque inside that loop so that the compiler recomputes per-thread index
// values instead of holding them in registers for the whole loop.
template <typename T, typename TI, typename TO, int MAXE, bool P2, int NTT, int WC, int EPT, int NC>
__global__ __launch_bounds__(NTT) void k_pass(PassArgs a, int ntiles)
{
    constexpr bool PF = WC > 0;
    if constexpr (!PF) {
        // one tile per block (WC < 0: of the compile-time width -WC)
        pass_tile<T, TI, TO, MAXE, P2, NTT, (WC < 0 ? -WC : 0), NC>(a, xcd_remap(blockIdx.x, ntiles));
        return;
    }
    constexpr bool BIG = NTT != NT;
    extern __shared__ __align__(16) unsigned char smem[];
    static_assert(!PF || NC == 0 || (P2 && MAXE == 8 && !BIG && NC * WC == 16 * NT), "no compile-time stages");
    FftDesc fdc{};
    if constexpr (NC > 0) {
        fdc.N = NC;
        fdc.M = NC / 2;
    }
    const FftDesc &fd = NC > 0 ? fdc : a.fd;
    const int N = fd.N, M = fd.M, W = PF ? WC : a.W, rs = BIG ? W : W + 1;
    const int lgW = 31 - __clz(W), lgs = lgW - 1;
    const cx<T> *tw = tw_table<T, BIG>(smem, a.tw, a.twf);
    T *buf = reinterpret_cast<T *>(smem + (BIG ? 0 : (size_t)N * sizeof(cx<T>)));
    const int ncb = (a.ncols + W - 1) / W;
    const int grid = gridDim.x;
    const int lb = xcd_remap(blockIdx.x, grid);
    const int mode = a.in_mode;
    // first tile row of the loaded rows
    const int row0 = mode == IN_ZPAD ? 1 : (mode == IN_SPECS ? M + 1 : 0);
    const bool rcont = a.irs == 1 && a.ics != 1;
    const TI *in0 = static_cast<const TI *>(a.in);
    TO *out0 = static_cast<TO *>(a.out);
    auto tile_at = [&](int it, int &c0, int &nc, int64_t &ioff, int64_t &ooff) {
        int cb, bt;
        tile_of(a, ncb, it, cb, bt);
        c0 = cb * W;
        nc = min(W, a.ncols - c0);
        ioff = bt * a.ibs + c0 * a.ics;
        ooff = bt * a.obs + c0 * a.ocs;
    };
    if (!BIG) load_twiddles<T, NTT>(reinterpret_cast<cx<T> *>(smem), a.tw, N);
    TI pf[PF ? EPT : 1];
    if constexpr (PF) {
        if (lb < ntiles) {
            int c0, nc;
            int64_t io, oo;
            tile_at(lb, c0, nc, io, oo);
            fetch_pair<TI, NTT, WC, EPT, false>(pf, in0 + io, a.nrows_in, a.irs, a.ics, 0, nc, 0, 0, threadIdx.x);
        }
    }
    for (int it = lb; it < ntiles; it += grid) {
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        tid &= NTT - 1; // the range (known bits) of the thread index
        int c0, nc;
        int64_t io, oo;
        tile_at(it, c0, nc, io, oo);
        if (mode == IN_ZPAD) {
            zero_rows<T, NTT>(buf, rs, lgW, 0, 1, tid);
            zero_rows<T, NTT>(buf, rs, lgW, 1 + a.nrows_in, N, tid);
        } else if (mode == IN_ZPAD0) {
            zero_rows<T, NTT>(buf, rs, lgW, a.nrows_in, N, tid);
        }
        if constexpr (PF) {
            put_pair<T, TI, NTT, WC, EPT>(buf, rs, row0, pf, a.nrows_in, rcont, tid);
            const int nx = it + grid;
            if (nx < ntiles) {
                int c1, n1;
                int64_t i1, o1;
                tile_at(nx, c1, n1, i1, o1);
                fetch_pair<TI, NTT, WC, EPT, false>(pf, in0 + i1, a.nrows_in, a.irs, a.ics, 0, n1, 0, 0, tid);
            }
        } else {
            if (mode == IN_HERM && a.nsum > 1)
                tile_load_sum<T, TI, NTT>(buf, rs, 0, in0 + io, a.nrows_in, nc, a.irs, a.ics, lgW, a.nsum,
                                          a.sstride, tid);
            else
                tile_load<T, TI, NTT>(buf, rs, row0, in0 + io, a.nrows_in, nc, a.irs, a.ics, lgW, tid);
        }
        __syncthreads();
        bool inv = false;
        if (mode == IN_EVEN) {
            pre_even<T, NTT>(buf, rs, lgW, M, tid);
        } else if (mode == IN_HERM) {
            pre_herm<T, MAXE, NTT>(buf, rs, lgs, M, false, tid);
            inv = true;
        } else if (mode == IN_SPECS) {
            pre_herm<T, MAXE, NTT>(buf, rs, lgs, M, true, tid);
            inv = true;
        }
        if (mode == IN_ZPAD && a.nrows_in <= M - 1)
            fft_tile_zpad<T, MAXE, NTT, P2>(buf, rs, lgs, fd, tw, tid);
        else
            fft_tile<T, MAXE, NTT, P2>(buf, rs, lgs, fd, tw, inv, tid);
        if (mode == IN_ZPAD || mode == IN_ZPAD0) post_cs<T, MAXE, NTT>(buf, rs, lgs, M, tid);
        if (a.accum)
            tile_store_acc<T, TO, NTT>(buf, rs, a.out_r0, out0 + oo, a.out_nrows, nc, a.ors, a.ocs, (T)a.scale, lgW,
                                       tid);
        else
            tile_store<T, TO, NTT>(buf, rs, a.out_r0, out0 + oo, a.out_nrows, nc, a.ors, a.ocs, (T)a.scale, lgW,
                                   tid);
        __syncthreads();
    }
}

template <typename T, typename TI, typename TO, int MAXE, bool P2, int NTT = NT, int WC = 0, int EPT = 0, int NC = 0>
static void launch_pass_k(const PassArgs &a, int ntiles, size_t lds, hipStream_t st)
{
    const void *fn = (const void *)&k_pass<T, TI, TO, MAXE, P2, NTT, WC, EPT, NC>;
    set_lds(fn, lds);
    int grid = ntiles;
    if (WC > 0) {
        const int r = resident_blocks(fn, NTT, lds);
        if (r > 0 && r < ntiles) grid = r;
    }
    hipLaunchKernelGGL((k_pass<T, TI, TO, MAXE, P2, NTT, WC, EPT, NC>), dim3((unsigned)grid), dim3(NTT), lds, st,
                       a, ntiles);
}

// A compile-time width |WC|: the transform length of the default tile budget
// (N |WC| / 2 = 8 NT, lengths 256, 512, 1024) also at compile time when it is
// the plan's.
template <typename T, typename TI, typename TO, int MAXE, bool P2, int WC, int EPT>
static void launch_pass_w(const PassArgs &a, int ntiles, size_t lds, hipStream_t st)
{
    constexpr int AW = WC < 0 ? -WC : WC;
    constexpr int NCT = (MAXE == 8 && P2 && (AW == 4 || AW == 8 || AW == 16)) ? 16 * NT / AW : 0;
    if constexpr (NCT > 0)
        if (a.fd.N == NCT) return launch_pass_k<T, TI, TO, MAXE, P2, NT, WC, EPT, NCT>(a, ntiles, lds, st);
    launch_pass_k<T, TI, TO, MAXE, P2, NT, WC, EPT>(a, ntiles, lds, st);
}

// Compile-time tile widths W = 4, 8, 16 (the default widths of 2M = 1024,
// 512, 256 and of the lengths near them) with plain loads get the register
// prefetch when EPT
// registers per thread cover the loaded rows.  FP32 tiles: only the forward
// zero-padded transforms (EPT = MAXE); for the inverse passes the
// prefetching loop measured slower than one tile per block.
template <int WC, int EPT>
static bool pass_fits(const PassArgs &a)
{
    return a.W == WC && PairMap<NT, WC, EPT>::covers(a.nrows_in, a.irs == 1 && a.ics != 1);
}

template <typename T, typename TI, typename TO, int MAXE, bool P2>
static void launch_pass_m(const PassArgs &a, int ntiles, size_t lds, hipStream_t st)
{
    // other lengths from 2M = 512 up (the small uneven boxes of a batch measured
    // faster with one tile per block)
    if constexpr (MAXE == 8) {
        if (!(a.in_mode == IN_HERM && a.nsum > 1) && (P2 || a.fd.N >= 512)) {
            constexpr bool wide = sizeof(T) == 8; // FP64 tiles: every mode, EPT up to 2 MAXE
            if (!wide && a.in_mode != IN_ZPAD && a.in_mode != IN_ZPAD0) {
                // one tile per block, the default widths at compile time
                if (P2 && a.W == 8) return launch_pass_w<T, TI, TO, MAXE, P2, -8, 0>(a, ntiles, lds, st);
                if (P2 && a.W == 16) return launch_pass_w<T, TI, TO, MAXE, P2, -16, 0>(a, ntiles, lds, st);
                return launch_pass_k<T, TI, TO, MAXE, P2>(a, ntiles, lds, st);
            }
            if (pass_fits<8, 8>(a)) return launch_pass_w<T, TI, TO, 8, P2, 8, 8>(a, ntiles, lds, st);
            if (pass_fits<16, 8>(a)) return launch_pass_w<T, TI, TO, 8, P2, 16, 8>(a, ntiles, lds, st);
            if (pass_fits<4, 8>(a)) return launch_pass_w<T, TI, TO, 8, P2, 4, 8>(a, ntiles, lds, st);
            if constexpr (wide) {
                if (pass_fits<8, 16>(a)) return launch_pass_w<T, TI, TO, 8, P2, 8, 16>(a, ntiles, lds, st);
                if (pass_fits<16, 16>(a)) return launch_pass_w<T, TI, TO, 8, P2, 16, 16>(a, ntiles, lds, st);
                if (pass_fits<4, 16>(a)) return launch_pass_w<T, TI, TO, 8, P2, 4, 16>(a, ntiles, lds, st);
            }
        }
    }
    launch_pass_k<T, TI, TO, MAXE, P2>(a, ntiles, lds, st);
}

template <typename T, typename TI, typename TO>
static hipError_t launch_pass_t(const PassArgs &a, hipStream_t st)
{
    const int ncb = (a.ncols + a.W - 1) / a.W;
    const int64_t ntl = (int64_t)ncb * a.nbatch;
    const size_t lds = tile_lds<T>(a.fd.N, a.W);
    const int work = (a.W / 2) * a.fd.N;
    const bool p2 = is_pow2(a.fd.N);
    if (ntl <= 0) return hipSuccess;
    if (ntl > INT32_MAX) return hipErrorInvalidValue;
    const int ntiles = (int)ntl;
    if (big_fft(a.fd.N)) {
        if (a.W != 2 || work > 8 * NTB) return hipErrorInvalidValue;
        if (work <= 4 * NTB) {
            if (p2)
                launch_pass_k<T, TI, TO, 4, true, NTB>(a, ntiles, lds, st);
            else
                launch_pass_k<T, TI, TO, 4, false, NTB>(a, ntiles, lds, st);
        } else {
            if (p2)
                launch_pass_k<T, TI, TO, 8, true, NTB>(a, ntiles, lds, st);
            else
                launch_pass_k<T, TI, TO, 8, false, NTB>(a, ntiles, lds, st);
        }
        return hipGetLastError();
    }
    if (work <= 4 * NT) {
        if (p2)
            launch_pass_m<T, TI, TO, 4, true>(a, ntiles, lds, st);
        else
            launch_pass_m<T, TI, TO, 4, false>(a, ntiles, lds, st);
    } else if (work <= 8 * NT) {
        if (p2)
            launch_pass_m<T, TI, TO, 8, true>(a, ntiles, lds, st);
        else
            launch_pass_m<T, TI, TO, 8, false>(a, ntiles, lds, st);
    } else if (work <= 16 * NT) {
        if (p2)
            launch_pass_m<T, TI, TO, 16, true>(a, ntiles, lds, st);
        else
            launch_pass_m<T, TI, TO, 16, false>(a, ntiles, lds, st);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static bool pass_strides_ok(const PassArgs &a)
{
    // loads address rows [0, nrows_in) of the input, stores rows [0, out_nrows) of the output
    return tile_strides_ok(a.nrows_in, a.irs, a.ncols, a.ics) && tile_strides_ok(a.out_nrows, a.ors, a.ncols, a.ocs);
}

// Several independent passes in one launch, one tile per block: block b runs
// tile b - first[i] of pass i (first[i] <= b < first[i + 1]).  The passes
// share the element types; the tile budget and the LDS are those of the
// largest tile.  Used where the passes are small (the per-family transforms
// of uneven boxes), so that they fill the device together.
template <typename T, typename TI, typename TO, int MAXE, bool P2>
__global__ __launch_bounds__(NT) void k_pass_multi(MultiPassArgs m)
{
    const int b = xcd_remap(blockIdx.x, m.first[m.n]);
    int i = 0;
    while (i + 1 < m.n && b >= m.first[i + 1]) ++i;
    pass_tile<T, TI, TO, MAXE, P2, NT>(m.p[i], b - m.first[i]);
}

template <typename T, typename TI, typename TO>
static hipError_t launch_multi_t(MultiPassArgs &m, hipStream_t st)
{
    size_t lds = 0;
    int work = 0, tot = 0;
    bool p2 = true;
    for (int i = 0; i < m.n; ++i) {
        const PassArgs &a = m.p[i];
        if (big_fft(a.fd.N) || a.W < 2 || !pass_strides_ok(a)) return hipErrorInvalidValue;
        const int64_t ntl = (int64_t)((a.ncols + a.W - 1) / a.W) * a.nbatch;
        if (ntl < 0 || tot + ntl > INT32_MAX) return hipErrorInvalidValue;
        m.first[i] = tot;
        tot += (int)ntl;
        lds = std::max(lds, tile_lds<T>(a.fd.N, a.W));
        work = std::max(work, (a.W / 2) * a.fd.N);
        p2 = p2 && is_pow2(a.fd.N);
    }
    m.first[m.n] = tot;
    if (tot == 0) return hipSuccess;
    auto go = [&](const void *fn, auto kern) {
        set_lds(fn, lds);
        hipLaunchKernelGGL(kern, dim3((unsigned)tot), dim3(NT), lds, st, m);
    };
#define IPS_MULTI(MX, PP) go((const void *)&k_pass_multi<T, TI, TO, MX, PP>, k_pass_multi<T, TI, TO, MX, PP>)
    if (work <= 4 * NT) {
        if (p2) IPS_MULTI(4, true); else IPS_MULTI(4, false);
    } else if (work <= 8 * NT) {
        if (p2) IPS_MULTI(8, true); else IPS_MULTI(8, false);
    } else if (work <= 16 * NT) {
        if (p2) IPS_MULTI(16, true); else IPS_MULTI(16, false);
    } else {
        return hipErrorInvalidValue;
    }
#undef IPS_MULTI
    return hipGetLastError();
}

hipError_t launch_pass_multi(const PassArgs *p, int n, bool in_f32, bool out_f32, hipStream_t st)
{
    if (n < 1 || n > kMultiPass) return hipErrorInvalidValue;
    MultiPassArgs m{};
    m.n = n;
    for (int i = 0; i < n; ++i) m.p[i] = p[i];
    if (!in_f32 && !out_f32) return launch_multi_t<double, double, double>(m, st);
    if (in_f32 && out_f32) return launch_multi_t<float, float, float>(m, st);
    if (!in_f32 && out_f32) return launch_multi_t<float, double, float>(m, st);
    return launch_multi_t<float, float, double>(m, st);
}

hipError_t launch_pass_f32t(const PassArgs &a, hipStream_t st)
{
    if (!pass_strides_ok(a)) return hipErrorInvalidValue;
    return launch_pass_t<float, double, double>(a, st);
}

hipError_t launch_pass(const PassArgs &a, bool in_f32, bool out_f32, hipStream_t st)
{
    if (!pass_strides_ok(a)) return hipErrorInvalidValue;
    if (!in_f32 && !out_f32) return launch_pass_t<double, double, double>(a, st);
    if (in_f32 && out_f32) return launch_pass_t<float, float, float>(a, st);
    if (!in_f32 && out_f32) return launch_pass_t<float, double, float>(a, st);
    return launch_pass_t<float, float, double>(a, st);
}

} // namespace ips
