// HIP kernels of the infinite-domain Poisson solver (gfx950).
//
// Stage map (paper sections):
//   k_pass    (pass.hip) pencil transforms: DST-I / zero-padded cos+sin / even (DCT-I) /
//             hermitian synthesis along one axis (Sections 3, 4, 5)
//   k_cc      (conv.hip) boundary values as sums over slices of 2D (3D problems) or 1D
//             (2D problems) discrete convolutions, accumulated in Fourier
//             space with the kernel spectra (Section 4, eqs. Trap2D,
//             Trap2Dconvolution, convolution)
//   k_gtilde  transfer of the boundary values of the compact operator to the
//             right-hand side next to the boundary (eq. harmonic4thOrderNH2D)
//   k_r6t     sixth-order right-hand side on the layers near the boundary,
//             from its sine coefficients (eqs. 6thOrderRelation2D/3D)
//   k_rcore,  boundary terms of that right-hand side and its cubic
//   k_dcorr   extrapolation next to the boundary (Section 5)
//   k_final   spectral combination phi_star + phi_H and first inverse pass
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <type_traits>
#include <mutex>
#include <tuple>

#include "common.h"
#include "kernels.h"

namespace ips {

// Allow more than 64 KiB of dynamic LDS where a tile needs it (gfx950 has
// 160 KiB).  Each kernel's limit is raised once per process, to the largest
// size requested so far, so that launches inside a stream capture make no
// further attribute calls.
void set_lds(const void *fn, size_t bytes)
{
    if (bytes <= 65536) return;
    static std::mutex mu;
    static std::map<const void *, size_t> done;
    std::lock_guard<std::mutex> lk(mu);
    auto it = done.find(fn);
    if (it != done.end() && it->second >= bytes) return;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess)
        done[fn] = bytes;
    else
        (void)hipGetLastError();
}


// Blocks of a kernel that fit on the device at once (occupancy times the
// number of compute units), cached per kernel, block size and LDS size.
int resident_blocks(const void *fn, int nthreads, size_t lds)
{
    static std::mutex mu;
    static std::map<std::tuple<const void *, int, size_t, int>, int> done;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_tuple(fn, nthreads, lds, dev);
    auto it = done.find(key);
    if (it != done.end()) return it->second;
    int per = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, nthreads, lds) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const int r = per * ncu;
    done[key] = r;
    return r;
}

// ---------------------------------------------------------------------------
// Domain extension: the caller's block of n nodes at offset off inside the
// extended grid ne (one block row of threads per grid line of the last axis).
//   extract = false: ext[off + i] = a[i]    (embed)
//   extract = true : a[i] = ext[off + i]    (restrict; a is the output)
// ---------------------------------------------------------------------------
__global__ void k_embed(const double *src, double *dst, int64_t line0, int64_t n1, int64_t n2, int64_t e1,
                        int64_t e2, int64_t o0, int64_t o1, int64_t o2, int extract)
{
    const int64_t line = line0 + blockIdx.y; // i0 * n1 + i1
    const int64_t i0 = line / n1, i1 = line % n1;
    const int64_t ebase = ((i0 + o0) * e1 + (i1 + o1)) * e2 + o2, cbase = line * n2;
    for (int64_t i2 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i2 < n2; i2 += (int64_t)gridDim.x * blockDim.x) {
        if (extract)
            dst[cbase + i2] = src[ebase + i2];
        else
            dst[ebase + i2] = src[cbase + i2];
    }
}

hipError_t launch_embed(const double *src, double *dst, int d, const int64_t *n, const int64_t *ne,
                        const int64_t *off, bool extract, hipStream_t st)
{
    int64_t c[3] = {1, 1, 1}, e[3] = {1, 1, 1}, o[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) {
        c[3 - d + a] = n[a];
        e[3 - d + a] = ne[a];
        o[3 - d + a] = off[a];
    }
    const int64_t lines = c[0] * c[1];
    const unsigned gx = (unsigned)std::min<int64_t>((c[2] + NT - 1) / NT, 64);
    // grid.y covers at most 65535 lines per launch
    for (int64_t l0 = 0; l0 < lines; l0 += 65535) {
        const unsigned nl = (unsigned)std::min<int64_t>(65535, lines - l0);
        hipLaunchKernelGGL(k_embed, dim3(gx, nl), dim3(NT), 0, st, src, dst, l0, c[1], c[2], e[1], e[2], o[0], o[1],
                           o[2], extract ? 1 : 0);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small element-wise kernels
// ---------------------------------------------------------------------------
// out[s][i] = sum over c of part[s][c][i] (i < len, s < nset, c < nchunk): the
// lanes take 64 consecutive i, the 16 waves of a block every 16th chunk with
// eight loads in flight, combined in LDS in a fixed order.
constexpr int kRedWaves = 16;

__global__ __launch_bounds__(64 * kRedWaves) void k_reduce(const double *part, double *out, int64_t len,
                                                           int nchunk)
{
    __shared__ double red[kRedWaves][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t i = blockIdx.x * (int64_t)64 + lane;
    const double *src = part + (int64_t)blockIdx.y * nchunk * len + i;
    double s = 0.0;
    if (i < len) {
        for (int c0 = wave; c0 < nchunk; c0 += 8 * kRedWaves) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int c = c0 + u * kRedWaves;
                v[u] = c < nchunk ? src[(int64_t)c * len] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
    }
    red[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && i < len) {
        for (int w = 1; w < kRedWaves; ++w) s += red[w][lane];
        out[(int64_t)blockIdx.y * len + i] = s;
    }
}

hipError_t launch_reduce(const double *part, double *out, int64_t len, int nchunk, int nset, hipStream_t st)
{
    const int64_t nb = (len + 63) / 64;
    if (nb > INT32_MAX || nset < 1 || nset > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)nb, (unsigned)nset), dim3(64 * kRedWaves), 0, st, part, out, len,
                       nchunk);
    return hipGetLastError();
}

__global__ void k_fill(double *p, int64_t n, double v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_to_f32(const double *src, float *dst, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

hipError_t launch_to_f32(const double *src, float *dst, int64_t n, hipStream_t st)
{
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>((n + NT - 1) / NT, 8192));
    hipLaunchKernelGGL(k_to_f32, dim3(nb), dim3(NT), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t st)
{
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>((n + NT - 1) / NT, 8192));
    hipLaunchKernelGGL(k_fill, dim3(nb), dim3(NT), 0, st, p, n, v);
    return hipGetLastError();
}

// Node index helpers ---------------------------------------------------------
__device__ __forceinline__ int64_t node_off(const int64_t *n, int d, const int *i)
{
    int64_t o = 0;
    for (int a = 0; a < d; ++a) o = o * n[a] + i[a];
    return o;
}

__device__ __forceinline__ bool on_boundary(const Geo &g, const int *i)
{
    for (int a = 0; a < g.d; ++a)
        if (i[a] == 0 || i[a] == g.M[a]) return true;
    return false;
}

// ---------------------------------------------------------------------------
// Boundary values -> phi (faces, then edges and corners by lowest axis)
// ---------------------------------------------------------------------------
__global__ void k_bwrite(BwriteArgs a)
{
    const Geo &g = a.geo;
    const int d = g.d;
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int fam = 0; fam < d; ++fam) {
        // ranges of the in-face axes: lower axes exclude their end nodes
        int lo[2] = {0, 0}, len[2] = {1, 1}, ax[2] = {0, 0}, na = 0;
        for (int b = 0; b < d; ++b) {
            if (b == fam) continue;
            ax[na] = b;
            lo[na] = b < fam ? 1 : 0;
            len[na] = b < fam ? g.M[b] - 1 : g.M[b] + 1;
            ++na;
        }
        const int64_t cnt = 2 * (int64_t)len[0] * len[1];
        if (e < cnt) {
            const int f = (int)(e / ((int64_t)len[0] * len[1]));
            const int64_t r = e % ((int64_t)len[0] * len[1]);
            int j[2];
            j[0] = lo[0] + (int)(na == 2 ? r / len[1] : r);
            j[1] = na == 2 ? lo[1] + (int)(r % len[1]) : 0;
            int idx[3];
            idx[fam] = f ? g.M[fam] : 0;
            for (int q = 0; q < na; ++q) idx[ax[q]] = j[q];
            const double v =
                a.F[fam][f * a.fs[fam][0] + j[0] * a.fs[fam][1] + (na == 2 ? j[1] * a.fs[fam][2] : 0)];
            a.phi[node_off(a.n, d, idx)] = a.scale[fam] * v;
            return;
        }
        e -= cnt;
    }
}

hipError_t launch_bwrite(const BwriteArgs &a, hipStream_t st)
{
    int64_t tot = 0;
    const Geo &g = a.geo;
    for (int fam = 0; fam < g.d; ++fam) {
        int64_t c = 2;
        for (int b = 0; b < g.d; ++b)
            if (b != fam) c *= b < fam ? g.M[b] - 1 : g.M[b] + 1;
        tot += c;
    }
    hipLaunchKernelGGL(k_bwrite, dim3((unsigned)((tot + NT - 1) / NT)), dim3(NT), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Shell layer sizes
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ int64_t shell_size(const Geo &g, int a)
{
    int64_t s = 1;
    for (int b = 0; b < g.d; ++b)
        if (b != a) s *= g.M[b] - 1;
    return s;
}

// ---------------------------------------------------------------------------
// Parity packing of the shell spectra (see ShellSpec::P)
// ---------------------------------------------------------------------------
__global__ void k_pack(PackArgs a)
{
    const Geo &g = a.geo;
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int fam = 0; fam < g.d; ++fam) {
        const int64_t ss = shell_size(g, fam);
        if (e < ss) {
            const double *G = a.G[fam];
            double *P = a.P[fam];
            const double g0 = G[e], g1 = G[ss + e];
            double v[6];
            v[0] = g0 - g1; // par 0 (even k), t 0
            v[3] = g0 + g1; // par 1 (odd k), t 0
            if (a.withD) {
                const double *D = a.D[fam];
                const double d1 = D[e], d2 = D[ss + e], d3 = D[2 * ss + e], d4 = D[3 * ss + e];
                v[1] = d1 - d4;
                v[2] = d2 - d3;
                v[4] = d1 + d4;
                v[5] = d2 + d3;
            }
            const int nt = a.withD ? 6 : 1;
            for (int t = 0; t < 6; ++t)
                if (t % 3 < nt) P[t * ss + e] = v[t];
            if (fam == 2 && g.d == 3 && a.P2T) {
                // e = (k0-1) * I1 + (k1-1)  ->  (k1-1) * I0 + (k0-1)
                const int I0 = g.M[0] - 1, I1 = g.M[1] - 1;
                const int64_t et = (e % I1) * I0 + e / I1;
                for (int t = 0; t < 6; ++t)
                    if (t % 3 < nt) {
                        if (a.p2t_f32)
                            static_cast<float *>(a.P2T)[t * ss + et] = (float)v[t];
                        else
                            static_cast<double *>(a.P2T)[t * ss + et] = v[t];
                    }
            }
            if (fam == 1 && g.d == 3 && a.P1T) {
                // e = (k0-1) * I2 + (k2-1)  ->  (k2-1) * I0 + (k0-1)
                const int I0 = g.M[0] - 1, I2 = g.M[2] - 1;
                const int64_t et = (e % I2) * I0 + e / I2;
                for (int t = 0; t < 6; ++t)
                    if (t % 3 < nt) a.P1T[t * ss + et] = v[t];
            }
            return;
        }
        e -= ss;
    }
}

hipError_t launch_pack(const PackArgs &a, hipStream_t st)
{
    int64_t tot = 0;
    for (int fam = 0; fam < a.geo.d; ++fam) tot += shell_size(a.geo, fam);
    hipLaunchKernelGGL(k_pack, dim3((unsigned)((tot + NT - 1) / NT)), dim3(NT), 0, st, a);
    return hipGetLastError();
}

// 1/x from the hardware reciprocal refined by two Newton steps
// (each doubles the correct bits: the result is within an ulp or two of 1/x).
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// FP32: one Newton step on the hardware reciprocal.
__device__ __forceinline__ float recip(float x)
{
    float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}


// ---------------------------------------------------------------------------
// Sixth-order right-hand side of the harmonic part, interior contribution.
// The stencils applied to the interior part of u1 act on its sine
// coefficients as the symbol m_R(k); so the coefficients of that part of the
// right-hand side are
//     V(k) = prod(2/M) * m_R(k) * gt_hat(k) / Lambda(k).
// Its values on the layers j = 1..5 and M-5..M-1 of every axis a are
//     T_a[j][k_other] = sum_{k_a} sin(pi k_a j / M_a) V(k)
// (followed by an inverse sine transform over the other axes).  Parity:
// sin(pi k (M-j)/M) = (-1)^(k+1) sin(pi k j / M).
//
// k_r6t computes the three (two in 2D) contractions in one launch and never
// stores V: each thread owns one position (k_b, k_c) and sums over a quarter
// of the k_a, rebuilding V(k) from the packed shell spectra:
//   gt_hat = sin(pi k_a/M_a) G_a(k_b, k_c) + sin(pi k_l/M_l) G_l(.., k_a, ..)
//            + sin(pi k_w/M_w) G_w(.., k_a, ..)
// where l is the axis that varies across the lanes of a wave and w the
// other one.  The lanes read G_w contiguously (3D: for a = 2 from the
// transposed family-1 copy) and G_l at one of two addresses (parity of
// k_l).  With lambda_a the only varying eigenvalue,
//   Lambda = A0 + A1 lambda_a,  m_R = B0 + lambda_a (B1 + B2 lambda_a).
// Block: 64 PPT positions x 4 wave groups; group g takes k_a = 1 + g + 4t,
// so its parity is fixed and the layer pairs split into odd and even sums.
// Each thread carries PPT positions (64 apart) through the k_a loop: their
// loads and reciprocals are independent, which hides more latency per wave.
// ---------------------------------------------------------------------------
template <int D, int PPT, int KU>
__global__ __launch_bounds__(NT) void k_r6t(R6Args a)
{
    constexpr int PB = 64 * PPT, NG = NT / 64;
    __shared__ double red[NG][5][PB];
    const Geo &g = a.geo;
    int ax = 0, blk = blockIdx.x;
    while (ax < D - 1 && blk >= a.nblk[ax]) {
        blk -= a.nblk[ax];
        ++ax;
    }
    const int lane = threadIdx.x & 63;
    const int grp = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int Ia = g.M[ax] - 1;
    int la, wa;
    if (D == 3) {
        la = ax == 2 ? 0 : 2;
        wa = ax == 1 ? 0 : 1;
    } else {
        la = 1 - ax;
        wa = -1;
    }
    const int Il = g.M[la] - 1;
    const int Iw = D == 3 ? g.M[wa] - 1 : 1;
    const int npos = Il * Iw;
    const int para = (grp & 1) ? 0 : 1; // parity of k_a in this group
    const int64_t ssa = shell_size(g, ax), ssl = shell_size(g, la);
    // per position q (PPT independent positions per thread, 64 apart)
    double A0[PPT], A1[PPT], B0[PPT], B1[PPT], B2[PPT], gown[PPT], sbl[PPT], scw[PPT];
    const double *pb[PPT], *pc[PPT];
    int64_t bs = 1, cs = 0;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int p = blk * PB + q * 64 + lane;
        const int pp = p < npos ? p : 0;
        const int kl = 1 + pp % Il;
        const int kw = 1 + pp / Il;
        // symbols as polynomials in lambda_a
        const double lamL = a.tab[la].lam[kl - 1];
        A0[q] = lamL;
        A1[q] = 1.0 + g.c2[ax][la] * lamL;
        B0[q] = 0.0;
        B1[q] = g.c4[la][ax] * lamL * lamL;
        B2[q] = g.c4[ax][la] * lamL;
        if (D == 3) {
            const double lamW = a.tab[wa].lam[kw - 1];
            A0[q] += lamW + g.c2[la][wa] * lamL * lamW;
            A1[q] += g.c2[ax][wa] * lamW;
            B0[q] = g.c4[la][wa] * lamL * lamL * lamW + g.c4[wa][la] * lamL * lamW * lamW;
            B1[q] += g.c4[wa][ax] * lamW * lamW;
            B2[q] += g.c4[ax][wa] * lamW;
        }
        // own family (normal to a): fixed value for this group's parity
        int64_t oown;
        if (D == 3)
            oown = ax == 2 ? (int64_t)(kl - 1) * Iw + (kw - 1) : (int64_t)(kw - 1) * Il + (kl - 1);
        else
            oown = kl - 1;
        gown[q] = a.P[ax][(int64_t)para * 3 * ssa + oown];
        // family normal to the lane axis: two addresses per wave
        sbl[q] = a.tab[la].s[kl - 1];
        pb[q] = a.P[la] + (int64_t)(kl & 1) * 3 * ssl;
        if (D == 3) {
            if (ax == 0) {
                pb[q] += kw - 1; // G_2[k0][k1], k0 = k_a
                bs = Iw;
            } else if (ax == 1) {
                pb[q] += (int64_t)(kw - 1) * (g.M[1] - 1); // G_2[k0][k1], k1 = k_a
            } else {
                pb[q] += (int64_t)(kw - 1) * (g.M[2] - 1); // G_0[k1][k2], k2 = k_a
            }
        }
        // family normal to the wave axis (3D): contiguous across the lanes
        pc[q] = nullptr;
        scw[q] = 0.0;
        if (D == 3) {
            const int64_t ssw = shell_size(g, wa);
            scw[q] = a.tab[wa].s[kw - 1];
            const double *base = ax == 2 ? a.P1T : a.P[wa];
            pc[q] = base + (int64_t)(kw & 1) * 3 * ssw + (kl - 1);
            cs = ax == 2 ? (g.M[0] - 1) : (g.M[2] - 1);
        }
    }
    const double *tl = a.tab[ax].lam;
    const double *ts = a.tab[ax].s;
    double acc[PPT][5];
#pragma unroll
    for (int q = 0; q < PPT; ++q)
#pragma unroll
        for (int j = 0; j < 5; ++j) acc[q][j] = 0.0;
    // split s of gridDim.y: every gridDim.y-th wavenumber of this group's
    // residue (the parity of k_a stays that of the group)
    const int ks = gridDim.y, sp = blockIdx.y, step = NG * ks;
    // one wavenumber: pbv, pcv are the family values at (position q, ka)
    auto term = [&](int ka, const double *pbv, const double *pcv) {
        const double lk = tl[ka - 1], sk = ts[ka - 1];
        double sj[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) sj[j] = ts[j * Ia + ka - 1];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            double gt = sk * gown[q] + sbl[q] * pbv[q];
            if (D == 3) gt += scw[q] * pcv[q];
            const double L = fma(A1[q], lk, A0[q]);
            const double R = fma(fma(B2[q], lk, B1[q]), lk, B0[q]);
            const double v = R * gt * recip(L);
#pragma unroll
            for (int j = 0; j < 5; ++j) acc[q][j] = fma(sj[j], v, acc[q][j]);
        }
    };
    // KU wavenumbers per iteration, their strided family loads issued first
    // (more loads in flight per wave)
    int ka = 1 + grp + NG * sp;
    for (; ka + (KU - 1) * step <= Ia; ka += KU * step) {
        double pbv[KU][PPT], pcv[KU][PPT];
#pragma unroll
        for (int u = 0; u < KU; ++u)
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                const int64_t k1 = ka - 1 + u * step;
                pbv[u][q] = pb[q][k1 * bs];
                pcv[u][q] = D == 3 ? pc[q][k1 * cs] : 0.0;
            }
#pragma unroll
        for (int u = 0; u < KU; ++u) term(ka + u * step, pbv[u], pcv[u]);
    }
    for (; ka <= Ia; ka += step) {
        double pbv[PPT], pcv[PPT];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            pbv[q] = pb[q][(int64_t)(ka - 1) * bs];
            pcv[q] = D == 3 ? pc[q][(int64_t)(ka - 1) * cs] : 0.0;
        }
        term(ka, pbv, pcv);
    }
#pragma unroll
    for (int q = 0; q < PPT; ++q)
#pragma unroll
        for (int j = 0; j < 5; ++j) red[grp][j][q * 64 + lane] = acc[q][j];
    __syncthreads();
    // group g finishes positions g*64/...: every thread of the block writes
    // its share of the PB positions
    // several splits: FP64 partials [split][10][positions] of this axis,
    // summed into T by k_r6t_sum
    double *Td = ks > 1 ? a.part + a.part_off[ax] + (int64_t)sp * 10 * npos : static_cast<double *>(a.T[ax]);
    float *Tf = static_cast<float *>(a.T[ax]);
    for (int i = threadIdx.x; i < PB; i += NT) {
        const int p = blk * PB + i;
        if (p >= npos) continue;
        const int kl = 1 + p % Il, kw = 1 + p / Il;
        const int64_t pout = (D == 3 && ax == 2) ? (int64_t)(kl - 1) * Iw + (kw - 1) : p;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const double od = red[0][j][i] + red[2][j][i];
            const double ev = red[1][j][i] + red[3][j][i];
            const double v1 = g.pref * (od + ev), v2 = g.pref * (od - ev);
            if (a.t_f32 && ks == 1) {
                Tf[j * (int64_t)npos + pout] = (float)v1;
                Tf[(5 + j) * (int64_t)npos + pout] = (float)v2;
            } else {
                Td[j * (int64_t)npos + pout] = v1;
                Td[(5 + j) * (int64_t)npos + pout] = v2;
            }
        }
    }
}

// T[ax][l][p] = sum over the splits of part[ax][s][l][p] (10 layers of npos)
__global__ void k_r6t_sum(R6Args a, int ax, int ks)
{
    const int64_t len = 10 * shell_size(a.geo, ax);
    const double *src = a.part + a.part_off[ax];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int sp = 0; sp < ks; ++sp) v += src[(int64_t)sp * len + i];
        if (a.t_f32)
            static_cast<float *>(a.T[ax])[i] = (float)v;
        else
            static_cast<double *>(a.T[ax])[i] = v;
    }
}

template <int PPT, int KU>
static hipError_t launch_r6t_p(R6Args a, hipStream_t st)
{
    const int d = a.geo.d;
    int tot = 0;
    for (int ax = 0; ax < d; ++ax) {
        const int np = (int)shell_size(a.geo, ax);
        a.nblk[ax] = (np + 64 * PPT - 1) / (64 * PPT);
        tot += a.nblk[ax];
    }
    const int ks = r6t_splits(a.geo);
    if (ks > 1 && !a.part) return hipErrorInvalidValue;
    if (d == 3)
        hipLaunchKernelGGL((k_r6t<3, PPT, KU>), dim3(tot, ks), dim3(NT), 0, st, a);
    else
        hipLaunchKernelGGL((k_r6t<2, PPT, KU>), dim3(tot, ks), dim3(NT), 0, st, a);
    hipError_t e = hipGetLastError();
    for (int ax = 0; ax < d && ks > 1 && e == hipSuccess; ++ax) {
        const int64_t len = 10 * shell_size(a.geo, ax);
        const unsigned nb = (unsigned)std::min<int64_t>((len + NT - 1) / NT, 4096);
        hipLaunchKernelGGL(k_r6t_sum, dim3(nb), dim3(NT), 0, st, a, ax, ks);
        e = hipGetLastError();
    }
    return e;
}

// two positions per thread, two wavenumbers per iteration (measured against
// one and four of each)
hipError_t launch_r6t(R6Args a, hipStream_t st) { return launch_r6t_p<2, 2>(a, st); }

int r6t_splits(const Geo &g)
{
    int tot = 0, mina = 1 << 30;
    for (int ax = 0; ax < g.d; ++ax) {
        tot += (int)((shell_size(g, ax) + 127) / 128);
        mina = std::min(mina, g.M[ax] - 1);
    }
    const int want = (1024 + tot - 1) / tot;
    const int cap = std::max(1, mina / 128);
    return std::max(1, std::min(want, cap));
}

// ---------------------------------------------------------------------------
// D = R - R_spec on the nodes with an index in {1, 2, M-2, M-1}, in two steps.
//   k_rcore: R on the core nodes with an index along axis a in
//            {2..5, M-5..M-2}:  R = R_spec + boundary terms, where a
//            D2^2 D2 stencil centred on index 2 or M-2 of some axis x reaches
//            the face of x: c4[x][y] D2_y g / h_x^4 for every y != x.
//            C[a][l][other], l = 0..7 for the layers 2,3,4,5,M-5,..,M-2.
//   k_dcorr: R at the shell nodes by tensor-product cubic extrapolation
//            (index 1 <- 4,-6,4,-1 times indices 2..5, mirrored at M-1),
//            minus R_spec.  A node belongs to the lowest axis that has an
//            index in {1, 2, M-2, M-1} there; other layers hold 0.
// Both read R_spec only from the layers of their own axis.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int layer5(int i, int M)
{
    return i <= 5 ? i - 1 : 5 + (M - 1 - i);
}

template <int D>
__device__ __forceinline__ void other_axes(int a, int *ob)
{
    int q = 0;
    for (int b = 0; b < D; ++b)
        if (b != a) ob[q++] = b;
}

// R_spec value (FP32 or FP64 storage)
__device__ __forceinline__ double rs_at(const DcorrArgs &a, int fam, int64_t o)
{
    return a.rs_f32 ? (double)static_cast<const float *>(a.RS[fam])[o] : static_cast<const double *>(a.RS[fam])[o];
}

template <int D>
__global__ __launch_bounds__(NT) void k_rcore(DcorrArgs a)
{
    const Geo &g = a.geo;
    const int fam = blockIdx.y >> 3, l = blockIdx.y & 7;
    const int64_t ss = shell_size(g, fam);
    const int e = blockIdx.x * NT + threadIdx.x;
    if (e >= ss) return;
    int ob[2] = {0, 0};
    other_axes<D>(fam, ob);
    int i[3] = {0, 0, 0};
    const int Mf = g.M[fam];
    i[fam] = l < 4 ? 2 + l : Mf - 2 - (7 - l);
    if (D == 3) {
        const int Ic = g.M[ob[1]] - 1;
        i[ob[0]] = 1 + e / Ic;
        i[ob[1]] = 1 + e % Ic;
    } else {
        i[ob[0]] = 1 + e;
    }
    bool core = true;
    for (int b = 0; b < D; ++b) core = core && i[b] >= 2 && i[b] <= g.M[b] - 2;
    double v = 0.0;
    if (core) {
        v = rs_at(a, fam, (int64_t)layer5(i[fam], Mf) * ss + e);
#pragma unroll
        for (int x = 0; x < D; ++x) {
            if (i[x] != 2 && i[x] != g.M[x] - 2) continue;
            int q[3] = {i[0], i[1], i[2]};
            q[x] = i[x] == 2 ? 0 : g.M[x];
            double t = 0.0;
#pragma unroll
            for (int y = 0; y < D; ++y) {
                if (y == x) continue;
                int qm[3] = {q[0], q[1], q[2]}, qp[3] = {q[0], q[1], q[2]};
                qm[y] -= 1;
                qp[y] += 1;
                const double f0 = a.phi[node_off(a.n, D, q)];
                const double fm = a.phi[node_off(a.n, D, qm)];
                const double fp = a.phi[node_off(a.n, D, qp)];
                t += g.c4[x][y] * (fm - 2.0 * f0 + fp) / (g.h[y] * g.h[y]);
            }
            const double h2 = g.h[x] * g.h[x];
            v += t / (h2 * h2);
        }
    }
    a.C[fam][(int64_t)l * ss + e] = v;
}

template <int D>
__global__ __launch_bounds__(NT) void k_dcorr(DcorrArgs a)
{
    const Geo &g = a.geo;
    const int fam = blockIdx.y >> 2, jj = blockIdx.y & 3;
    const int64_t ss = shell_size(g, fam);
    const int e = blockIdx.x * NT + threadIdx.x;
    if (e >= ss) return;
    int ob[2] = {0, 0};
    other_axes<D>(fam, ob);
    const int Mf = g.M[fam];
    const int L4[4] = {1, 2, Mf - 2, Mf - 1};
    int i[3] = {0, 0, 0};
    i[fam] = L4[jj];
    int Ic = 1;
    if (D == 3) {
        Ic = g.M[ob[1]] - 1;
        i[ob[0]] = 1 + e / Ic;
        i[ob[1]] = 1 + e % Ic;
    } else {
        i[ob[0]] = 1 + e;
    }
    bool owned = true;
    for (int b = 0; b < fam; ++b) {
        const int m = g.M[b];
        if (i[b] == 1 || i[b] == 2 || i[b] == m - 2 || i[b] == m - 1) owned = false;
    }
    double out = 0.0;
    if (owned) {
        const double *C = a.C[fam];
        // along the family axis (uniform over the block)
        const bool exa = jj == 0 || jj == 3;
        int l0;
        if (jj == 0)
            l0 = 0;
        else if (jj == 3)
            l0 = 7;
        else
            l0 = jj == 1 ? 0 : 7;
        const int dl = jj == 3 ? -1 : 1;
        // in-face axes: 1 or 4 taps each
        int nt[2] = {1, 1}, p0[2] = {0, 0}, dp[2] = {0, 0};
        for (int q = 0; q < D - 1; ++q) {
            const int b = ob[q], m = g.M[b];
            if (i[b] == 1) {
                nt[q] = 4;
                p0[q] = 2;
                dp[q] = 1;
            } else if (i[b] == m - 1) {
                nt[q] = 4;
                p0[q] = m - 2;
                dp[q] = -1;
            } else {
                p0[q] = i[b];
            }
        }
        const double wt[4] = {4.0, -6.0, 4.0, -1.0};
        double R = 0.0;
        for (int t0 = 0; t0 < nt[0]; ++t0) {
            const double w0 = nt[0] == 1 ? 1.0 : wt[t0];
            const int pb = p0[0] + dp[0] * t0;
            for (int t1 = 0; t1 < (D == 3 ? nt[1] : 1); ++t1) {
                const double w1 = (D == 3 && nt[1] == 4) ? wt[t1] : 1.0;
                const int pc = D == 3 ? p0[1] + dp[1] * t1 : 1;
                const int64_t o = D == 3 ? (int64_t)(pb - 1) * Ic + (pc - 1) : pb - 1;
                double v;
                if (exa) {
                    const double c0 = C[(int64_t)(l0)*ss + o], c1 = C[(int64_t)(l0 + dl) * ss + o];
                    const double c2 = C[(int64_t)(l0 + 2 * dl) * ss + o], c3 = C[(int64_t)(l0 + 3 * dl) * ss + o];
                    v = 4.0 * c0 - 6.0 * c1 + 4.0 * c2 - c3;
                } else {
                    v = C[(int64_t)l0 * ss + o];
                }
                R += w0 * w1 * v;
            }
        }
        out = R - rs_at(a, fam, (int64_t)layer5(i[fam], Mf) * ss + e);
    }
    a.D[fam][(int64_t)jj * ss + e] = out;
}

hipError_t launch_dcorr(const DcorrArgs &a, hipStream_t st)
{
    const int d = a.geo.d;
    int64_t mx = 1;
    for (int fam = 0; fam < d; ++fam) mx = std::max(mx, shell_size(a.geo, fam));
    const unsigned nb = (unsigned)((mx + NT - 1) / NT);
    if (d == 3) {
        hipLaunchKernelGGL(k_rcore<3>, dim3(nb, 8 * d), dim3(NT), 0, st, a);
        hipLaunchKernelGGL(k_dcorr<3>, dim3(nb, 4 * d), dim3(NT), 0, st, a);
    } else {
        hipLaunchKernelGGL(k_rcore<2>, dim3(nb, 8 * d), dim3(NT), 0, st, a);
        hipLaunchKernelGGL(k_dcorr<2>, dim3(nb, 4 * d), dim3(NT), 0, st, a);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// g~ = -(L_h B) on the interior nodes next to the boundary, split into one
// layer pair per axis (a node belongs to the lowest axis whose index is 1 or
// M-1 there; other layers hold 0 at that node).  Every neighbour of such a
// node is a grid node, so all are loaded at once and those off the boundary
// are dropped.
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(NT) void k_gtilde(GtArgs a)
{
    const Geo &g = a.geo;
    const int fam = blockIdx.y >> 1, f = blockIdx.y & 1;
    const int64_t ss = shell_size(g, fam);
    const int e = blockIdx.x * NT + threadIdx.x;
    if (e >= ss) return;
    int ob[2] = {0, 0};
    other_axes<D>(fam, ob);
    int i[3] = {0, 0, 0};
    i[fam] = f ? g.M[fam] - 1 : 1;
    if (D == 3) {
        const int Ic = g.M[ob[1]] - 1;
        i[ob[0]] = 1 + e / Ic;
        i[ob[1]] = 1 + e % Ic;
    } else {
        i[ob[0]] = 1 + e;
    }
    // with M = 2 both layers are the same nodes: keep only the first
    bool owned = !(f == 1 && g.M[fam] == 2);
    for (int b = 0; b < fam; ++b)
        if (i[b] == 1 || i[b] == g.M[b] - 1) owned = false;
    double s = 0.0;
    if (owned) {
#pragma unroll
        for (int p = 0; p < D; ++p) {
            double w = 1.0 / (g.h[p] * g.h[p]);
#pragma unroll
            for (int q = 0; q < D; ++q)
                if (q != p) w -= 2.0 * g.c2[p][q] / (g.h[p] * g.h[p] * g.h[q] * g.h[q]);
#pragma unroll
            for (int sg = -1; sg <= 1; sg += 2) {
                int j[3] = {i[0], i[1], i[2]};
                j[p] += sg;
                const double v = a.phi[node_off(a.n, D, j)];
                s += on_boundary(g, j) ? w * v : 0.0;
            }
        }
#pragma unroll
        for (int p = 0; p < D; ++p)
#pragma unroll
            for (int q = p + 1; q < D; ++q) {
                const double w = g.c2[p][q] / (g.h[p] * g.h[p] * g.h[q] * g.h[q]);
#pragma unroll
                for (int sp = -1; sp <= 1; sp += 2)
#pragma unroll
                    for (int sq = -1; sq <= 1; sq += 2) {
                        int j[3] = {i[0], i[1], i[2]};
                        j[p] += sp;
                        j[q] += sq;
                        const double v = a.phi[node_off(a.n, D, j)];
                        s += on_boundary(g, j) ? w * v : 0.0;
                    }
            }
        s = -s;
    }
    a.G[fam][(int64_t)f * ss + e] = s;
}

hipError_t launch_gtilde(const GtArgs &a, hipStream_t st)
{
    const int d = a.geo.d;
    int64_t mx = 1;
    for (int fam = 0; fam < d; ++fam) mx = std::max(mx, shell_size(a.geo, fam));
    const unsigned nb = (unsigned)((mx + NT - 1) / NT);
    if (d == 3)
        hipLaunchKernelGGL(k_gtilde<3>, dim3(nb, 2 * d), dim3(NT), 0, st, a);
    else
        hipLaunchKernelGGL(k_gtilde<2>, dim3(nb, 2 * d), dim3(NT), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Final pass along axis 0: raw DST of B along axis 0 -> beta (raw DST of rho),
// spectral combination
//   c(k) = prod(2/M) [ -beta / (pi^2 sum k^2/L^2)
//                      + (gt_hat (1 + m_R/Lambda) + D_hat) / Lambda ]   (order 6)
//   c(k) = prod(2/M) [ -beta / (pi^2 sum k^2/L^2) + gt_hat / Lambda ]     (order 4)
// then the inverse sine transform along axis 0, written back in place.
// ---------------------------------------------------------------------------
// The 12 staged values of one row or column of the final pass, read as
// 16-byte vectors (records are 16-byte aligned in both spaces).
__device__ __forceinline__ void load12(const float *p, float *r)
{
    const float4 *v = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float4 t = v[i];
        r[4 * i] = t.x;
        r[4 * i + 1] = t.y;
        r[4 * i + 2] = t.z;
        r[4 * i + 3] = t.w;
    }
}
__device__ __forceinline__ void load12(const double *p, double *r)
{
    const double2 *v = reinterpret_cast<const double2 *>(p);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const double2 t = v[i];
        r[2 * i] = t.x;
        r[2 * i + 1] = t.y;
    }
}

// Staged row kx-1 = i of the final pass (see k_final for the layout).
template <typename TR>
__device__ __forceinline__ void final_row(const FinalArgs &a, int i, int kB, double lamB, double qB,
                                          TR *r)
{
    const Geo &geo = a.geo;
    const int d = geo.d;
    const int I0 = geo.M[0] - 1;
    const int nt = a.order == 6 ? 3 : 1;
    const double c2xz = d == 3 ? geo.c2[0][2] : 0.0;
    const double c4xz = d == 3 ? geo.c4[0][2] : 0.0, c4zx = d == 3 ? geo.c4[2][0] : 0.0;
    const double lx = a.tab[0].lam[i];
    r[0] = (TR)lx;
    r[1] = (TR)(a.tab[0].q[i] + qB);
    r[2] = (TR)a.tab[0].s[i];
    r[3] = (TR)a.tab[0].s[I0 + i];
    r[10] = (TR)(lx + c2xz * lx * lamB);
    r[11] = (TR)(lx * lamB * (c4xz * lx + c4zx * lamB));
    // family 1: other index (k0, k2) in 3D (transposed copy: k0 contiguous), (k0) in 2D
    const int64_t ss1 = shell_size(geo, 1);
    const double *P1 = d == 3 ? a.sh.P1T : a.sh.P[1];
    const int64_t o = d == 3 ? (int64_t)(kB - 1) * I0 + i : i;
    for (int par = 0; par < 2; ++par)
        for (int t = 0; t < nt; ++t) r[4 + par * 3 + t] = (TR)P1[(par * 3 + t) * ss1 + o];
    for (int par = 0; par < 2; ++par)
        for (int t = nt; t < 3; ++t) r[4 + par * 3 + t] = (TR)0;
}

template <typename T, int MAXE, bool P2, int WC, int NTT, int NC>
__global__ __launch_bounds__(NTT) void k_final(FinalArgs a, int ntiles)
{
    constexpr bool BIG = NTT != NT;
    // FP64 tiles of a compile-time width (short transforms) without
    // compile-time stages: persistent blocks that fetch the next tile into
    // registers while the current one is processed (for FP32 tiles, and for
    // the compile-time stages with their direct global I/O, one tile per
    // block measured faster)
    constexpr bool PF = WC > 0 && !BIG && sizeof(T) == 8 && NC == 0;
    // one-tile blocks with compile-time stages: direct global I/O in the
    // first forward and the last inverse stage (LGSC: log2 of the sequences)
    constexpr bool DIO = NC > 0 && !PF;
    constexpr int LGSC = WC == 4 ? 1 : WC == 8 ? 2 : 3;
    extern __shared__ __align__(16) unsigned char smem[];
    // WC > 0: tile width known at compile time (row offsets become shifts)
    // NC > 0: the transform length, known at compile time (only the
    // compile-time Stockham stages of that length are built in)
    static_assert(NC == 0 || (P2 && MAXE == 8 && !BIG && NC * WC == 16 * NT), "no compile-time stages");
    FftDesc fdc{};
    if constexpr (NC > 0) {
        fdc.N = NC;
        fdc.M = NC / 2;
    }
    const FftDesc &fd = NC > 0 ? fdc : a.fd;
    const int N = fd.N, M = fd.M, W = WC > 0 ? WC : a.W, rs = BIG ? W : W + 1;
    const int lgW = WC > 0 ? __builtin_ctz(WC > 0 ? WC : 1) : 31 - __clz(W), lgs = lgW - 1;
    const cx<T> *tw = tw_table<T, BIG>(smem, a.tw, a.twf);
    const size_t twb = BIG ? 0 : (size_t)N * sizeof(cx<T>);
    T *buf = reinterpret_cast<T *>(smem + twb);
    const int ncb = (a.ncols + W - 1) / W;
    const int grid = gridDim.x;
    // logical order: groups of a.group neighbouring column blocks (together one
    // 128-byte line of every row), then the batch, then the group index -- the
    // blocks that share a line run side by side on one XCD, and each XCD sweeps
    // all batches over a narrow band of columns, so the per-element shell data
    // of that band stays in its L2
    auto decode = [&](int lb, int &cb, int &bt) {
        const int G = a.group;
        const int full = ncb / G;
        if (lb < G * full * a.nbatch) {
            const int pr = lb / (G * a.nbatch), rem = lb % (G * a.nbatch);
            bt = rem / G;
            cb = G * pr + rem % G;
        } else {
            const int left = ncb - G * full; // the last, partial group
            const int rem = lb - G * full * a.nbatch;
            bt = rem / left;
            cb = G * full + rem % left;
        }
    };
    const int lb0 = xcd_remap(blockIdx.x, grid);
    const bool rcont = a.irs == 1 && a.ics != 1;
    if (!BIG) load_twiddles<T, NTT>(reinterpret_cast<cx<T> *>(smem), a.tw, N);
    T pf[PF ? MAXE : 1];
    if constexpr (PF) {
        if (lb0 < ntiles) {
            int cb, bt;
            decode(lb0, cb, bt);
            const int c0 = cb * W;
            fetch_pair<T, NTT, (PF ? WC : 2), MAXE, false>(pf, static_cast<const T *>(a.buf) + bt * a.ibs + c0 * a.ics,
                                                          a.nrows_in, a.irs, a.ics, 0, min(W, a.ncols - c0), 0, 0,
                                                          threadIdx.x);
        }
    }
    for (int it = lb0; it < ntiles; it += grid) {
    int tid = threadIdx.x;
    if constexpr (PF) {
        asm volatile("" : "+v"(tid));
        tid &= NTT - 1;
    }
    int cb, bt;
    decode(it, cb, bt);
    const int c0 = cb * W;
    const int nc = min(W, a.ncols - c0);
    T *g = static_cast<T *>(a.buf) + bt * a.ibs + c0 * a.ics;
    // Compile-time transforms of one-tile blocks read their input rows in the
    // first stage of the forward transform and write their output rows in the
    // last stage of the inverse, straight from and to B (no tile load or store).
    const bool direct = DIO && !a.pre && a.nrows_in <= M - 1;
    if (!direct) {
        zero_rows<T, NTT>(buf, rs, lgW, 0, 1, tid);
        zero_rows<T, NTT>(buf, rs, lgW, 1 + a.nrows_in, N, tid);
    }
    if constexpr (PF) {
        put_pair<T, T, NTT, (PF ? WC : 2), MAXE>(buf, rs, 1, pf, a.nrows_in, rcont, tid);
        const int nx = it + grid;
        if (nx < ntiles) {
            int cb1, bt1;
            decode(nx, cb1, bt1);
            const int c1 = cb1 * W;
            fetch_pair<T, NTT, (PF ? WC : 2), MAXE, false>(pf, static_cast<const T *>(a.buf) + bt1 * a.ibs + c1 * a.ics,
                                                          a.nrows_in, a.irs, a.ics, 0, min(W, a.ncols - c1), 0, 0,
                                                          tid);
        }
    } else if (!direct) {
        tile_load<T, T, NTT>(buf, rs, 1, g, a.nrows_in, nc, a.irs, a.ics, lgW, tid);
    }
    const Geo &geo = a.geo;
    const int d = geo.d;
    const bool six = a.order == 6;
    const int nt = six ? 3 : 1;
    // Staged per row kx and per column ky (12 doubles each):
    //   [0] lambda  [1] q (rows: + q_z)  [2] sin(pi k/M)  [3] sin(2 pi k/M)
    //   [4..9] packed shell values of the family whose other index is fixed
    //          along the row/column, parity 0 then 1, three kinds each
    //   [10] lambda + c2[.][2] lambda lambda_z   (part of Lambda)
    //   [11] c4[.][2] lambda^2 lambda_z + c4[2][.] lambda lambda_z^2   (part of m_R)
    // so that per element Lambda = r10 + c10 + lambda_z + c2[0][1] lx ly and
    // m_R = r11 + c11 + lx ly (c4[0][1] lx + c4[1][0] ly).
    constexpr int SV = 12;
    // The row invariants come from the per-solve table in global memory
    // (written by k_final_rows); the column invariants are staged in LDS after
    // the tile, 16-byte aligned and addressed from smem, so that every access
    // to them is an LDS instruction (a pointer that may point to either space
    // would make every access a flat one). Staged values and the per-element
    // combination are in the transform type (FP32 in the mixed modes).
    const size_t soff = (twb + (size_t)N * rs * sizeof(T) + 15) & ~(size_t)15;
    const T *__restrict__ rv = static_cast<const T *>(a.rowtab) + (int64_t)bt * (M - 1) * SV;
    T *cv = reinterpret_cast<T *>(smem + soff);
    const int I0 = geo.M[0] - 1, I1 = geo.M[1] - 1, I2 = d == 3 ? geo.M[2] - 1 : 1;
    const int kB = bt + 1;
    const int64_t ss0 = shell_size(geo, 0), ss1 = shell_size(geo, 1);
    // batch (axis 2) constants and the per-element family 2
    double lamB = 0.0, qB = 0.0, s1B = 0.0, s2B = 0.0;
    int64_t ss2 = 0;
    if (d == 3) {
        lamB = a.tab[2].lam[kB - 1];
        qB = a.tab[2].q[kB - 1];
        s1B = a.tab[2].s[kB - 1];
        s2B = a.tab[2].s[I2 + kB - 1];
        ss2 = shell_size(geo, 2);
    }
    const double c2xz = d == 3 ? geo.c2[0][2] : 0.0, c2yz = d == 3 ? geo.c2[1][2] : 0.0;
    const double c4xz = d == 3 ? geo.c4[0][2] : 0.0, c4zx = d == 3 ? geo.c4[2][0] : 0.0;
    const double c4yz = d == 3 ? geo.c4[1][2] : 0.0, c4zy = d == 3 ? geo.c4[2][1] : 0.0;
    for (int i = tid; i < nc; i += NTT) {
        T *r = cv + i * SV;
        const int j = c0 + i; // k1 - 1
        const double ly = a.tab[1].lam[j];
        r[0] = (T)ly;
        r[1] = (T)a.tab[1].q[j];
        r[2] = (T)a.tab[1].s[j];
        r[3] = (T)a.tab[1].s[I1 + j];
        r[10] = (T)(ly + c2yz * ly * lamB);
        r[11] = (T)(ly * lamB * (c4yz * ly + c4zy * lamB));
        // family 0: other index (k1, k2) in 3D, (k1) in 2D
        const int64_t o = d == 3 ? (int64_t)j * I2 + (kB - 1) : j;
        for (int par = 0; par < 2; ++par)
            for (int t = 0; t < nt; ++t) r[4 + par * 3 + t] = (T)a.sh.P[0][(par * 3 + t) * ss0 + o];
    }
    __syncthreads();
    // forward transform of the zero-padded rows 1..M0-1 (unless B already holds the spectrum)
    if (direct) {
        if constexpr (DIO) {
            stage_ct_gin<T, T, NTT, NC, WC + 1, LGSC>(buf, g, a.nrows_in, nc, a.irs, a.ics, tid);
            fft_ct_tail<T, NTT, NC, WC + 1, LGSC, false>(buf, tw, tid);
        }
    } else if (!a.pre) {
        if (a.nrows_in <= M - 1)
            fft_tile_zpad<T, MAXE, NTT, P2>(buf, rs, lgs, fd, tw, tid);
        else
            fft_tile<T, MAXE, NTT, P2>(buf, rs, lgs, fd, tw, false, tid);
    }
    // One sweep over the row pairs (k, N-k) of every complex sequence s
    // (real columns 2s and 2s+1):
    //   sine coefficients  S_a = (z(N-k).y - z(k).y)/2,  S_b = (z(k).x - z(N-k).x)/2
    //   (raw DST of rho along axis 0 at kx = k; the cosine part is not needed),
    //   spectral combination of each column into its coefficient c(k),
    //   and the hermitian input of the inverse sine transform:
    //   z(k) = (c_b, -c_a), z(N-k) = (-c_b, c_a), rows 0 and M zero.
    // Each thread owns both rows of its pair, so no barrier is needed between
    // the reads and the writes.
    const T c2xy = (T)geo.c2[0][1], c4xy = (T)geo.c4[0][1], c4yx = (T)geo.c4[1][0];
    const T lamBt = (T)lamB, s1Bt = (T)s1B, s2Bt = (T)s2B, preft = (T)geo.pref;
    const int nseq = 1 << lgs;
    // Row k per thread (consecutive k across the lanes): the row invariants
    // are read once and serve every column of the tile; the family-2 values
    // come from the transposed copy [par][t][k1][k0], contiguous in k0 = kx.
    const T *Pt = d == 3 ? static_cast<const T *>(a.sh.P2T) + ((kB & 1) ? 3 * ss2 : 0) : nullptr;
    for (int k = tid; k <= M; k += NTT) {
        if (k == 0 || k == M) {
            for (int sq = 0; sq < nseq; ++sq) lds_cs(buf, rs, k, sq, cx<T>{(T)0, (T)0});
            continue;
        }
        T r[SV];
        load12(rv + (k - 1) * SV, r);
        const T lx = r[0], rq = r[1], rs1 = r[2], rs2 = r[3], r10 = r[10], r11 = r[11];
        // family 1 at (kx, kz) for even / odd ky
        const T Pe0 = r[4], Pe1 = r[5], Pe2 = r[6], Po0 = r[7], Po1 = r[8], Po2 = r[9];
        const int kx = k;
        const bool kodd = (kx & 1) != 0; // family 0 at (ky, kz): parity of kx
        for (int sq = 0; sq < nseq; ++sq) {
            const cx<T> z1 = lds_c(buf, rs, k, sq), z2 = lds_c(buf, rs, N - k, sq);
            T cab[2];
            // the spectrum as loaded (pre), or from the forward transform
            const T beta2[2] = {a.pre ? z1.x : (T)0.5 * (z2.y - z1.y), a.pre ? z1.y : (T)0.5 * (z1.x - z2.x)};
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {
                const int c = 2 * sq + h2;
                T cval = (T)0;
                if (c < nc) {
                    const int ky = 1 + c0 + c; // c0 is even: ky is odd for h2 = 0
                    T q1[SV];
                    load12(cv + c * SV, q1);
                    const T P0 = h2 ? Pe0 : Po0, P1v = h2 ? Pe1 : Po1, P2v = h2 ? Pe2 : Po2;
                    const T Pc[3] = {kodd ? q1[7] : q1[4], kodd ? q1[8] : q1[5], kodd ? q1[9] : q1[6]};
                    const T ly = q1[0], lxy = lx * ly;
                    const T Lm = r10 + q1[10] + lamBt + c2xy * lxy;
                    T gt = rs1 * Pc[0] + q1[2] * P0;
                    T dh = (T)0;
                    if (six) dh = rs1 * Pc[1] + rs2 * Pc[2] + q1[2] * P1v + q1[3] * P2v;
                    if (d == 3) {
                        const T *Pe = Pt + (int64_t)(ky - 1) * I0 + (kx - 1);
                        gt += s1Bt * Pe[0];
                        if (six) dh += s1Bt * Pe[ss2] + s2Bt * Pe[2 * ss2];
                    }
                    const T iL = recip(Lm);
                    T harm;
                    if (six) {
                        const T Rm = r11 + q1[11] + lxy * (c4xy * lx + c4yx * ly);
                        harm = (gt * ((T)1 + Rm * iL) + dh) * iL;
                    } else {
                        harm = gt * iL;
                    }
                    cval = preft * (harm - beta2[h2] * recip(rq + q1[1]));
                }
                cab[h2] = cval;
            }
            lds_cs(buf, rs, k, sq, cx<T>{cab[1], -cab[0]});
            lds_cs(buf, rs, N - k, sq, cx<T>{-cab[1], cab[0]});
        }
    }
    __syncthreads();
    if (direct) {
        if constexpr (DIO) {
            fft_ct_head<T, NTT, NC, WC + 1, LGSC, true>(buf, tw, tid);
            stage_ct_gout<T, T, NTT, NC, WC + 1, LGSC>(buf, tw, g, 1, a.nrows_in, nc, a.irs, a.ics, (T)0.5, tid);
        }
    } else {
        fft_tile<T, MAXE, NTT, P2>(buf, rs, lgs, fd, tw, true, tid);
        tile_store<T, T, NTT>(buf, rs, 1, g, a.nrows_in, nc, a.irs, a.ics, (T)0.5, lgW, tid);
    }
    if constexpr (!PF) break; // one tile per block: no loop for the compiler to hoist out of
    __syncthreads();          // the next tile reuses the LDS
    }
}

template <typename T, int MAXE, bool P2, int WC, int NTT = NT, int NC = 0>
static void launch_final_n(const FinalArgs &a, int nblk, size_t lds, hipStream_t st)
{
    const void *fn = (const void *)&k_final<T, MAXE, P2, WC, NTT, NC>;
    set_lds(fn, lds);
    int grid = nblk;
    if (WC > 0 && NTT == NT && sizeof(T) == 8 && NC == 0) { // persistent blocks (PF in k_final)
        const int r = resident_blocks(fn, NTT, lds);
        if (r > 0 && r < nblk) grid = r;
    }
    hipLaunchKernelGGL((k_final<T, MAXE, P2, WC, NTT, NC>), dim3(grid), dim3(NTT), lds, st, a, nblk);
}

// Compile-time widths 4, 8, 16 of the default tile budget (N WC / 2 = 8 NT):
// the transform length at compile time too when it is the plan's.
template <typename T, int MAXE, bool P2, int WC, int NTT = NT>
static void launch_final_w(const FinalArgs &a, int nblk, size_t lds, hipStream_t st)
{
    constexpr int NCT = (MAXE == 8 && P2 && NTT == NT && (WC == 4 || WC == 8 || WC == 16)) ? 16 * NT / WC : 0;
    if constexpr (NCT > 0)
        if (a.fd.N == NCT) return launch_final_n<T, MAXE, P2, WC, NTT, NCT>(a, nblk, lds, st);
    launch_final_n<T, MAXE, P2, WC, NTT>(a, nblk, lds, st);
}

template <typename T, int MAXE, bool P2>
static void launch_final_k(const FinalArgs &a, int nblk, hipStream_t st)
{
    // tile + staged column (W) invariants, 12 values of type T each (the row
    // invariants are in the global row table)
    const size_t lds = tile_lds<T>(a.fd.N, a.W) + 16 + (size_t)a.W * 12 * sizeof(T);
    // compile-time widths also prefetch the next tile: MAXE registers per
    // thread must cover the tile's rows
    const bool rc = a.irs == 1 && a.ics != 1;
    if (a.W == 8 && PairMap<NT, 8, MAXE>::covers(a.nrows_in, rc))
        launch_final_w<T, MAXE, P2, 8>(a, nblk, lds, st);
    else if (a.W == 16 && PairMap<NT, 16, MAXE>::covers(a.nrows_in, rc))
        launch_final_w<T, MAXE, P2, 16>(a, nblk, lds, st);
    else if (a.W == 32 && PairMap<NT, 32, MAXE>::covers(a.nrows_in, rc))
        launch_final_w<T, MAXE, P2, 32>(a, nblk, lds, st);
    else
        launch_final_w<T, MAXE, P2, 0>(a, nblk, lds, st);
}

template <typename T>
static void launch_final_t(const FinalArgs &a, int nblk, int work, hipStream_t st)
{
    const bool p2 = is_pow2(a.fd.N);
    if (big_fft(a.fd.N)) {
        // tile + staged columns only (the rows come from the global table)
        const size_t lds = tile_lds<T>(a.fd.N, a.W) + 16 + (size_t)a.W * 12 * sizeof(T);
        if (work <= 4 * NTB) {
            if (p2)
                launch_final_w<T, 4, true, 2, NTB>(a, nblk, lds, st);
            else
                launch_final_w<T, 4, false, 2, NTB>(a, nblk, lds, st);
        } else {
            if (p2)
                launch_final_w<T, 8, true, 2, NTB>(a, nblk, lds, st);
            else
                launch_final_w<T, 8, false, 2, NTB>(a, nblk, lds, st);
        }
        return;
    }
    if (work <= 4 * NT) {
        if (p2)
            launch_final_k<T, 4, true>(a, nblk, st);
        else
            launch_final_k<T, 4, false>(a, nblk, st);
    } else if (work <= 8 * NT) {
        if (p2)
            launch_final_k<T, 8, true>(a, nblk, st);
        else
            launch_final_k<T, 8, false>(a, nblk, st);
    } else if (work <= 16 * NT) {
        if (p2)
            launch_final_k<T, 16, true>(a, nblk, st);
        else
            launch_final_k<T, 16, false>(a, nblk, st);
    } else {
        if (p2)
            launch_final_k<T, 32, true>(a, nblk, st);
        else
            launch_final_k<T, 32, false>(a, nblk, st);
    }
}

// Row table of the final pass in global memory, one per batch index
// (rowtab[kB - 1][kx - 1][12]); 2D has a single batch index.
__global__ void k_final_rows(FinalArgs a)
{
    const int I0 = a.geo.M[0] - 1;
    const int64_t tot = (int64_t)I0 * a.nbatch;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % I0), b = (int)(e / I0);
        const int kB = b + 1;
        double lamB = 0.0, qB = 0.0;
        if (a.geo.d == 3) {
            lamB = a.tab[2].lam[kB - 1];
            qB = a.tab[2].q[kB - 1];
        }
        if (a.mixed)
            final_row<float>(a, i, kB, lamB, qB, static_cast<float *>(a.rowtab) + e * 12);
        else
            final_row<double>(a, i, kB, lamB, qB, static_cast<double *>(a.rowtab) + e * 12);
    }
}

hipError_t launch_final_rows(const FinalArgs &a, hipStream_t st)
{
    if (!a.rowtab) return hipErrorInvalidValue;
    const int64_t tot = (int64_t)(a.geo.M[0] - 1) * a.nbatch;
    const unsigned nb = (unsigned)std::min<int64_t>((tot + NT - 1) / NT, 4096);
    hipLaunchKernelGGL(k_final_rows, dim3(nb), dim3(NT), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_final(const FinalArgs &a, hipStream_t st)
{
    const int ncb = (a.ncols + a.W - 1) / a.W;
    const int nblk = ncb * a.nbatch;
    const int work = (a.W / 2) * a.fd.N;
    if (!a.rowtab) return hipErrorInvalidValue; // the row invariants are read from it
    if (big_fft(a.fd.N) && (a.geo.d != 2 || a.W != 2 || work > 8 * NTB))
        return hipErrorInvalidValue;
    if (!big_fft(a.fd.N) && work > 32 * NT) return hipErrorInvalidValue;
    if (!tile_strides_ok(a.nrows_in, a.irs, a.ncols, a.ics)) return hipErrorInvalidValue;
    if (a.mixed)
        launch_final_t<float>(a, nblk, work, st);
    else
        launch_final_t<double>(a, nblk, work, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Kernel samples for the boundary convolutions: for faces normal to axis a,
// K[dd][ib][ic] = G(sqrt(((dd+1) h_a)^2 + (ib h_b)^2 + (ic h_c)^2)),
// dd = 0..M_a-2, ib = 0..M_b, ic = 0..M_c  (2D: K[dd][ib]).
// ---------------------------------------------------------------------------
__global__ void k_ksample(double *out, int d, int a, int b, int c, int Ma, int Mb, int Mc,
                          double ha, double hb, double hc)
{
    const int64_t nb = Mb + 1, ncn = d == 3 ? Mc + 1 : 1;
    const int64_t tot = (int64_t)(Ma - 1) * nb * ncn;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int ic = (int)(e % ncn);
        const int ib = (int)((e / ncn) % nb);
        const int dd = (int)(e / (ncn * nb));
        const double x = (dd + 1) * ha, y = ib * hb, z = ic * hc;
        const double r = sqrt(x * x + y * y + (d == 3 ? z * z : 0.0));
        double G;
        if (d == 3)
            G = -1.0 / (4.0 * M_PI * r);
        else
            G = log(r) / (2.0 * M_PI);
        out[e] = G;
    }
}

hipError_t launch_ksample(double *out, int d, int a, int b, int c, const int *M, const double *h,
                          hipStream_t st)
{
    const int64_t tot = (int64_t)(M[a] - 1) * (M[b] + 1) * (d == 3 ? M[c] + 1 : 1);
    const int nb = (int)std::min<int64_t>((tot + NT - 1) / NT, 65536);
    hipLaunchKernelGGL(k_ksample, dim3(nb), dim3(NT), 0, st, out, d, a, b, c, M[a], M[b],
                       d == 3 ? M[c] : 0, h[a], h[b], d == 3 ? h[c] : 0.0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 1D: phi* by one sine-transform pencil, end values by direct sums of
// G(r) = r/2, phi_H linear between them.
// ---------------------------------------------------------------------------
// screen != 0: the end values come from the screening charge instead: with the
// sine coefficients alpha_k of phi*, sigma_lo = -sum (pi k/L) alpha_k and
// sigma_hi = sum (pi k/L)(-1)^k alpha_k are the outward derivatives at the two
// ends and g(x) = sum over both ends of G(|x - end|) sigma, i.e.
// g_0 = (L/2) sigma_hi and g_M = (L/2) sigma_lo (G = r/2 vanishes at r = 0).
template <int MAXE, int NTT>
__global__ __launch_bounds__(NTT) void k_1d(const double *rho, double *phi, int M, double h,
                                            FftDesc fd, const cx<double> *twg, AxisTabs tab, int screen)
{
    constexpr bool BIG = NTT != NT;
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = fd.N, rs = BIG ? 2 : 3, lgW = 1;
    const cx<double> *tw = BIG ? twg : reinterpret_cast<const cx<double> *>(smem);
    double *buf = reinterpret_cast<double *>(smem + (BIG ? 0 : (size_t)N * sizeof(cx<double>)));
    __shared__ double red[2][NTT];
    if (!BIG) load_twiddles<double, NTT>(reinterpret_cast<cx<double> *>(smem), twg, N);
    // end values
    double s0 = 0.0, s1 = 0.0;
    for (int j = 1 + threadIdx.x; j < M; j += NTT) {
        s0 += (0.5 * j * h) * rho[j];
        s1 += (0.5 * (M - j) * h) * rho[j];
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    zero_rows<double, NTT>(buf, rs, lgW, 0, 1);
    zero_rows<double, NTT>(buf, rs, lgW, M, N);
    tile_load<double, double, NTT>(buf, rs, 1, rho + 1, M - 1, 1, 1, 1, lgW);
    __syncthreads();
    for (int w = NTT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    double g0 = h * red[0][0], g1 = h * red[1][0];
    fft_tile<double, MAXE, NTT>(buf, rs, 0, fd, tw, false);
    post_cs<double, MAXE, NTT>(buf, rs, 0, M);
    __syncthreads();
    double slo = 0.0, shi = 0.0;
    const double L = M * h, piL = 3.14159265358979323846264338327950288 / L;
    for (int k = 1 + threadIdx.x; k < M; k += NTT) {
        const double al = -(2.0 / M) * buf[(M + k) * rs] / tab.q[k - 1];
        buf[(M + k) * rs] = al;
        const double t = (k * piL) * al;
        slo -= t;
        shi += (k & 1) ? -t : t;
    }
    if (screen) {
        red[0][threadIdx.x] = slo;
        red[1][threadIdx.x] = shi;
        __syncthreads();
        for (int w = NTT / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                red[0][threadIdx.x] += red[0][threadIdx.x + w];
                red[1][threadIdx.x] += red[1][threadIdx.x + w];
            }
            __syncthreads();
        }
        g0 = 0.5 * L * red[1][0];
        g1 = 0.5 * L * red[0][0];
    }
    __syncthreads();
    pre_herm<double, MAXE, NTT>(buf, rs, 0, M, true);
    fft_tile<double, MAXE, NTT>(buf, rs, 0, fd, tw, true);
    for (int j = threadIdx.x; j <= M; j += NTT) {
        double v;
        if (j == 0)
            v = g0;
        else if (j == M)
            v = g1;
        else
            v = 0.5 * buf[j * rs] + g0 + (g1 - g0) * ((double)j / M);
        phi[j] = v;
    }
}

hipError_t launch_1d(const double *rho, double *phi, int M, double h, const FftDesc &fd,
                     const cx<double> *tw, const AxisTabs &tab, int screen, hipStream_t st)
{
    const size_t lds = tile_lds<double>(fd.N, 2);
    if (big_fft(fd.N)) {
        if (fd.N > 8 * NTB) return hipErrorInvalidValue;
        if (fd.N <= 4 * NTB) {
            set_lds((const void *)&k_1d<4, NTB>, lds);
            hipLaunchKernelGGL((k_1d<4, NTB>), dim3(1), dim3(NTB), lds, st, rho, phi, M, h, fd, tw, tab, screen);
        } else {
            set_lds((const void *)&k_1d<8, NTB>, lds);
            hipLaunchKernelGGL((k_1d<8, NTB>), dim3(1), dim3(NTB), lds, st, rho, phi, M, h, fd, tw, tab, screen);
        }
    } else if (fd.N <= 4 * NT) {
        set_lds((const void *)&k_1d<4, NT>, lds);
        hipLaunchKernelGGL((k_1d<4, NT>), dim3(1), dim3(NT), lds, st, rho, phi, M, h, fd, tw, tab, screen);
    } else if (fd.N <= 8 * NT) {
        set_lds((const void *)&k_1d<8, NT>, lds);
        hipLaunchKernelGGL((k_1d<8, NT>), dim3(1), dim3(NT), lds, st, rho, phi, M, h, fd, tw, tab, screen);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace ips
