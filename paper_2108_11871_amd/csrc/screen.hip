// Boundary values from the screening charge (James-type methods, Sections 1
// and 2), the alternative to the volume sums of Section 4:
//   g(x) = surface integral of G(|x - s|) sigma(s) dS(s),  sigma = d phi*/dn,
// sigma from the sine coefficients alpha of phi* (Section 3).
//   k_sigma_rows, k_sigma_cols : face sine coefficients of sigma, sums over
//                  the normal wavenumber
//   k_screen_src : the weighted surface nodes (position, W sigma) of every face
//   k_screen_g   : the corrected surface trapezoidal sums at every boundary node
//                  (direct sums)
//   k_face_charge, k_par_mul, k_perp_mfma / k_perp, k_surf_assemble : the same sums in 3D by
//                  transforms (with the slot passes of the plan)
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace ips {

namespace {

// Gregory end factors of the trapezoid weights on nodes 0..M (M >= 6):
// 3/8, 7/6, 23/24 from each end, 1 elsewhere.
__device__ __forceinline__ double gregory(int i, int M)
{
    const int e = i < M - i ? i : M - i;
    if (e == 0) return 3.0 / 8.0;
    if (e == 1) return 7.0 / 6.0;
    if (e == 2) return 23.0 / 24.0;
    return 1.0;
}

// 1/sqrt(x) from the hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return y;
}

__device__ __forceinline__ int64_t face_elems(const ScreenArgs &a, int fam)
{
    int64_t s = 1;
    for (int b = 0; b < a.d; ++b)
        if (b != fam) s *= a.M[b] - 1;
    return s;
}

} // namespace

// ---------------------------------------------------------------------------
// Face coefficients of sigma.  Y holds the raw sine spectrum of rho_I over all
// axes, Y[(k2 I0 + k0) I1 + k1] (3D) or Y[k0 I1 + k1] (2D), so that
// alpha_k = -pref Y_k / q(k), q = sum_a (pi k_a/L_a)^2.  For the faces normal
// to axis a:
//   S[a][0][k_other] = -sum_{k_a} (pi k_a/L_a) alpha_k          (face x_a = lo)
//   S[a][1][k_other] =  sum_{k_a} (pi k_a/L_a) (-1)^{k_a} alpha_k (face x_a = hi)
// stored as [side][k_b - 1][k_c - 1], the other axes in increasing order.
// k_sigma_rows takes the family whose sum runs over the contiguous axis
// (a = 1): one wave per output pair, its lanes stride over k_1 and reduce by
// shuffles; k_sigma_cols takes the others.  Both issue kSigU loads per lane
// before using them.
// ---------------------------------------------------------------------------
constexpr int kSigU = 8;

__global__ __launch_bounds__(NT) void k_sigma_rows(ScreenArgs a, int64_t nout)
{
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
    if (w >= nout) return;
    const int I0 = a.M[0] - 1, I1 = a.M[1] - 1;
    // face layout of family 1: [side][k0][k2] (3D) or [side][k0]
    int k0, k2 = 1;
    if (a.d == 3) {
        const int I2 = a.M[2] - 1;
        k0 = 1 + (int)(w / I2);
        k2 = 1 + (int)(w % I2);
    } else {
        k0 = 1 + (int)w;
    }
    const double *row = a.Y + (a.d == 3 ? ((int64_t)(k2 - 1) * I0 + (k0 - 1)) * I1 : (int64_t)(k0 - 1) * I1);
    double qo = a.tab[0].q[k0 - 1];
    if (a.d == 3) qo += a.tab[2].q[k2 - 1];
    double lo = 0.0, hi = 0.0;
    for (int base = 1 + lane; base <= I1; base += 64 * kSigU) {
        double y[kSigU];
#pragma unroll
        for (int u = 0; u < kSigU; ++u) {
            const int k1 = base + 64 * u;
            y[u] = k1 <= I1 ? row[k1 - 1] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kSigU; ++u) {
            const int k1 = base + 64 * u;
            if (k1 <= I1) {
                const double alpha = -a.pref * y[u] / (qo + a.tab[1].q[k1 - 1]);
                const double t = (k1 * a.piL[1]) * alpha;
                lo -= t;
                hi += (k1 & 1) ? -t : t;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo += __shfl_xor(lo, off);
        hi += __shfl_xor(hi, off);
    }
    if (lane == 0) {
        a.S[1][w] = lo;
        a.S[1][nout + w] = hi;
    }
}

// ---------------------------------------------------------------------------
// Surface nodes: for every face (axis a, side) and every node inside it,
// position (origin at grid node 0) and weight W sigma, W the product of the
// Gregory-corrected trapezoid weights h_b gamma(i_b) of the in-face axes.
// src[0..2][j] = coordinates, src[3][j] = W sigma; faces in the order
// (a = 0 lo, a = 0 hi, a = 1 lo, ...), nodes in face layout order.
// ---------------------------------------------------------------------------
__global__ void k_screen_src(ScreenArgs a)
{
    const int64_t tot = a.nsrc;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < tot; j += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = j;
        int fam = 0, side = 0;
        for (;; ++fam) {
            const int64_t fe = face_elems(a, fam);
            if (r < 2 * fe) {
                side = (int)(r / fe);
                r -= side * fe;
                break;
            }
            r -= 2 * fe;
        }
        int i[3] = {0, 0, 0};
        i[fam] = side ? a.M[fam] : 0;
        if (a.d == 3) {
            const int b = fam == 0 ? 1 : 0, c = fam == 2 ? 1 : 2;
            const int Ic = a.M[c] - 1;
            i[b] = 1 + (int)(r / Ic);
            i[c] = 1 + (int)(r % Ic);
        } else {
            i[1 - fam] = 1 + (int)r;
        }
        double W = 1.0;
        for (int b = 0; b < a.d; ++b)
            if (b != fam) W *= a.h[b] * gregory(i[b], a.M[b]);
        const double sig = a.sig[fam][(int64_t)side * face_elems(a, fam) + r];
        for (int b = 0; b < 3; ++b) a.src[(int64_t)b * tot + j] = b < a.d ? i[b] * a.h[b] : 0.0;
        a.src[3 * tot + j] = W * sig;
    }
}

// ---------------------------------------------------------------------------
// g at every boundary node: the sum over all surface nodes of (W sigma) G(r),
// the target itself left out, plus tau_a sigma(x) when x lies inside a face of
// axis a.  One target per thread; the surface nodes stream through LDS.
// Boundary nodes are enumerated without repetition: the two axis-0 faces
// whole, then the axis-1 faces without axis-0 edges, then (3D) the axis-2
// faces without the edges of the other two.
// ---------------------------------------------------------------------------
constexpr int kSrcChunk = 512;

__global__ __launch_bounds__(NT) void k_screen_g(ScreenArgs a, double *phi)
{
    __shared__ double sx[kSrcChunk], sy[kSrcChunk], sz[kSrcChunk], sw[kSrcChunk];
    const int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x;
    const int d = a.d;
    const int64_t n0 = a.M[0] + 1, n1 = a.M[1] + 1, n2 = d == 3 ? a.M[2] + 1 : 1;
    // decode the boundary node of this thread
    int i[3] = {0, 0, 0};
    bool live = t < a.ntgt;
    if (live) {
        int64_t r = t;
        const int64_t f0 = n1 * n2;                 // one axis-0 face
        const int64_t f1 = (n0 - 2) * n2;           // one axis-1 face without axis-0 edges
        if (r < 2 * f0) {
            i[0] = r < f0 ? 0 : a.M[0];
            r %= f0;
            i[1] = (int)(r / n2);
            i[2] = (int)(r % n2);
        } else if ((r -= 2 * f0) < 2 * f1) {
            i[1] = r < f1 ? 0 : a.M[1];
            r %= f1;
            i[0] = 1 + (int)(r / n2);
            i[2] = (int)(r % n2);
        } else {
            r -= 2 * f1;
            const int64_t f2 = (n0 - 2) * (n1 - 2);
            i[2] = r < f2 ? 0 : a.M[2];
            r %= f2;
            i[0] = 1 + (int)(r / (n1 - 2));
            i[1] = 1 + (int)(r % (n1 - 2));
        }
    }
    const double x = i[0] * a.h[0], y = i[1] * a.h[1], z = d == 3 ? i[2] * a.h[2] : 0.0;
    double acc = 0.0;
    for (int64_t c0 = 0; c0 < a.nsrc; c0 += kSrcChunk) {
        const int nc = (int)min((int64_t)kSrcChunk, a.nsrc - c0);
        __syncthreads();
        for (int j = threadIdx.x; j < nc; j += NT) {
            sx[j] = a.src[c0 + j];
            sy[j] = a.src[a.nsrc + c0 + j];
            sz[j] = a.src[2 * a.nsrc + c0 + j];
            sw[j] = a.src[3 * a.nsrc + c0 + j];
        }
        __syncthreads();
        if (!live) continue;
        if (d == 3) {
            for (int j = 0; j < nc; ++j) {
                const double dx = x - sx[j], dy = y - sy[j], dz = z - sz[j];
                const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                if (r2 > 0.0) acc = fma(sw[j], rsqrt_nr(r2), acc);
            }
        } else {
            for (int j = 0; j < nc; ++j) {
                const double dx = x - sx[j], dy = y - sy[j];
                const double r2 = fma(dx, dx, dy * dy);
                if (r2 > 0.0) acc = fma(sw[j], log(r2), acc);
            }
        }
    }
    if (!live) return;
    // 3D: G = -1/(4 pi r); 2D: G = log(r)/(2 pi) = log(r^2)/(4 pi)
    constexpr double inv4pi = 0.0795774715459476678844418816862571810;
    double g = d == 3 ? -inv4pi * acc : inv4pi * acc;
    // singular correction inside a face (sigma vanishes on the face edges)
    int nb = 0, fam = -1;
    for (int b = 0; b < d; ++b)
        if (i[b] == 0 || i[b] == a.M[b]) {
            ++nb;
            fam = b;
        }
    if (nb == 1) {
        const int side = i[fam] == 0 ? 0 : 1;
        int64_t r;
        if (d == 3) {
            const int b = fam == 0 ? 1 : 0, c = fam == 2 ? 1 : 2;
            r = (int64_t)(i[b] - 1) * (a.M[c] - 1) + (i[c] - 1);
        } else {
            r = i[1 - fam] - 1;
        }
        g += a.tau[fam] * a.sig[fam][(int64_t)side * face_elems(a, fam) + r];
    }
    phi[((int64_t)i[0] * n1 + i[1]) * n2 + i[2]] = g;
}

// ---------------------------------------------------------------------------
// Fast evaluation of the 3D surface sums.  With f_(f,s) = W sigma on face
// (axis f, side s) -- all nodes, zero on the edges -- a boundary node x owned
// by face (a, s) (a the lowest axis with x on its boundary) receives
//   P_a[s](x)        from the two faces of axis a: 2D convolutions over the
//                    face axes with G at in-plane distance (same face, the
//                    origin left out) or at distance L_a (opposite face),
//                    by zero-padded slot transforms (circulant length 2M);
//   Q_(a<-b)[s](x)   from the two faces of each other axis b: the two faces
//                    share the third axis c, so this is a convolution along c
//                    and, per wavenumber of c, a dense product over the other
//                    coordinates with the table KT[k][i][j] of G at
//                    (i h_a, j h_b) transformed along c;
// plus the singular correction tau_a sigma(x) inside a face.  Every source
// face enters every target once, which is the sum of the direct rule.
// ---------------------------------------------------------------------------
namespace {

__device__ __forceinline__ void face_axes(int f, int &b, int &c)
{
    b = f == 0 ? 1 : 0;
    c = f == 2 ? 1 : 2;
}

__device__ __forceinline__ void pair_axes(int pr, int &a, int &b, int &c)
{
    a = pr == 2 ? 1 : 0;
    b = pr == 0 ? 1 : 2;
    c = 3 - a - b;
}

__device__ __forceinline__ double green3(double r2)
{
    constexpr double inv4pi = 0.0795774715459476678844418816862571810;
    return r2 > 0.0 ? -inv4pi * rsqrt_nr(r2) : 0.0;
}

} // namespace

__global__ void k_par_sample(double *out, int Mb, int Mc, double hb, double hc, double La)
{
    const int64_t nb = Mb + 1, nc = Mc + 1, tot = 2 * nb * nc;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(e / (nb * nc));
        const int ib = (int)((e / nc) % nb), ic = (int)(e % nc);
        const double x = ib * hb, y = ic * hc, z = t ? La : 0.0;
        out[e] = green3(fma(x, x, fma(y, y, z * z)));
    }
}

hipError_t launch_par_sample(double *out, int f, const int *M, const double *h, hipStream_t st)
{
    const int b = f == 0 ? 1 : 0, c = f == 2 ? 1 : 2;
    const int64_t tot = 2 * (int64_t)(M[b] + 1) * (M[c] + 1);
    const unsigned nbk = (unsigned)std::min<int64_t>((tot + NT - 1) / NT, 65535);
    hipLaunchKernelGGL(k_par_sample, dim3(nbk), dim3(NT), 0, st, out, M[b], M[c], h[b], h[c], M[f] * h[f]);
    return hipGetLastError();
}

__global__ void k_perp_sample(double *out, int Ma, int Mb, int Mc, double ha, double hb, double hc)
{
    const int64_t na = Ma + 1, nb = Mb + 1, tot = (int64_t)(Mc + 1) * na * nb;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int dc = (int)(e / (na * nb));
        const int i = (int)((e / nb) % na), j = (int)(e % nb);
        const double x = i * ha, y = j * hb, z = dc * hc;
        out[e] = green3(fma(x, x, fma(y, y, z * z)));
    }
}

hipError_t launch_perp_sample(double *out, int a, int b, int c, const int *M, const double *h, hipStream_t st)
{
    const int64_t tot = (int64_t)(M[c] + 1) * (M[a] + 1) * (M[b] + 1);
    const unsigned nbk = (unsigned)std::min<int64_t>((tot + NT - 1) / NT, 65535);
    hipLaunchKernelGGL(k_perp_sample, dim3(nbk), dim3(NT), 0, st, out, M[a], M[b], M[c], h[a], h[b], h[c]);
    return hipGetLastError();
}

// f = W sigma on every node of every face (zero on the face edges)
__global__ void k_face_charge(SurfArgs s)
{
    const int f = blockIdx.y;
    int b, c;
    face_axes(f, b, c);
    const int nb = s.M[b] + 1, nc = s.M[c] + 1, Ib = s.M[b] - 1, Ic = s.M[c] - 1;
    const int64_t tot = 2 * (int64_t)nb * nc;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int side = (int)(e / ((int64_t)nb * nc));
        const int ib = (int)((e / nc) % nb), ic = (int)(e % nc);
        double v = 0.0;
        if (ib > 0 && ib < s.M[b] && ic > 0 && ic < s.M[c]) {
            const double W = s.h[b] * gregory(ib, s.M[b]) * s.h[c] * gregory(ic, s.M[c]);
            v = W * s.sig[f][((int64_t)side * Ib + (ib - 1)) * Ic + (ic - 1)];
        }
        s.FA[f][e] = v;
    }
}

hipError_t launch_face_charge(const SurfArgs &s, hipStream_t st)
{
    int64_t mx = 0;
    for (int f = 0; f < 3; ++f) {
        const int b = f == 0 ? 1 : 0, c = f == 2 ? 1 : 2;
        mx = std::max(mx, 2 * (int64_t)(s.M[b] + 1) * (s.M[c] + 1));
    }
    const unsigned nbk = (unsigned)std::min<int64_t>((mx + NT - 1) / NT, 65535);
    hipLaunchKernelGGL(k_face_charge, dim3(nbk, 3), dim3(NT), 0, st, s);
    return hipGetLastError();
}

// slot spectra of the two faces of axis f times the kernel spectra, in place:
// side s receives K_same X_s + K_opp X_(1-s).  Slot r of an axis with M panels
// carries wavenumber r (r <= M, cosine) or r - M (sine).
__global__ void k_par_mul(SurfArgs s)
{
    const int f = blockIdx.y;
    int b, c;
    face_axes(f, b, c);
    const int Mb = s.M[b], Mc = s.M[c], Nb = 2 * Mb, Nc = 2 * Mc;
    const int64_t plane = (int64_t)Nb * Nc, kp = (int64_t)(Mb + 1) * (Mc + 1);
    double *X = s.XH[f];
    const double *K = s.KP[f];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < plane; e += (int64_t)gridDim.x * blockDim.x) {
        const int rb = (int)(e / Nc), rc = (int)(e % Nc);
        const int kb = rb <= Mb ? rb : rb - Mb, kc = rc <= Mc ? rc : rc - Mc;
        const double ks = K[(int64_t)kb * (Mc + 1) + kc], ko = K[kp + (int64_t)kb * (Mc + 1) + kc];
        const double x0 = X[e], x1 = X[plane + e];
        X[e] = fma(ks, x0, ko * x1);
        X[plane + e] = fma(ko, x0, ks * x1);
    }
}

hipError_t launch_par_mul(const SurfArgs &s, hipStream_t st)
{
    int64_t mx = 0;
    for (int f = 0; f < 3; ++f) {
        const int b = f == 0 ? 1 : 0, c = f == 2 ? 1 : 2;
        mx = std::max(mx, 4 * (int64_t)s.M[b] * s.M[c]);
    }
    const unsigned nbk = (unsigned)std::min<int64_t>((mx + NT - 1) / NT, 65535);
    hipLaunchKernelGGL(k_par_mul, dim3(nbk, 3), dim3(NT), 0, st, s);
    return hipGetLastError();
}

// Perpendicular pairs.  Block (k, g): wavenumber k of the shared axis c of
// pair (a, b), both slots (cosine k, sine k), and the table rows i of row
// group g.  With i = |s M_a - u| and j = |t - s' M_b| (u = i or M_a - i by the
// side s of face a, t = j or M_b - j by the side s' of face b):
//   targets on face (a, s), node t:   sum over (s', u) of KT[k][i][j] XB[s'][u]
//   targets on face (b, s'), node u:  sum over (s, t) of KT[k][i][j] XA[s][t]
// The first sum runs over the rows of every group: each block writes its
// partial for every target, one copy per (group, s') -- the inverse transform
// adds the copies.  The second is complete within a row; the row of side
// s = 0 and that of s = 1 land in two copies.  Rows of KT[k] stream through
// LDS in tiles, the next tile held in registers while the current one is
// used (two tiles in flight); threads own columns j for the first sum, waves
// own rows for the second.
// Slot-major layouts: X*[q][side][node], partials PA[q][2 G][2][M_b + 1]
// (copy g * 2 + s', then s) and PB[q][2][2][M_a + 1] (copy s, then s').
constexpr int kPerpJpt = 3; // columns per thread: M_b + 1 <= 3 * NT
constexpr int kPerpPf = 8; // table elements per thread in each of the two prefetch buffers:
                            // tile rows * (M_b + 1) <= 8 * NT

bool perp_fits(const int *M)
{
    for (int a = 0; a < 3; ++a)
        if (M[a] + 1 > kPerpJpt * NT) return false;
    return true;
}

int perp_groups(const int *M, int pr)
{
    const int a = pr == 2 ? 1 : 0, b = pr == 0 ? 1 : 2, c = 3 - a - b;
    (void)b;
    // about 1024 blocks per launch, at least 8 rows per group
    const int want = (1024 + M[c]) / (M[c] + 1);
    return std::max(1, std::min(want, (M[a] + 1) / 8));
}

static size_t perp_lds_bytes(const int *M, int pr)
{
    const int a = pr == 2 ? 1 : 0, b = pr == 0 ? 1 : 2;
    // xa, xb, the tile
    return (size_t)(4 * (M[b] + 1) + 4 * (M[a] + 1) + kPerpPf * NT) * sizeof(double);
}

__global__ __launch_bounds__(NT) void k_perp(SurfArgs s, int pr)
{
    extern __shared__ __align__(16) unsigned char smem[];
    int a, b, c;
    pair_axes(pr, a, b, c);
    const int Ma = s.M[a], Mb = s.M[b], Mc = s.M[c];
    const int na = Ma + 1, nb = Mb + 1;
    const int k = blockIdx.x, g = blockIdx.y, G = gridDim.y;
    const bool two = k > 0 && k < Mc; // the sine slot exists
    const int q0 = k, q1 = Mc + k;
    const int ibeg = (int)((int64_t)g * na / G), iend = (int)((int64_t)(g + 1) * na / G);
    const int rows = kPerpPf * NT / nb;
    double *xa = reinterpret_cast<double *>(smem); // [2][nb][2 slots]
    double *xb = xa + 4 * nb;                      // [2][na][2 slots]
    double *tile = xb + 4 * na;                    // [rows][nb]
    const double *XA = s.XA[pr], *XB = s.XB[pr];
    const double *slab = s.KT[pr] + (int64_t)k * na * nb;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double pfa[kPerpPf], pfb[kPerpPf];
    auto fetch = [&](double(&pf)[kPerpPf], int i0) {
        const int cnt = min(rows, iend - i0) * nb;
        const double *src = slab + (int64_t)i0 * nb;
#pragma unroll
        for (int m = 0; m < kPerpPf; ++m) {
            const int e = threadIdx.x + m * NT;
            if (e < cnt) pf[m] = src[e];
        }
    };
    auto put = [&](const double(&pf)[kPerpPf], int nr) {
#pragma unroll
        for (int m = 0; m < kPerpPf; ++m) {
            const int e = threadIdx.x + m * NT;
            if (e < nr * nb) tile[e] = pf[m];
        }
    };
    // the first two tiles are requested before anything else
    if (ibeg < iend) fetch(pfa, ibeg);
    if (ibeg + rows < iend) fetch(pfb, ibeg + rows);
    for (int e = threadIdx.x; e < 2 * nb; e += NT) {
        xa[2 * e] = XA[(int64_t)q0 * 2 * nb + e];
        xa[2 * e + 1] = two ? XA[(int64_t)q1 * 2 * nb + e] : 0.0;
    }
    for (int e = threadIdx.x; e < 2 * na; e += NT) {
        xb[2 * e] = XB[(int64_t)q0 * 2 * na + e];
        xb[2 * e + 1] = two ? XB[(int64_t)q1 * 2 * na + e] : 0.0;
    }
    double acc[kPerpJpt][2][2][2]; // [column][target side s][source side s'][slot]
#pragma unroll
    for (int jj = 0; jj < kPerpJpt; ++jj)
#pragma unroll
        for (int v = 0; v < 8; ++v) (&acc[jj][0][0][0])[v] = 0.0;
    double *PB = s.PB[pr];
    const int64_t pbq = 4 * (int64_t)na;
    auto work = [&](int i0, int nr) {
        // targets on face a: threads own the columns
        for (int r = 0; r < nr; ++r) {
            const int i = i0 + r;
            double x[2][2][2]; // [s][s'][slot] = XB[s'][u_s(i)][slot]
#pragma unroll
            for (int sd = 0; sd < 2; ++sd) {
                const int u = sd ? Ma - i : i;
#pragma unroll
                for (int sp = 0; sp < 2; ++sp) {
                    x[sd][sp][0] = xb[(sp * na + u) * 2];
                    x[sd][sp][1] = xb[(sp * na + u) * 2 + 1];
                }
            }
#pragma unroll
            for (int jj = 0; jj < kPerpJpt; ++jj) {
                const int j = threadIdx.x + jj * NT;
                if (j < nb) {
                    const double K = tile[r * nb + j];
#pragma unroll
                    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
                        for (int sp = 0; sp < 2; ++sp) {
                            acc[jj][sd][sp][0] = fma(K, x[sd][sp][0], acc[jj][sd][sp][0]);
                            acc[jj][sd][sp][1] = fma(K, x[sd][sp][1], acc[jj][sd][sp][1]);
                        }
                }
            }
        }
        // targets on face b: each wave reduces whole rows over the columns, two
        // rows (r, r + 4) at a time so that they share the loads of xa
        for (int r = wave; r < nr; r += 2 * (NT / 64)) {
            const int r2 = r + NT / 64;
            const bool has2 = r2 < nr;
            double v[16]; // [row][s][s'][slot]
#pragma unroll
            for (int t = 0; t < 16; ++t) v[t] = 0.0;
            for (int j = lane; j < nb; j += 64) {
                const double K1 = tile[r * nb + j];
                const double K2 = has2 ? tile[r2 * nb + j] : 0.0;
#pragma unroll
                for (int sp = 0; sp < 2; ++sp) {
                    const int t = sp ? Mb - j : j;
#pragma unroll
                    for (int sd = 0; sd < 2; ++sd) {
                        const double x0 = xa[(sd * nb + t) * 2], x1 = xa[(sd * nb + t) * 2 + 1];
                        const int o = sd * 4 + sp * 2;
                        v[o] = fma(K1, x0, v[o]);
                        v[o + 1] = fma(K1, x1, v[o + 1]);
                        v[8 + o] = fma(K2, x0, v[8 + o]);
                        v[8 + o + 1] = fma(K2, x1, v[8 + o + 1]);
                    }
                }
            }
            // halving reduction: after the exchanges over lane bits 5, 4, 3, 2
            // a lane holds one of the 16 values, index lane >> 2
            double w8[8], w4[4], w2[2];
            const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8, h2 = lane & 4;
#pragma unroll
            for (int m = 0; m < 8; ++m)
                w8[m] = (h5 ? v[m + 8] : v[m]) + __shfl_xor(h5 ? v[m] : v[m + 8], 32);
#pragma unroll
            for (int m = 0; m < 4; ++m)
                w4[m] = (h4 ? w8[m + 4] : w8[m]) + __shfl_xor(h4 ? w8[m] : w8[m + 4], 16);
#pragma unroll
            for (int m = 0; m < 2; ++m)
                w2[m] = (h3 ? w4[m + 2] : w4[m]) + __shfl_xor(h3 ? w4[m] : w4[m + 2], 8);
            double w = (h2 ? w2[1] : w2[0]) + __shfl_xor(h2 ? w2[0] : w2[1], 4);
            w += __shfl_xor(w, 2);
            w += __shfl_xor(w, 1);
            const int vi = lane >> 2; // row (vi >> 3), s = (vi >> 2) & 1, s' = (vi >> 1) & 1, slot = vi & 1
            if ((lane & 3) == 0 && (vi < 8 || has2)) {
                const int i = i0 + (vi < 8 ? r : r2);
                const int sd = (vi >> 2) & 1, sp = (vi >> 1) & 1, sl = vi & 1;
                const int u = sd ? Ma - i : i;
                if (!sl || two)
                    PB[(int64_t)(sl ? q1 : q0) * pbq + (sd * 2 + sp) * na + u] = w;
            }
        }
    };
    for (int i0 = ibeg; i0 < iend; i0 += 2 * rows) {
        int nr = min(rows, iend - i0);
        __syncthreads(); // the previous tile is consumed (and xa, xb are stored)
        put(pfa, nr);
        __syncthreads();
        if (i0 + 2 * rows < iend) fetch(pfa, i0 + 2 * rows);
        work(i0, nr);
        const int i1 = i0 + rows;
        if (i1 >= iend) break;
        nr = min(rows, iend - i1);
        __syncthreads();
        put(pfb, nr);
        __syncthreads();
        if (i1 + 2 * rows < iend) fetch(pfb, i1 + 2 * rows);
        work(i1, nr);
    }
    // partials of the targets on face a: copy (g, s'), t = j (s' = 0) or M_b - j (s' = 1)
    double *PA = s.PA[pr];
    const int64_t paq = (int64_t)G * 4 * nb;
#pragma unroll
    for (int jj = 0; jj < kPerpJpt; ++jj) {
        const int j = threadIdx.x + jj * NT;
        if (j < nb)
#pragma unroll
            for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                for (int sd = 0; sd < 2; ++sd) {
                    const int t = sp ? Mb - j : j;
                    const int64_t o = ((int64_t)(g * 2 + sp) * 2 + sd) * nb + t;
                    PA[q0 * paq + o] = acc[jj][sd][sp][0];
                    if (two) PA[q1 * paq + o] = acc[jj][sd][sp][1];
                }
    }
}

// The same sums on the matrix cores (FP64 16x16x4 MFMA), for face sides up
// to kPerpMfmaMax nodes.  Per wavenumber k both sums are products of the
// table slab K = KT[k] (rows i, columns j) with eight vectors, the
// combinations n = 4 s + 2 s' + slot of target side, source side and slot
// (the N dimension of the instruction, 16 wide, half used):
//   targets on face a:  D_A[j][n] = sum_i K[i][j] xb[s'][u_s(i)][slot]
//   targets on face b:  D_B[i][n] = sum_j K[i][j] xa[s][t_s'(j)][slot]
// Rows of the slab stream through LDS in tiles of 16 (the next tile held in
// registers).  D_A: each wave owns every fourth 16-column block and keeps its
// accumulators over all tiles (K dimension: the 16 rows of a tile, four
// steps).  D_B: the four waves split the columns of a tile (K dimension, four
// columns a step) and their partial 16 x 16 products are summed through LDS.
// Operand layouts of the instruction (lane l): A[m][kk] with m = l % 16,
// kk = l / 16; B[kk][n] with n = l % 16, kk = l / 16; result element v of
// lane l is D[4 v + l / 16][l % 16].
constexpr int kPerpMfmaMax = 320;                 // M_a + 1, M_b + 1 at most
constexpr int kPerpTR = 16;                        // slab rows per tile
constexpr int kPerpJB = (kPerpMfmaMax + 15) / 16;  // 16-column blocks of a row
constexpr int kPerpJPW = (kPerpJB + 3) / 4;        // column blocks per wave
constexpr int kPerpMPf = (kPerpTR * kPerpMfmaMax + NT - 1) / NT; // prefetch registers per thread
typedef double perp_v4d __attribute__((ext_vector_type(4)));

bool perp_mfma_fits(const int *M)
{
    for (int a = 0; a < 3; ++a)
        if (M[a] + 1 > kPerpMfmaMax) return false;
    return true;
}

static size_t perp_mfma_lds_bytes(const int *M, int pr)
{
    const int a = pr == 2 ? 1 : 0, b = pr == 0 ? 1 : 2;
    // xa, xb, the tile (which also holds the cross-wave sums of D_B)
    return (size_t)(4 * (M[b] + 1) + 4 * (M[a] + 1) + std::max(kPerpTR * (M[b] + 1), 4 * 256)) * sizeof(double);
}

__global__ __launch_bounds__(NT) void k_perp_mfma(SurfArgs s, int pr)
{
    extern __shared__ __align__(16) unsigned char smem[];
    int a, b, c;
    pair_axes(pr, a, b, c);
    const int Ma = s.M[a], Mb = s.M[b], Mc = s.M[c];
    const int na = Ma + 1, nb = Mb + 1;
    const int k = blockIdx.x, g = blockIdx.y, G = gridDim.y;
    const bool two = k > 0 && k < Mc; // the sine slot exists
    const int q0 = k, q1 = Mc + k;
    const int ibeg = (int)((int64_t)g * na / G), iend = (int)((int64_t)(g + 1) * na / G);
    double *xa = reinterpret_cast<double *>(smem); // [2][nb][2 slots]
    double *xb = xa + 4 * nb;                      // [2][na][2 slots]
    double *tile = xb + 4 * na;                    // [kPerpTR][nb]
    double *red = tile;                            // [4 waves][64 lanes][4], after the tile is used
    const double *XA = s.XA[pr], *XB = s.XB[pr];
    const double *slab = s.KT[pr] + (int64_t)k * na * nb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lm = lane & 15, lk = lane >> 4; // operand row / column, K index
    // this lane's combination n (B operands and results): s, s', slot
    const int nsd = (lm >> 2) & 1, nsp = (lm >> 1) & 1, nsl = lm & 1;
    const bool nval = lm < 8;
    double pf[kPerpMPf];
    auto fetch = [&](int i0) {
        const int cnt = min(kPerpTR, iend - i0) * nb;
        const double *src = slab + (int64_t)i0 * nb;
#pragma unroll
        for (int m = 0; m < kPerpMPf; ++m) {
            const int e = tid + m * NT;
            if (e < cnt) pf[m] = src[e];
        }
    };
    if (ibeg < iend) fetch(ibeg);
    for (int e = tid; e < 2 * nb; e += NT) {
        xa[2 * e] = XA[(int64_t)q0 * 2 * nb + e];
        xa[2 * e + 1] = two ? XA[(int64_t)q1 * 2 * nb + e] : 0.0;
    }
    for (int e = tid; e < 2 * na; e += NT) {
        xb[2 * e] = XB[(int64_t)q0 * 2 * na + e];
        xb[2 * e + 1] = two ? XB[(int64_t)q1 * 2 * na + e] : 0.0;
    }
    const int njb = (nb + 15) >> 4, nj4 = (nb + 3) >> 2;
    perp_v4d accA[kPerpJPW];
#pragma unroll
    for (int q = 0; q < kPerpJPW; ++q) accA[q] = perp_v4d{0.0, 0.0, 0.0, 0.0};
    double *PB = s.PB[pr];
    const int64_t pbq = 4 * (int64_t)na;
    for (int i0 = ibeg; i0 < iend; i0 += kPerpTR) {
        const int nr = min(kPerpTR, iend - i0);
        __syncthreads(); // the previous sums are consumed (and xa, xb are stored)
#pragma unroll
        for (int m = 0; m < kPerpMPf; ++m) {
            const int e = tid + m * NT;
            if (e < nr * nb) tile[e] = pf[m];
        }
        __syncthreads();
        if (i0 + kPerpTR < iend) fetch(i0 + kPerpTR);
        // D_A: B operands of the four K steps (rows 4 st + lk of the tile)
        double bA[4];
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int r = 4 * st + lk, i = i0 + r;
            const int u = nsd ? Ma - i : i;
            bA[st] = (nval && r < nr) ? xb[(nsp * na + u) * 2 + nsl] : 0.0;
        }
        // (K steps outermost: the column blocks' accumulations are independent)
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int r = 4 * st + lk;
#pragma unroll
            for (int q = 0; q < kPerpJPW; ++q) {
                const int jb = wave + 4 * q;
                if (jb < njb) {
                    const int j = 16 * jb + lm;
                    const double av = (r < nr && j < nb) ? tile[r * nb + j] : 0.0;
                    accA[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bA[st], accA[q], 0, 0, 0);
                }
            }
        }
        // D_B: this wave's columns (steps wave, wave + 4, ...), rows lm of the
        // tile, in four independent accumulations
        perp_v4d dB[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) dB[x] = perp_v4d{0.0, 0.0, 0.0, 0.0};
        for (int st0 = wave; st0 < nj4; st0 += 16) {
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                const int st = st0 + 4 * x;
                const int j = 4 * st + lk;
                const double av = (lm < nr && j < nb) ? tile[lm * nb + j] : 0.0;
                const int t = nsp ? Mb - j : j;
                const double bv = (nval && j < nb) ? xa[(nsd * nb + t) * 2 + nsl] : 0.0;
                dB[x] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, dB[x], 0, 0, 0);
            }
        }
        __syncthreads(); // every wave is done with the tile
#pragma unroll
        for (int v = 0; v < 4; ++v) red[(wave * 64 + lane) * 4 + v] = (dB[0][v] + dB[1][v]) + (dB[2][v] + dB[3][v]);
        __syncthreads();
        {
            // thread tid sums element (lane l, v) = (tid >> 2, tid & 3) over the waves
            const int l = tid >> 2, v = tid & 3;
            const double w = red[(0 * 64 + l) * 4 + v] + red[(1 * 64 + l) * 4 + v] + red[(2 * 64 + l) * 4 + v] +
                             red[(3 * 64 + l) * 4 + v];
            const int r = 4 * v + (l >> 4), n = l & 15;
            if (n < 8 && r < nr) {
                const int sd = (n >> 2) & 1, sp = (n >> 1) & 1, sl = n & 1;
                const int i = i0 + r, u = sd ? Ma - i : i;
                if (!sl || two) PB[(int64_t)(sl ? q1 : q0) * pbq + (sd * 2 + sp) * na + u] = w;
            }
        }
    }
    // D_A: element v of lane l is column j = 16 jb + 4 v + lk, combination lm
    double *PA = s.PA[pr];
    const int64_t paq = (int64_t)G * 4 * nb;
    if (nval) {
#pragma unroll
        for (int q = 0; q < kPerpJPW; ++q) {
            const int jb = wave + 4 * q;
            if (jb >= njb) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = 16 * jb + 4 * v + lk;
                if (j >= nb) continue;
                const int t = nsp ? Mb - j : j;
                const int64_t o = ((int64_t)(g * 2 + nsp) * 2 + nsd) * nb + t;
                if (!nsl || two) PA[(nsl ? q1 : q0) * paq + o] = accA[q][v];
            }
        }
    }
}

hipError_t launch_perp(const SurfArgs &s, hipStream_t st)
{
    if (!perp_fits(s.M)) return hipErrorInvalidValue;
    for (int pr = 0; pr < 3; ++pr) {
        const int c = pr == 0 ? 2 : (pr == 1 ? 1 : 0);
        if (s.groups[pr] != perp_groups(s.M, pr)) return hipErrorInvalidValue;
        if (perp_mfma_fits(s.M)) {
            const size_t lds = perp_mfma_lds_bytes(s.M, pr);
            set_lds((const void *)&k_perp_mfma, lds);
            hipLaunchKernelGGL(k_perp_mfma, dim3(s.M[c] + 1, s.groups[pr]), dim3(NT), lds, st, s, pr);
        } else {
            const size_t lds = perp_lds_bytes(s.M, pr);
            set_lds((const void *)&k_perp, lds);
            hipLaunchKernelGGL(k_perp, dim3(s.M[c] + 1, s.groups[pr]), dim3(NT), lds, st, s, pr);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// g at every boundary node from the parallel and perpendicular sums of its
// owner face (the lowest axis on whose boundary it lies), plus the singular
// correction inside a face.
__global__ void k_surf_assemble(SurfArgs s, double *phi, int64_t ntgt)
{
    const int64_t n0 = s.M[0] + 1, n1 = s.M[1] + 1, n2 = s.M[2] + 1;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < ntgt; t += (int64_t)gridDim.x * blockDim.x) {
        int i[3];
        int64_t r = t;
        const int64_t f0 = n1 * n2, f1 = (n0 - 2) * n2;
        if (r < 2 * f0) {
            i[0] = r < f0 ? 0 : s.M[0];
            r %= f0;
            i[1] = (int)(r / n2);
            i[2] = (int)(r % n2);
        } else if ((r -= 2 * f0) < 2 * f1) {
            i[1] = r < f1 ? 0 : s.M[1];
            r %= f1;
            i[0] = 1 + (int)(r / n2);
            i[2] = (int)(r % n2);
        } else {
            r -= 2 * f1;
            const int64_t f2 = (n0 - 2) * (n1 - 2);
            i[2] = r < f2 ? 0 : s.M[2];
            r %= f2;
            i[0] = 1 + (int)(r / (n1 - 2));
            i[1] = 1 + (int)(r % (n1 - 2));
        }
        int own = -1, nbd = 0;
        for (int q = 2; q >= 0; --q)
            if (i[q] == 0 || i[q] == s.M[q]) {
                own = q;
                ++nbd;
            }
        const int a = own, side = i[a] == 0 ? 0 : 1;
        int b, c;
        face_axes(a, b, c);
        double g = s.PP[a][((int64_t)side * (s.M[b] + 1) + i[b]) * (s.M[c] + 1) + i[c]];
        for (int pr = 0; pr < 3; ++pr) {
            int pa, pb, pc;
            pair_axes(pr, pa, pb, pc);
            const int ncp = s.M[pc] + 1;
            if (pa == a) // targets on the a faces of the pair, indexed by (b-coordinate, c-coordinate)
                g += s.QA[pr][((int64_t)side * (s.M[pb] + 1) + i[pb]) * ncp + i[pc]];
            else if (pb == a) // targets on the b faces, indexed by (a-coordinate, c-coordinate)
                g += s.QB[pr][((int64_t)side * (s.M[pa] + 1) + i[pa]) * ncp + i[pc]];
        }
        if (nbd == 1) {
            const int Ic = s.M[c] - 1;
            g += s.tau[a] * s.sig[a][((int64_t)side * (s.M[b] - 1) + (i[b] - 1)) * Ic + (i[c] - 1)];
        }
        phi[((int64_t)i[0] * n1 + i[1]) * n2 + i[2]] = g;
    }
}

hipError_t launch_surf_assemble(const SurfArgs &s, double *phi, hipStream_t st)
{
    const int64_t n0 = s.M[0] + 1, n1 = s.M[1] + 1, n2 = s.M[2] + 1;
    const int64_t ntgt = 2 * n1 * n2 + 2 * (n0 - 2) * n2 + 2 * (n0 - 2) * (n1 - 2);
    const unsigned nbk = (unsigned)std::min<int64_t>((ntgt + NT - 1) / NT, 65535);
    hipLaunchKernelGGL(k_surf_assemble, dim3(nbk), dim3(NT), 0, st, s, phi, ntgt);
    return hipGetLastError();
}

// Face coefficients of the families whose sum runs over a strided axis of Y
// (axis 0, and axis 2 in 3D): the lanes take 64 consecutive k_1 (contiguous in
// Y), the waves every fourth term of the sum, combined in LDS in a fixed order.
// blockIdx.y: the remaining wavenumber (k_2 for fam 0, k_0 for fam 2; 3D).
__global__ __launch_bounds__(NT) void k_sigma_cols(ScreenArgs a, int fam)
{
    __shared__ double red[NT / 64][2][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int I0 = a.M[0] - 1, I1 = a.M[1] - 1;
    const int k1 = blockIdx.x * 64 + lane + 1;
    const int ko = blockIdx.y + 1;
    const int Ia = a.M[fam] - 1;
    double lo = 0.0, hi = 0.0;
    if (k1 <= I1) {
        // Y at (k0, k1, k2) = col[(ka - 1) step] with ka the summed wavenumber
        int64_t step;
        const double *col;
        double qo = a.tab[1].q[k1 - 1];
        if (fam == 0) {
            step = I1;
            col = a.Y + (a.d == 3 ? (int64_t)(ko - 1) * I0 * I1 : 0) + (k1 - 1);
            if (a.d == 3) qo += a.tab[2].q[ko - 1];
        } else {
            step = (int64_t)I0 * I1;
            col = a.Y + (int64_t)(ko - 1) * I1 + (k1 - 1);
            qo += a.tab[0].q[ko - 1];
        }
        const double *qa = a.tab[fam].q;
        for (int base = 1 + wave; base <= Ia; base += (NT / 64) * kSigU) {
            double y[kSigU];
#pragma unroll
            for (int u = 0; u < kSigU; ++u) {
                const int ka = base + (NT / 64) * u;
                y[u] = ka <= Ia ? col[(ka - 1) * step] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kSigU; ++u) {
                const int ka = base + (NT / 64) * u;
                if (ka <= Ia) {
                    const double alpha = -a.pref * y[u] / (qo + qa[ka - 1]);
                    const double t = (ka * a.piL[fam]) * alpha;
                    lo -= t;
                    hi += (ka & 1) ? -t : t;
                }
            }
        }
    }
    red[wave][0][lane] = lo;
    red[wave][1][lane] = hi;
    __syncthreads();
    if (wave == 0 && k1 <= I1) {
        for (int w = 1; w < NT / 64; ++w) {
            lo += red[w][0][lane];
            hi += red[w][1][lane];
        }
        // face layouts: fam 0 [side][k1][k2] (3D) or [side][k1]; fam 2 [side][k0][k1]
        int64_t o;
        if (fam == 0)
            o = a.d == 3 ? (int64_t)(k1 - 1) * (a.M[2] - 1) + (ko - 1) : (int64_t)(k1 - 1);
        else
            o = (int64_t)(ko - 1) * I1 + (k1 - 1);
        const int64_t fe = face_elems(a, fam);
        a.S[fam][o] = lo;
        a.S[fam][fe + o] = hi;
    }
}

hipError_t launch_screen(const ScreenArgs &a, double *phi, hipStream_t st)
{
    (void)phi;
    // family 1 (sum over the contiguous axis): one wave per output
    int64_t nf1 = 1;
    for (int b = 0; b < a.d; ++b)
        if (b != 1) nf1 *= a.M[b] - 1;
    const int64_t nb = (nf1 + NT / 64 - 1) / (NT / 64);
    if (nb > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sigma_rows, dim3((unsigned)nb), dim3(NT), 0, st, a, nf1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned nx = (unsigned)((a.M[1] - 1 + 63) / 64);
    hipLaunchKernelGGL(k_sigma_cols, dim3(nx, a.d == 3 ? a.M[2] - 1 : 1), dim3(NT), 0, st, a, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (a.d == 3) {
        hipLaunchKernelGGL(k_sigma_cols, dim3(nx, a.M[0] - 1), dim3(NT), 0, st, a, 2);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_screen_g(const ScreenArgs &a, double *phi, hipStream_t st)
{
    const unsigned nbs = (unsigned)std::min<int64_t>((a.nsrc + NT - 1) / NT, 65535);
    hipLaunchKernelGGL(k_screen_src, dim3(nbs), dim3(NT), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nbt = (a.ntgt + NT - 1) / NT;
    if (nbt > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_screen_g, dim3((unsigned)nbt), dim3(NT), 0, st, a, phi);
    return hipGetLastError();
}

} // namespace ips
