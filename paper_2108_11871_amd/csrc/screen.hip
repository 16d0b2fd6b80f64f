// Boundary values from the screening charge (James-type methods, Sections 1
// and 2), the alternative to the volume sums of Section 4:
//   g(x) = surface integral of G(|x - s|) sigma(s) dS(s),  sigma = d phi*/dn,
// sigma from the sine coefficients alpha of phi* (Section 3).
//   k_sigma_sums : face sine coefficients of sigma, sums over the normal wavenumber
//   k_screen_src : the weighted surface nodes (position, W sigma) of every face
//   k_screen_g   : the corrected surface trapezoidal sums at every boundary node
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
// One wave per output pair: its lanes stride over k_a and reduce by shuffles.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_sigma_sums(ScreenArgs a, int64_t nfam0, int64_t nfam1)
{
    const int lane = threadIdx.x & 63;
    int64_t w = (int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
    int fam = 0;
    if (w >= nfam0) {
        w -= nfam0;
        fam = 1;
        if (w >= nfam1) {
            w -= nfam1;
            fam = 2;
        }
    }
    if (fam >= a.d || w >= face_elems(a, fam)) return;
    const int I0 = a.M[0] - 1, I1 = a.M[1] - 1, I2 = a.d == 3 ? a.M[2] - 1 : 1;
    // the two fixed wavenumbers of this output (face layout order)
    int k[3] = {0, 0, 0};
    if (a.d == 3) {
        const int b = fam == 0 ? 1 : 0, c = fam == 2 ? 1 : 2;
        const int Ic = a.M[c] - 1;
        k[b] = 1 + (int)(w / Ic);
        k[c] = 1 + (int)(w % Ic);
    } else {
        k[1 - fam] = 1 + (int)w;
    }
    const int Ia = a.M[fam] - 1;
    double lo = 0.0, hi = 0.0;
    for (int ka = 1 + lane; ka <= Ia; ka += 64) {
        k[fam] = ka;
        const int64_t idx = a.d == 3 ? ((int64_t)(k[2] - 1) * I0 + (k[0] - 1)) * I1 + (k[1] - 1)
                                     : (int64_t)(k[0] - 1) * I1 + (k[1] - 1);
        double q = 0.0;
        for (int b = 0; b < a.d; ++b) q += a.tab[b].q[k[b] - 1];
        const double alpha = -a.pref * a.Y[idx] / q;
        const double t = (ka * a.piL[fam]) * alpha;
        lo -= t;
        hi += (ka & 1) ? -t : t;
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo += __shfl_xor(lo, off);
        hi += __shfl_xor(hi, off);
    }
    (void)I2;
    if (lane == 0) {
        const int64_t fe = face_elems(a, fam);
        a.S[fam][w] = lo;
        a.S[fam][fe + w] = hi;
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

// One block per wavenumber k of the shared axis c of pair (a, b): both slots
// (cosine k, sine k) of
//   YA[s][t][.] = sum_(s', u) KT[k][|s M_a - u|][|t - s' M_b|] XB[s'][u][.]   (targets on face (a, s))
//   YB[s'][u][.] = sum_(s, t) KT[k][|s M_a - u|][|t - s' M_b|] XA[s][t][.]   (targets on face (b, s'))
// The table slab KT[k] streams through LDS in tiles of rows i; the targets on
// a are owned by the threads (columns j, accumulated over the rows), the
// targets on b by the rows (each wave reduces its rows over the columns).
// With i = |s M_a - u| and j = |t - s' M_b|: u = i or M_a - i by side s, and
// t = j or M_b - j by side s'.
constexpr int kPerpJpt = 3; // columns per thread: M_b + 1 <= 3 * NT

static size_t perp_lds_bytes(const int *M, int rows)
{
    int mx = 0;
    for (int a = 0; a < 3; ++a) mx = std::max(mx, M[a] + 1);
    // xa, xb, two halves of YB, the second halves of YA, the tile
    return (size_t)(4 * mx + 4 * mx + 8 * mx + 4 * mx + rows * mx) * sizeof(double);
}

int perp_rows(const int *M)
{
    int mx = 0;
    for (int a = 0; a < 3; ++a) mx = std::max(mx, M[a] + 1);
    if (mx > kPerpJpt * NT) return 0;
    const int r = (int)((size_t)(160 * 1024) / (sizeof(double) * (size_t)mx)) - 20;
    return std::max(0, std::min(16, r));
}

__global__ __launch_bounds__(NT) void k_perp(SurfArgs s, int pr)
{
    extern __shared__ __align__(16) unsigned char smem[];
    int a, b, c;
    pair_axes(pr, a, b, c);
    const int Ma = s.M[a], Mb = s.M[b], Mc = s.M[c];
    const int na = Ma + 1, nb = Mb + 1, Nc = 2 * Mc;
    const int k = blockIdx.x;
    const int nq = (k == 0 || k == Mc) ? 1 : 2;
    const int q0 = k, q1 = Mc + k;
    double *xa = reinterpret_cast<double *>(smem); // [2][nb][2]
    double *xb = xa + 4 * nb;                      // [2][na][2]
    double *yb0 = xb + 4 * na;                     // [2][na][2] from the rows u = i (source side 0)
    double *yb1 = yb0 + 4 * na;                    // [2][na][2] from the rows u = M_a - i (source side 1)
    double *ls = yb1 + 4 * na;                     // [2][nb][2] targets on a, parts of source side 1
    double *tile = ls + 4 * nb;                    // [rows][nb]
    const double *XA = s.XA[pr], *XB = s.XB[pr];
    for (int e = threadIdx.x; e < 2 * nb; e += NT) {
        const int64_t o = (int64_t)e * Nc;
        xa[2 * e] = XA[o + q0];
        xa[2 * e + 1] = nq > 1 ? XA[o + q1] : 0.0;
    }
    for (int e = threadIdx.x; e < 2 * na; e += NT) {
        const int64_t o = (int64_t)e * Nc;
        xb[2 * e] = XB[o + q0];
        xb[2 * e + 1] = nq > 1 ? XB[o + q1] : 0.0;
    }
    for (int e = threadIdx.x; e < 8 * na; e += NT) yb0[e] = 0.0;
    double acc[kPerpJpt][2][2][2]; // [column][target side s][source side s'][slot]
#pragma unroll
    for (int jj = 0; jj < kPerpJpt; ++jj)
#pragma unroll
        for (int v = 0; v < 8; ++v) (&acc[jj][0][0][0])[v] = 0.0;
    const double *slab = s.KT[pr] + (int64_t)k * na * nb;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i0 = 0; i0 < na; i0 += s.rows) {
        const int nr = min(s.rows, na - i0);
        __syncthreads();
        for (int e = threadIdx.x; e < nr * nb; e += NT) tile[e] = slab[(int64_t)i0 * nb + e];
        __syncthreads();
        // targets on face a (threads own the columns)
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
        // targets on face b (each wave reduces whole rows)
        for (int r = wave; r < nr; r += NT / 64) {
            const int i = i0 + r;
            double ps[2][2][2]; // [source side s][target side s'][slot]
#pragma unroll
            for (int v = 0; v < 8; ++v) (&ps[0][0][0])[v] = 0.0;
            for (int j = lane; j < nb; j += 64) {
                const double K = tile[r * nb + j];
#pragma unroll
                for (int sp = 0; sp < 2; ++sp) {
                    const int t = sp ? Mb - j : j;
#pragma unroll
                    for (int sd = 0; sd < 2; ++sd) {
                        ps[sd][sp][0] = fma(K, xa[(sd * nb + t) * 2], ps[sd][sp][0]);
                        ps[sd][sp][1] = fma(K, xa[(sd * nb + t) * 2 + 1], ps[sd][sp][1]);
                    }
                }
            }
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                double w = (&ps[0][0][0])[v];
                for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off);
                (&ps[0][0][0])[v] = w;
            }
            if (lane == 0) {
#pragma unroll
                for (int sp = 0; sp < 2; ++sp) {
                    // source side 0: u = i; source side 1: u = M_a - i
                    yb0[(sp * na + i) * 2] = ps[0][sp][0];
                    yb0[(sp * na + i) * 2 + 1] = ps[0][sp][1];
                    yb1[(sp * na + (Ma - i)) * 2] = ps[1][sp][0];
                    yb1[(sp * na + (Ma - i)) * 2 + 1] = ps[1][sp][1];
                }
            }
        }
    }
    __syncthreads();
    // targets on a: t = j from source side 0, t = M_b - j from side 1
#pragma unroll
    for (int jj = 0; jj < kPerpJpt; ++jj) {
        const int j = threadIdx.x + jj * NT;
        if (j < nb)
#pragma unroll
            for (int sd = 0; sd < 2; ++sd) {
                ls[(sd * nb + (Mb - j)) * 2] = acc[jj][sd][1][0];
                ls[(sd * nb + (Mb - j)) * 2 + 1] = acc[jj][sd][1][1];
            }
    }
    __syncthreads();
    double *YA = s.YA[pr], *YB = s.YB[pr];
#pragma unroll
    for (int jj = 0; jj < kPerpJpt; ++jj) {
        const int j = threadIdx.x + jj * NT;
        if (j < nb)
#pragma unroll
            for (int sd = 0; sd < 2; ++sd) {
                const int64_t o = ((int64_t)sd * nb + j) * Nc;
                YA[o + q0] = acc[jj][sd][0][0] + ls[(sd * nb + j) * 2];
                if (nq > 1) YA[o + q1] = acc[jj][sd][0][1] + ls[(sd * nb + j) * 2 + 1];
            }
    }
    for (int e = threadIdx.x; e < 2 * na; e += NT) {
        const int64_t o = (int64_t)e * Nc;
        YB[o + q0] = yb0[2 * e] + yb1[2 * e];
        if (nq > 1) YB[o + q1] = yb0[2 * e + 1] + yb1[2 * e + 1];
    }
}

hipError_t launch_perp(const SurfArgs &s, hipStream_t st)
{
    if (s.rows < 1 || perp_rows(s.M) < s.rows) return hipErrorInvalidValue;
    const size_t lds = perp_lds_bytes(s.M, s.rows);
    set_lds((const void *)&k_perp, lds);
    for (int pr = 0; pr < 3; ++pr) {
        const int c = pr == 0 ? 2 : (pr == 1 ? 1 : 0);
        hipLaunchKernelGGL(k_perp, dim3(s.M[c] + 1), dim3(NT), lds, st, s, pr);
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

hipError_t launch_screen(const ScreenArgs &a, double *phi, hipStream_t st)
{
    int64_t nf[3] = {0, 0, 0};
    for (int f = 0; f < a.d; ++f) {
        int64_t s = 1;
        for (int b = 0; b < a.d; ++b)
            if (b != f) s *= a.M[b] - 1;
        nf[f] = s;
    }
    const int64_t waves = nf[0] + nf[1] + nf[2];
    const int64_t nb = (waves + NT / 64 - 1) / (NT / 64);
    if (nb > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sigma_sums, dim3((unsigned)nb), dim3(NT), 0, st, a, nf[0], nf[1]);
    return hipGetLastError();
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
