// Boundary values from the screening charge (James-type methods, Sections 1
// and 2), the alternative to the volume sums of Section 4:
//   g(x) = surface integral of G(|x - s|) sigma(s) dS(s),  sigma = d phi*/dn,
// sigma from the sine coefficients alpha of phi* (Section 3).
//   k_sigma_sums : face sine coefficients of sigma, sums over the normal wavenumber
//   k_screen_src : the weighted surface nodes (position, W sigma) of every face
//   k_screen_g   : the corrected surface trapezoidal sums at every boundary node
#include <hip/hip_runtime.h>

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
