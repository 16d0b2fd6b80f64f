// HIP kernels of the adjoint map rho_bar = A^T phi_bar (gfx950, FP64).
//
// The forward solve is linear, phi = A rho; each of its steps is transposed
// here in reverse order:
//   phi_I = phi_star_I + u_I,  phi_boundary = g,  g = B rho  (Sections 2, 4)
//   u_I   = L0^-1 (T g)                                        (order 4)
//   u_I   = L0^-1 (T g + E R_core(u1, g)),  u1_I = L0^-1 T g   (order 6)
// with T the transfer of boundary values to the right-hand side (eq.
// harmonic4thOrderNH2D), R_core the sixth-order stencils on the core and E
// the cubic extrapolation next to the boundary (eqs. 6thOrderRelation2D/3D).
// The phi_star map and L0^-1 are symmetric.  Writing w = phi_bar:
//   a      = L0^-1 w_I
//   f      = E^T a                    (core nodes; order 6)
//   U      = S f, S = sum_{x != y} c4[x][y] D2_x D2_x D2_y on every node
//   b      = L0^-1 U_I                (order 6)
//   lambda = w_boundary + T^T (a + b) + U_boundary
//   rho_bar_I = phi_star(w_I) + B^T lambda,  rho_bar_boundary = 0
// B^T spreads boundary values back over the interior with the same Green's
// function sums, evaluated by FFT convolutions with the plan's kernel
// spectra: for every slice s normal to a face family,
//   slice(s) = IFFT2[ K_hat(s - 1) . FFT2(lambda_face0)
//                     + K_hat(M - 1 - s) . FFT2(lambda_faceM) ].
#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

namespace ips {

constexpr int NTA = 256;

__device__ __forceinline__ int64_t grid_off(const int64_t *n, int d, const int *i)
{
    int64_t o = 0;
    for (int a = 0; a < d; ++a) o = o * n[a] + i[a];
    return o;
}

// Lambda(k) of L0 and the continuous eigenvalue sum q(k) for one mode.
template <int D>
__device__ __forceinline__ void mode_symbols(const AdjArgs &a, const int *k, double &L, double &q)
{
    double lam[3];
    L = 0.0;
    q = 0.0;
#pragma unroll
    for (int x = 0; x < D; ++x) {
        lam[x] = a.tab[x].lam[k[x] - 1];
        L += lam[x];
        q += a.tab[x].q[k[x] - 1];
    }
#pragma unroll
    for (int x = 0; x < D; ++x)
#pragma unroll
        for (int y = x + 1; y < D; ++y) L += a.geo.c2[x][y] * lam[x] * lam[y];
}

// X holds raw sine coefficients over the interior modes ([k0][k1][k2], last
// fastest).  Y (if given) <- -pref X / q  (the phi_star map);  X <- pref X / Lambda.
template <int D>
__global__ __launch_bounds__(NTA) void k_adj_spec(AdjArgs a, double *X, double *Y)
{
    const Geo &g = a.geo;
    int64_t tot = 1;
    for (int x = 0; x < D; ++x) tot *= g.M[x] - 1;
    for (int64_t e = blockIdx.x * (int64_t)NTA + threadIdx.x; e < tot; e += (int64_t)gridDim.x * NTA) {
        int k[3];
        int64_t r = e;
#pragma unroll
        for (int x = D - 1; x >= 0; --x) {
            const int I = g.M[x] - 1;
            k[x] = 1 + (int)(r % I);
            r /= I;
        }
        double L, q;
        mode_symbols<D>(a, k, L, q);
        const double v = X[e];
        if (Y) Y[e] = -g.pref * v / q;
        X[e] = g.pref * v / L;
    }
}

hipError_t launch_adj_spec(const AdjArgs &a, double *X, double *Y, hipStream_t st)
{
    const int nb = 4096;
    if (a.geo.d == 3)
        hipLaunchKernelGGL(k_adj_spec<3>, dim3(nb), dim3(NTA), 0, st, a, X, Y);
    else
        hipLaunchKernelGGL(k_adj_spec<2>, dim3(nb), dim3(NTA), 0, st, a, X, Y);
    return hipGetLastError();
}

// f = E^T a on the core (all indices in [2, M-2]), 0 on every other node of
// the grid-shaped array F.  E is the tensor product of one-axis maps
//   e(i, p) = [i == p] for i in [2, M-2],
//   e(1, p) = (4, -6, 4, -1)[p - 2]        for p in 2..5,
//   e(M-1, p) = (4, -6, 4, -1)[M - 2 - p]  for p in M-5..M-2,
// so E^T a at p sums a at (p or 1 or M-1 per axis) with the product weights.
// a is packed over the interior ([i0-1][i1-1][i2-1]).
template <int D>
__global__ __launch_bounds__(NTA) void k_adj_etrans(AdjArgs a, const double *A, double *F)
{
    const Geo &g = a.geo;
    int64_t tot = 1;
    for (int x = 0; x < D; ++x) tot *= a.n[x];
    const double wt[4] = {4.0, -6.0, 4.0, -1.0};
    for (int64_t e = blockIdx.x * (int64_t)NTA + threadIdx.x; e < tot; e += (int64_t)gridDim.x * NTA) {
        int i[3] = {0, 0, 0};
        int64_t r = e;
#pragma unroll
        for (int x = D - 1; x >= 0; --x) {
            i[x] = (int)(r % a.n[x]);
            r /= a.n[x];
        }
        bool core = true;
#pragma unroll
        for (int x = 0; x < D; ++x) core = core && i[x] >= 2 && i[x] <= g.M[x] - 2;
        double v = 0.0;
        if (core) {
            // per axis: up to three (source index, weight) options
            int src[3][3];
            double w[3][3];
            int cnt[3] = {1, 1, 1};
#pragma unroll
            for (int x = 0; x < D; ++x) {
                const int M = g.M[x], p = i[x];
                src[x][0] = p;
                w[x][0] = 1.0;
                if (p <= 5) {
                    src[x][cnt[x]] = 1;
                    w[x][cnt[x]] = wt[p - 2];
                    ++cnt[x];
                }
                if (p >= M - 5) {
                    src[x][cnt[x]] = M - 1;
                    w[x][cnt[x]] = wt[M - 2 - p];
                    ++cnt[x];
                }
            }
            const int c1 = D >= 2 ? cnt[1] : 1, c2 = D == 3 ? cnt[2] : 1;
            for (int t0 = 0; t0 < cnt[0]; ++t0)
                for (int t1 = 0; t1 < c1; ++t1)
                    for (int t2 = 0; t2 < c2; ++t2) {
                        int64_t o = src[0][t0] - 1;
                        double ww = w[0][t0];
                        if (D >= 2) {
                            o = o * (g.M[1] - 1) + (src[1][t1] - 1);
                            ww *= w[1][t1];
                        }
                        if (D == 3) {
                            o = o * (g.M[2] - 1) + (src[2][t2] - 1);
                            ww *= w[2][t2];
                        }
                        v += ww * A[o];
                    }
        }
        F[e] = v;
    }
}

// U = sum_{x != y} c4[x][y] D2_x D2_x D2_y F on every grid node, with F = 0
// off the core (the stencil is symmetric, so this is also its transpose).
template <int D>
__global__ __launch_bounds__(NTA) void k_adj_sop(AdjArgs a, const double *F, double *U)
{
    const Geo &g = a.geo;
    int64_t tot = 1;
    for (int x = 0; x < D; ++x) tot *= a.n[x];
    const double a4[5] = {1.0, -4.0, 6.0, -4.0, 1.0};
    const double a2[3] = {1.0, -2.0, 1.0};
    for (int64_t e = blockIdx.x * (int64_t)NTA + threadIdx.x; e < tot; e += (int64_t)gridDim.x * NTA) {
        int i[3] = {0, 0, 0};
        int64_t r = e;
#pragma unroll
        for (int x = D - 1; x >= 0; --x) {
            i[x] = (int)(r % a.n[x]);
            r /= a.n[x];
        }
        double v = 0.0;
#pragma unroll
        for (int x = 0; x < D; ++x)
#pragma unroll
            for (int y = 0; y < D; ++y) {
                if (y == x) continue;
                double s = 0.0;
#pragma unroll
                for (int dx = -2; dx <= 2; ++dx)
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy) {
                        int j[3] = {i[0], i[1], i[2]};
                        j[x] += dx;
                        j[y] += dy;
                        bool core = true;
#pragma unroll
                        for (int z = 0; z < D; ++z) core = core && j[z] >= 2 && j[z] <= g.M[z] - 2;
                        if (core) s += a4[dx + 2] * a2[dy + 1] * F[grid_off(a.n, D, j)];
                    }
                const double hx2 = g.h[x] * g.h[x];
                v += g.c4[x][y] * s / (hx2 * hx2 * g.h[y] * g.h[y]);
            }
        U[e] = v;
    }
}

// 3D: the same sums in separable form, one axis x at a time,
//   T_x = sum_{y != x} c4[x][y] / (h_x^4 h_y^2) D2_y F      (k_adj_d2y)
//   U  += D4_x T_x                                         (k_adj_d4x)
// with F and T_x taken as zero off the grid (F is zero outside the core: the
// extrapolation writes every node), which is the tap set of k_adj_sop.  One
// thread per node; the threads of a block take consecutive nodes of one plane
// of the first axis (grid.y), so every lane is busy whatever the line length.
__global__ __launch_bounds__(NTA) void k_adj_d2y(AdjArgs a, int x, const double *F, double *T)
{
    const Geo &g = a.geo;
    const int n[3] = {(int)a.n[0], (int)a.n[1], (int)a.n[2]};
    const int pl = blockIdx.x * NTA + threadIdx.x;
    if (pl >= n[1] * n[2]) return;
    const int i0 = blockIdx.y, i1 = pl / n[2], i2 = pl - i1 * n[2];
    const int64_t st[3] = {(int64_t)n[1] * n[2], n[2], 1};
    const double hx2 = g.h[x] * g.h[x];
    {
        const int i[3] = {i0, i1, i2};
        const int64_t e = i0 * st[0] + pl;
        double v = 0.0;
#pragma unroll
        for (int y = 0; y < 3; ++y) {
            if (y == x) continue;
            const double fm = i[y] > 0 ? F[e - st[y]] : 0.0;
            const double fp = i[y] < n[y] - 1 ? F[e + st[y]] : 0.0;
            v += g.c4[x][y] / (hx2 * hx2 * g.h[y] * g.h[y]) * (fm - 2.0 * F[e] + fp);
        }
        T[e] = v;
    }
}

__global__ __launch_bounds__(NTA) void k_adj_d4x(AdjArgs a, int x, const double *T, double *U)
{
    const int n[3] = {(int)a.n[0], (int)a.n[1], (int)a.n[2]};
    const int pl = blockIdx.x * NTA + threadIdx.x;
    if (pl >= n[1] * n[2]) return;
    const int i0 = blockIdx.y, i1 = pl / n[2], i2 = pl - i1 * n[2];
    const int64_t st[3] = {(int64_t)n[1] * n[2], n[2], 1};
    const double a4[5] = {1.0, -4.0, 6.0, -4.0, 1.0};
    {
        const int i[3] = {i0, i1, i2};
        const int64_t e = i0 * st[0] + pl;
        double v = 0.0;
#pragma unroll
        for (int dx = -2; dx <= 2; ++dx) {
            const int j = i[x] + dx;
            if (j >= 0 && j < n[x]) v += a4[dx + 2] * T[e + dx * st[x]];
        }
        U[e] = x == 0 ? v : U[e] + v;
    }
}

hipError_t launch_adj_r6(const AdjArgs &a, const double *A, double *F, double *U, double *T, hipStream_t st)
{
    const int nb = 4096;
    if (a.geo.d == 3) {
        hipLaunchKernelGGL(k_adj_etrans<3>, dim3(nb), dim3(NTA), 0, st, a, A, F);
        const dim3 grid((unsigned)((a.n[1] * a.n[2] + NTA - 1) / NTA), (unsigned)a.n[0]);
        for (int x = 0; x < 3; ++x) {
            hipLaunchKernelGGL(k_adj_d2y, grid, dim3(NTA), 0, st, a, x, F, T);
            hipLaunchKernelGGL(k_adj_d4x, grid, dim3(NTA), 0, st, a, x, T, U);
        }
    } else {
        hipLaunchKernelGGL(k_adj_etrans<2>, dim3(nb), dim3(NTA), 0, st, a, A, F);
        hipLaunchKernelGGL(k_adj_sop<2>, dim3(nb), dim3(NTA), 0, st, a, F, U);
    }
    return hipGetLastError();
}

// lambda on the face nodes of every family (faces own their edges and
// corners with precedence axis 0 > axis 1 > axis 2; other entries 0):
//   lambda = w + U - sum over interior neighbours i of the L_h stencil
//            weight times (y1 + y2)(i)
// y1, y2 packed over the interior (y2 and U may be NULL).
// LF[fam][f][j_b][j_c] over (M_b + 1) x (M_c + 1), (b, c) = a.fb[fam], a.fc[fam].
template <int D>
__global__ __launch_bounds__(NTA) void k_adj_lambda(AdjArgs a, const double *w, const double *y1,
                                                    const double *y2, const double *U)
{
    const Geo &g = a.geo;
    int fam = 0;
    int64_t e = blockIdx.x * (int64_t)NTA + threadIdx.x;
    while (fam < D && e >= a.lf_size[fam]) {
        e -= a.lf_size[fam];
        ++fam;
    }
    if (fam >= D) return;
    const int b = a.fb[fam], c = a.fc[fam];
    const int nb = g.M[b] + 1, ncn = D == 3 ? g.M[c] + 1 : 1;
    const int per = nb * ncn;
    const int f = (int)(e / per);
    const int rem = (int)(e % per);
    int i[3] = {0, 0, 0};
    i[fam] = f ? g.M[fam] : 0;
    i[b] = rem / ncn;
    if (D == 3) i[c] = rem % ncn;
    bool owned = true;
    for (int x = 0; x < fam; ++x)
        if (i[x] == 0 || i[x] == g.M[x]) owned = false;
    double lam = 0.0;
    if (owned) {
        const int64_t go = grid_off(a.n, D, i);
        lam = w[go];
        if (U) lam += U[go];
        double s = 0.0;
        // face-neighbour offsets
#pragma unroll
        for (int p = 0; p < D; ++p) {
            double wf = 1.0 / (g.h[p] * g.h[p]);
#pragma unroll
            for (int q = 0; q < D; ++q)
                if (q != p) wf -= 2.0 * g.c2[p][q] / (g.h[p] * g.h[p] * g.h[q] * g.h[q]);
#pragma unroll
            for (int sg = -1; sg <= 1; sg += 2) {
                int j[3] = {i[0], i[1], i[2]};
                j[p] += sg;
                bool in = true;
#pragma unroll
                for (int z = 0; z < D; ++z) in = in && j[z] >= 1 && j[z] <= g.M[z] - 1;
                if (in) {
                    int64_t o = 0;
#pragma unroll
                    for (int z = 0; z < D; ++z) o = o * (g.M[z] - 1) + (j[z] - 1);
                    s += wf * (y1[o] + (y2 ? y2[o] : 0.0));
                }
            }
        }
        // edge-neighbour offsets
#pragma unroll
        for (int p = 0; p < D; ++p)
#pragma unroll
            for (int q = p + 1; q < D; ++q) {
                const double we = g.c2[p][q] / (g.h[p] * g.h[p] * g.h[q] * g.h[q]);
#pragma unroll
                for (int sp = -1; sp <= 1; sp += 2)
#pragma unroll
                    for (int sq = -1; sq <= 1; sq += 2) {
                        int j[3] = {i[0], i[1], i[2]};
                        j[p] += sp;
                        j[q] += sq;
                        bool in = true;
#pragma unroll
                        for (int z = 0; z < D; ++z) in = in && j[z] >= 1 && j[z] <= g.M[z] - 1;
                        if (in) {
                            int64_t o = 0;
#pragma unroll
                            for (int z = 0; z < D; ++z) o = o * (g.M[z] - 1) + (j[z] - 1);
                            s += we * (y1[o] + (y2 ? y2[o] : 0.0));
                        }
                    }
            }
        lam -= s;
    }
    a.LF[fam][e] = lam;
}

hipError_t launch_adj_lambda(const AdjArgs &a, const double *w, const double *y1, const double *y2,
                             const double *U, hipStream_t st)
{
    int64_t tot = 0;
    for (int fam = 0; fam < a.geo.d; ++fam) tot += a.lf_size[fam];
    const unsigned nb = (unsigned)((tot + NTA - 1) / NTA);
    if (a.geo.d == 3)
        hipLaunchKernelGGL(k_adj_lambda<3>, dim3(nb), dim3(NTA), 0, st, a, w, y1, y2, U);
    else
        hipLaunchKernelGGL(k_adj_lambda<2>, dim3(nb), dim3(NTA), 0, st, a, w, y1, y2, U);
    return hipGetLastError();
}

// Zero the boundary nodes of a grid-shaped array.
template <int D>
__global__ __launch_bounds__(NTA) void k_zero_boundary(AdjArgs a, double *out)
{
    int64_t tot = 1;
    for (int x = 0; x < D; ++x) tot *= a.n[x];
    for (int64_t e = blockIdx.x * (int64_t)NTA + threadIdx.x; e < tot; e += (int64_t)gridDim.x * NTA) {
        int64_t r = e;
        bool bnd = false;
#pragma unroll
        for (int x = D - 1; x >= 0; --x) {
            const int ix = (int)(r % a.n[x]);
            r /= a.n[x];
            bnd = bnd || ix == 0 || ix == a.geo.M[x];
        }
        if (bnd) out[e] = 0.0;
    }
}

hipError_t launch_zero_boundary(const AdjArgs &a, double *out, hipStream_t st)
{
    if (a.geo.d == 3)
        hipLaunchKernelGGL(k_zero_boundary<3>, dim3(4096), dim3(NTA), 0, st, a, out);
    else
        hipLaunchKernelGGL(k_zero_boundary<2>, dim3(4096), dim3(NTA), 0, st, a, out);
    return hipGetLastError();
}

// Face-to-slice expansion, first transform.  Tile rows = slots r of the
// transform axis (length N), tile columns = W consecutive column indices,
// batch = grid.y.  Input element (r, col):
//   3D: K_hat[s-1][kb(col)][kc(r)] LH0[col][r] + K_hat[M-1-s][kb][kc] LH1[col][r],
//       s = batch + 1, col = slot of the other in-face axis
//   2D: K_hat[s-1][k(r)] LH0[r] + K_hat[M-1-s][k(r)] LH1[r],  s = col + 1
// followed by the hermitian synthesis along the rows.  Rows 1..M-1 of the
// result, times `scale`, are stored (3D) or added (2D) to out[(row-1)*ors +
// col*ocs + batch*obs].
template <int MAXE, bool P2, int NTT>
__global__ __launch_bounds__(NTT) void k_expand(ExpandArgs a)
{
    constexpr bool BIG = NTT != NTA;
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = a.fd.N, M = a.fd.M, W = a.W, rs = BIG ? W : W + 1;
    const int lgW = 31 - __clz(W), lgs = lgW - 1;
    const cx<double> *tw = BIG ? a.tw : reinterpret_cast<const cx<double> *>(smem);
    double *buf = reinterpret_cast<double *>(smem + (BIG ? 0 : (size_t)N * sizeof(cx<double>)));
    const int ncb = (a.ncols + W - 1) / W;
    const int cb = blockIdx.x % ncb, bt = blockIdx.x / ncb;
    const int c0 = cb * W;
    const int nc = min(W, a.ncols - c0);
    if (!BIG) load_twiddles<double, NTT>(reinterpret_cast<cx<double> *>(smem), a.tw, N);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c = wave; c < W; c += NTT / 64) {
        const int col = c0 + c;
        int s, kb;
        const double *l0, *l1;
        if (a.d == 3) {
            s = bt + 1;
            kb = col <= a.Mb ? col : col - a.Mb;
            l0 = a.LH0 + (int64_t)col * N;
            l1 = a.LH1 + (int64_t)col * N;
        } else {
            s = col + 1;
            kb = 0;
            l0 = a.LH0;
            l1 = a.LH1;
        }
        const double *k0 = a.K + (int64_t)(s - 1) * a.Kd + (int64_t)kb * a.Kb;
        const double *k1 = a.K + (int64_t)(a.Ms - 1 - s) * a.Kd + (int64_t)kb * a.Kb;
        for (int r = lane; r < N; r += 64) {
            double v = 0.0;
            if (c < nc) {
                const int kc = r <= M ? r : r - M;
                v = k0[kc] * l0[r] + k1[kc] * l1[r];
            }
            buf[r * rs + c] = v;
        }
    }
    __syncthreads();
    pre_herm<double, MAXE, NTT>(buf, rs, lgs, M, false);
    fft_tile<double, MAXE, NTT, P2>(buf, rs, lgs, a.fd, tw, true);
    double *out = a.out + (int64_t)bt * a.obs + (int64_t)c0 * a.ocs;
    if (a.accum)
        tile_store_acc<double, double, NTT>(buf, rs, 1, out, M - 1, nc, a.ors, a.ocs, a.scale, lgW);
    else
        tile_store<double, double, NTT>(buf, rs, 1, out, M - 1, nc, a.ors, a.ocs, a.scale, lgW);
}

static bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

template <int MAXE, int NTT = NTA>
static void launch_expand_m(const ExpandArgs &a, unsigned nblk, size_t lds, hipStream_t st)
{
    if (pow2(a.fd.N)) {
        set_lds((const void *)&k_expand<MAXE, true, NTT>, lds);
        hipLaunchKernelGGL((k_expand<MAXE, true, NTT>), dim3(nblk), dim3(NTT), lds, st, a);
    } else {
        set_lds((const void *)&k_expand<MAXE, false, NTT>, lds);
        hipLaunchKernelGGL((k_expand<MAXE, false, NTT>), dim3(nblk), dim3(NTT), lds, st, a);
    }
}

hipError_t launch_expand(const ExpandArgs &a, hipStream_t st)
{
    const int ncb = (a.ncols + a.W - 1) / a.W;
    const unsigned nblk = (unsigned)ncb * (unsigned)a.nbatch;
    const int work = (a.W / 2) * a.fd.N;
    if (nblk == 0) return hipSuccess;
    if (!tile_strides_ok(a.fd.M, a.ors, a.ncols, a.ocs)) return hipErrorInvalidValue;
    if (a.fd.N > 2048) {
        // long transforms: one complex sequence per tile, global twiddles
        const size_t lds = (size_t)a.fd.N * a.W * sizeof(double);
        if (a.W != 2 || work > 8 * 1024) return hipErrorInvalidValue;
        if (work <= 4 * 1024)
            launch_expand_m<4, 1024>(a, nblk, lds, st);
        else
            launch_expand_m<8, 1024>(a, nblk, lds, st);
        return hipGetLastError();
    }
    const size_t lds = (size_t)a.fd.N * sizeof(cx<double>) + (size_t)a.fd.N * (a.W + 1) * sizeof(double);
    if (work <= 4 * NTA)
        launch_expand_m<4>(a, nblk, lds, st);
    else if (work <= 8 * NTA)
        launch_expand_m<8>(a, nblk, lds, st);
    else if (work <= 16 * NTA)
        launch_expand_m<16>(a, nblk, lds, st);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// 1D adjoint in one block: with w = phi_bar on the M+1 nodes,
//   lambda_0 = w_0 + sum_j w_j (1 - j/M),  lambda_M = w_M + sum_j w_j j/M,
//   rho_bar_s = phi_star(w_I)_s + h (G(s h) lambda_0 + G((M - s) h) lambda_M),
// G(r) = r/2, rho_bar on the two end nodes = 0.
template <int MAXE, int NTT>
__global__ __launch_bounds__(NTT) void k_adj_1d(const double *w, double *out, int M, double h,
                                                FftDesc fd, const cx<double> *twg, AxisTabs tab)
{
    constexpr bool BIG = NTT != NTA;
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = fd.N, rs = BIG ? 2 : 3, lgW = 1;
    const cx<double> *tw = BIG ? twg : reinterpret_cast<const cx<double> *>(smem);
    double *buf = reinterpret_cast<double *>(smem + (BIG ? 0 : (size_t)N * sizeof(cx<double>)));
    __shared__ double red[2][NTT];
    if (!BIG) load_twiddles<double, NTT>(reinterpret_cast<cx<double> *>(smem), twg, N);
    double s0 = 0.0, s1 = 0.0;
    for (int j = 1 + threadIdx.x; j < M; j += NTT) {
        s0 += w[j] * ((double)(M - j) / M);
        s1 += w[j] * ((double)j / M);
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    zero_rows<double, NTT>(buf, rs, lgW, 0, 1);
    zero_rows<double, NTT>(buf, rs, lgW, M, N);
    tile_load<double, double, NTT>(buf, rs, 1, w + 1, M - 1, 1, 1, 1, lgW);
    __syncthreads();
    for (int k = NTT / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) {
            red[0][threadIdx.x] += red[0][threadIdx.x + k];
            red[1][threadIdx.x] += red[1][threadIdx.x + k];
        }
        __syncthreads();
    }
    const double l0 = w[0] + red[0][0], l1 = w[M] + red[1][0];
    fft_tile<double, MAXE, NTT>(buf, rs, 0, fd, tw, false);
    post_cs<double, MAXE, NTT>(buf, rs, 0, M);
    for (int k = 1 + threadIdx.x; k < M; k += NTT)
        buf[(M + k) * rs] = -(2.0 / M) * buf[(M + k) * rs] / tab.q[k - 1];
    __syncthreads();
    pre_herm<double, MAXE, NTT>(buf, rs, 0, M, true);
    fft_tile<double, MAXE, NTT>(buf, rs, 0, fd, tw, true);
    for (int j = threadIdx.x; j <= M; j += NTT) {
        double v = 0.0;
        if (j > 0 && j < M)
            v = 0.5 * buf[j * rs] + h * (0.5 * (j * h) * l0 + 0.5 * ((M - j) * h) * l1);
        out[j] = v;
    }
}

hipError_t launch_adj_1d(const double *w, double *out, int M, double h, const FftDesc &fd,
                         const cx<double> *tw, const AxisTabs &tab, hipStream_t st)
{
    if (fd.N > 2048) {
        const size_t lds = (size_t)fd.N * 2 * sizeof(double);
        if (fd.N > 8 * 1024) return hipErrorInvalidValue;
        if (fd.N <= 4 * 1024) {
            set_lds((const void *)&k_adj_1d<4, 1024>, lds);
            hipLaunchKernelGGL((k_adj_1d<4, 1024>), dim3(1), dim3(1024), lds, st, w, out, M, h, fd, tw, tab);
        } else {
            set_lds((const void *)&k_adj_1d<8, 1024>, lds);
            hipLaunchKernelGGL((k_adj_1d<8, 1024>), dim3(1), dim3(1024), lds, st, w, out, M, h, fd, tw, tab);
        }
        return hipGetLastError();
    }
    const size_t lds = (size_t)fd.N * sizeof(cx<double>) + (size_t)fd.N * 3 * sizeof(double);
    if (fd.N <= 4 * NTA) {
        set_lds((const void *)&k_adj_1d<4, NTA>, lds);
        hipLaunchKernelGGL((k_adj_1d<4, NTA>), dim3(1), dim3(NTA), lds, st, w, out, M, h, fd, tw, tab);
    } else if (fd.N <= 8 * NTA) {
        set_lds((const void *)&k_adj_1d<8, NTA>, lds);
        hipLaunchKernelGGL((k_adj_1d<8, NTA>), dim3(1), dim3(NTA), lds, st, w, out, M, h, fd, tw, tab);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace ips
