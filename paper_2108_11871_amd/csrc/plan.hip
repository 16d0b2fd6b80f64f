// Host side of the solver: plans, workspace, the launch sequence of one
// solve, and the C ABI declared in include/ipoisson.h.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "ipoisson.h"
#include "kernels.h"

using namespace ips;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define IPS_HIP(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(IPS_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));          \
    } while (0)

constexpr int kLdsMaxN = 2048; // longest transform whose twiddles are staged in LDS
constexpr int kMaxN3 = 2048;   // 3D: longest transform (2M) per axis
constexpr int kMaxN12 = 8192;  // 1D and 2D: longest transform (one sequence per tile)

// FFT length N = 2M as a list of Stockham radices (8, 4, 2, 3, 5, 7, other primes)
bool factor_fft(int N, FftDesc &fd)
{
    fd.N = N;
    fd.M = N / 2;
    fd.nst = 0;
    int r = N;
    auto push = [&](int R) {
        if (fd.nst >= kMaxStages) return false;
        fd.rad[fd.nst++] = R;
        return true;
    };
    while (r % 8 == 0) {
        if (!push(8)) return false;
        r /= 8;
    }
    while (r % 4 == 0) {
        if (!push(4)) return false;
        r /= 4;
    }
    while (r % 2 == 0) {
        if (!push(2)) return false;
        r /= 2;
    }
    for (int p = 3; r > 1; p += 2) {
        while (r % p == 0) {
            if (!push(p)) return false;
            r /= p;
        }
    }
    int ns = 1;
    for (int st = 0; st < fd.nst; ++st) {
        fd.ns[st] = ns;
        const bool pow2 = (ns & (ns - 1)) == 0;
        fd.nsmag[st] = pow2 ? 0u : (unsigned)((((uint64_t)1 << 32) + ns - 1) / ns);
        int lg = 0;
        while ((1 << lg) < ns) ++lg;
        fd.nslg[st] = lg;
        ns *= fd.rad[st];
    }
    return true;
}

// Device bytes currently allocated by the library (every plan and batch).
std::atomic<int64_t> g_live_bytes{0};
// Allocations made by the calling thread since its current plan creation
// began (failure injection for tests: IPS_TEST_FAIL_ALLOC=k makes the k-th
// allocation of every plan creation fail, k >= 1; any other value, the first).
thread_local int g_alloc_seq = 0;

struct DevBuf {
    std::vector<void *> ptrs;
    std::vector<size_t> sizes;
    size_t bytes = 0;
    int alloc(void **p, size_t n)
    {
        *p = nullptr;
        if (n == 0) n = 8;
        ++g_alloc_seq;
        if (const char *e = getenv("IPS_TEST_FAIL_ALLOC")) {
            const int k = atoi(e) >= 1 ? atoi(e) : 1;
            if (g_alloc_seq >= k)
                return fail(IPS_E_NO_MEMORY, "allocation failure forced by IPS_TEST_FAIL_ALLOC");
        }
        hipError_t e = hipMalloc(p, n);
        if (e != hipSuccess) {
            *p = nullptr;
            (void)hipGetLastError();
            return fail(IPS_E_NO_MEMORY, "hipMalloc of " + std::to_string(n) + " bytes failed");
        }
        ptrs.push_back(*p);
        sizes.push_back(n);
        bytes += n;
        g_live_bytes += (int64_t)n;
        return IPS_OK;
    }
    void release()
    {
        for (size_t i = 0; i < ptrs.size(); ++i) {
            (void)hipFree(ptrs[i]);
            g_live_bytes -= (int64_t)sizes[i];
        }
        ptrs.clear();
        sizes.clear();
        bytes = 0;
    }
};

// Tile budget in complex elements per block (nseq * N): 2048 by default,
// IPS_TILE_WORK (1024, 2048 or 4096) overrides it for every plan, and plans
// created with IPS_FLAG_AUTOTUNE pick their own by measurement.
int tile_work_default()
{
    static const int base = [] {
        const char *e = getenv("IPS_TILE_WORK");
        int v = e ? atoi(e) : 2048;
        if (v != 1024 && v != 2048 && v != 4096) v = 2048;
        return v;
    }();
    return base;
}

// Columns per tile: a power of two, 2 * nseq with nseq * N <= maxwork,
// no wider than the columns present (rounded up to a power of two).
int tile_width(int N, int maxwork, int ncols)
{
    int nseq = 1;
    while (2 * nseq * N <= maxwork) nseq *= 2;
    int W = 2 * nseq;
    int need = 2;
    while (need < ncols) need *= 2;
    return std::min(W, need);
}

// Blocks of a column-contraction launch the chunking aims at (IPS_CC_BLOCKS
// overrides the default, for measurements).
int cc_block_target(int N)
{
    static const int v = [] {
        const char *e = getenv("IPS_CC_BLOCKS");
        const int x = e ? atoi(e) : 0;
        return x >= 256 && x <= 65536 ? x : 0;
    }();
    // fewer chunks (fewer partials for the face pass to sum) up to 2M = 512;
    // the strided pencils of 2M = 1024 measured faster with more blocks
    return v ? v : (N >= 1024 ? 6144 : 4112);
}

// In-face axes (b, c) of the kernel-spectrum table of face family `fam`, in
// storage order K[dd][k_b][k_c] (c contiguous).  The column-contraction
// kernels read K[dd][k_o][k_p] with k_p the transform (pencil) axis.
void kaxes(int d, int fam, int &b, int &c)
{
    if (d == 2) {
        b = 1 - fam;
        c = 0;
        return;
    }
    if (fam == 0) {
        b = 2;
        c = 1; // pencil y, batch slots of z
    } else if (fam == 1) {
        b = 2;
        c = 0; // pencil x, batch slots of z
    } else {
        b = 1;
        c = 0; // pencil x, batch slots of y
    }
}

// Interior nodes of a face of family a (product of I over the other axes).
int64_t shell_size_host(const Geo &g, int a)
{
    int64_t s = 1;
    for (int b = 0; b < g.d; ++b)
        if (b != a) s *= g.M[b] - 1;
    return s;
}

// In-face axes (b, c) of face family f in increasing order (the storage order
// of the surface arrays, c contiguous).
void face_axes(int f, int &b, int &c)
{
    b = f == 0 ? 1 : 0;
    c = f == 2 ? 1 : 2;
}

// Pairs of perpendicular face families (a, b), a < b, with their shared axis c.
void pair_axes(int pr, int &a, int &b, int &c)
{
    a = pr == 2 ? 1 : 0;
    b = pr == 0 ? 1 : 2;
    c = 3 - a - b;
}

} // namespace

struct ips_plan_s {
    int d = 0;
    int64_t n[3] = {1, 1, 1};
    // automatic domain extension: the solve runs on `inner` (the extended
    // grid), the caller's grid sits at ext_off inside it
    ips_plan inner = nullptr;
    int64_t ext_off[3] = {0, 0, 0};
    double *ext_in = nullptr, *ext_out = nullptr; // extended arrays (ext_in zero outside the caller's block)
    double h[3] = {1, 1, 1};
    int order = 6, precision = 0;
    int device = 0;
    int work = 2048; // tile budget (complex elements per block)
    Geo geo{};
    int M[3] = {0, 0, 0}, I[3] = {0, 0, 0}, N[3] = {0, 0, 0};
    FftDesc fd[3]{};
    cx<double> *tw[3] = {nullptr, nullptr, nullptr};
    cx<float> *twf[3] = {nullptr, nullptr, nullptr}; // FP32 twiddles (transforms longer than 2048)
    double *rowtab = nullptr;                          // final pass row table [batch][M0 - 1][12]
    AxisTabs tab[3]{};
    double *K[3] = {nullptr, nullptr, nullptr};
    void *A = nullptr; // slot transforms of rho along one axis (3D)
    void *B = nullptr; // raw DST of rho along the last d-1 axes, then phi in sine space
    double *part[3] = {nullptr, nullptr, nullptr};
    int nch[3] = {1, 1, 1};
    int chunk[3] = {1, 1, 1};
    double *F[3] = {nullptr, nullptr, nullptr};
    double *G[3] = {nullptr, nullptr, nullptr};
    double *T[3] = {nullptr, nullptr, nullptr};
    float *Tf[3] = {nullptr, nullptr, nullptr}; // the same buffer as FP32 (mixed modes)
    double *D[3] = {nullptr, nullptr, nullptr};
    double *P[3] = {nullptr, nullptr, nullptr}; // parity-packed shell spectra
    double *P1T = nullptr;                      // 3D: transposed family-1 copy
    void *P2T = nullptr;                        // 3D: transposed family-2 copy (final pass type)
    bool cube = false; // all families share sizes and chunking (batched launches)
    double *C[3] = {nullptr, nullptr, nullptr}; // sixth-order right-hand side on core layers
    double *r6part = nullptr;                    // split partials of the R_spec contraction (small shells)
    // boundary values from the screening charge (IPS_FLAG_SCREENING)
    bool screen = false;
    double tau[3] = {0, 0, 0};                   // singular corrections of the surface sums
    double *S[3] = {nullptr, nullptr, nullptr};  // face coefficients / sigma [2][I_b][I_c]
    double *src = nullptr;                       // surface nodes [4][nsrc] (direct sums)
    int64_t nsrc = 0, ntgt = 0;
    // 3D surface sums by transforms (surf_fast) instead of the direct sums:
    // tables KP (parallel faces, per family) and KT (perpendicular pairs), and
    // workspace per family (charges, their slot spectra, the parallel sums) and
    // per pair (spectra along the shared axis, overwritten by the transfers,
    // and the sums back on the face nodes)
    bool surf_fast = false;
    double *KP[3] = {nullptr, nullptr, nullptr}, *KT[3] = {nullptr, nullptr, nullptr};
    double *FA[3] = {nullptr, nullptr, nullptr}, *XH[3] = {nullptr, nullptr, nullptr};
    double *PP[3] = {nullptr, nullptr, nullptr};
    double *XA[3] = {nullptr, nullptr, nullptr}, *XB[3] = {nullptr, nullptr, nullptr};
    double *PA[3] = {nullptr, nullptr, nullptr}, *PB[3] = {nullptr, nullptr, nullptr};
    double *QA[3] = {nullptr, nullptr, nullptr}, *QB[3] = {nullptr, nullptr, nullptr};
    DevBuf mem;   // tables: twiddles, axis tables, kernel spectra (and an extended plan's arrays)
    // execution workspace: one block carved into the buffers above (B, A, part, F,
    // G, P, T, D, C, P1T, P2T, rowtab) and, for IPS_FLAG_ADJOINT plans, the adjoint's
    size_t ws_bytes = 0;  // bytes the carving needs
    void *ws = nullptr;   // bound block (plan-owned or the caller's), nullptr: none
    bool ws_adj = false;  // the adjoint buffers are part of the workspace
    DevBuf wsmem;         // plan-owned workspace block
    DevBuf adjmem;        // adjoint buffers of plans without ws_adj (first adjoint call)
    std::mutex exec_mu;   // serialises the enqueue of solves from the ips_solve cache
    // adjoint buffers (in the workspace, or allocated by the first adjoint call)
    bool adj_ready = false;
    double *AX = nullptr, *AY = nullptr, *AX2 = nullptr; // interior volumes
    double *AF = nullptr, *AU = nullptr;                 // grid-shaped (order 6)
    double *AZ = nullptr;                                // 3D expansion scratch
    double *LF[3] = {nullptr, nullptr, nullptr};         // face weights
    double *LH[3] = {nullptr, nullptr, nullptr};         // their slot spectra
    // stage timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> ev_rec;
    double stage_ms[IPS_STAGE_COUNT] = {};
    int64_t stage_calls[IPS_STAGE_COUNT] = {};
};

namespace {

// Tile budget of the final pass.  Its row invariants live in global memory,
// so the LDS holds only the tile: 2048 complex elements (8 columns at
// 2M = 512) measured fastest -- wider tiles (128-byte row segments) lose more
// to occupancy than they gain in coalescing, narrower ones lose coalescing.
int final_work(int precision)
{
    (void)precision;
    return 2048;
}

// Column blocks of the final pass taken together: they cover 256 bytes of
// each row (two 128-byte lines), which measured fastest with the direct
// global I/O of the compile-time stages (257^3: FP32 106 -> 102 us, FP64
// 196 -> 191 us against one line) (IPS_FINAL_GROUP overrides it, for
// measurements).
int final_group(int W, int tsz)
{
    static const int env = [] {
        const char *e = getenv("IPS_FINAL_GROUP");
        return e ? atoi(e) : 0;
    }();
    if (env >= 1 && env <= 16) return env;
    const int g = 256 / (W * tsz);
    return g < 1 ? 1 : g;
}

// LDS bytes of the final pass along axis 0 (tile, twiddles, staged column
// table).
size_t final_pass_lds(int d, const int64_t *n, int precision, int work)
{
    if (d < 2) return 0;
    const int N0 = 2 * (int)(n[0] - 1);
    const size_t tsz = precision != IPS_FP64 ? 4 : 8;
    const int W = tile_width(N0, N0 > kLdsMaxN ? work : final_work(precision), (int)(n[1] - 2));
    // tile (+ twiddles for short transforms) and staged columns; the row
    // invariants live in global memory
    if (N0 > kLdsMaxN) return (size_t)N0 * W * tsz + 8 + (size_t)W * 96;
    return (size_t)N0 * 2 * tsz + (size_t)N0 * (W + 1) * tsz + 8 + (size_t)W * 96;
}

int validate(int d, const int64_t *n, const double *h, int order, int precision, unsigned flags)
{
    if (d < 1 || d > 3) return fail(IPS_E_INVALID_ARG, "d must be 1, 2 or 3");
    if (!n || !h) return fail(IPS_E_INVALID_ARG, "n and h must not be NULL");
    if (flags & ~(IPS_FLAG_STAGE_TIMING | IPS_FLAG_ADJOINT | IPS_FLAG_AUTOTUNE | IPS_FLAG_BATCH_EAGER |
                  IPS_FLAG_NO_WORKSPACE | IPS_FLAG_SCREENING | IPS_FLAG_SCREEN_DIRECT))
        return fail(IPS_E_INVALID_ARG, "unknown flag bits");
    if ((flags & IPS_FLAG_SCREEN_DIRECT) && !(flags & IPS_FLAG_SCREENING))
        return fail(IPS_E_INVALID_ARG, "IPS_FLAG_SCREEN_DIRECT applies to IPS_FLAG_SCREENING plans only");
    if (flags & IPS_FLAG_SCREENING) {
        if (precision != IPS_FP64) return fail(IPS_E_UNSUPPORTED, "the screening variant runs in FP64 only");
        if (flags & IPS_FLAG_ADJOINT) return fail(IPS_E_UNSUPPORTED, "the screening variant has no adjoint");
        if (d >= 2 && n)
            for (int a = 0; a < d; ++a)
                if (n[a] < 7)
                    return fail(IPS_E_INVALID_ARG, "the screening variant needs n[i] >= 7 (surface end weights)");
    }
    if (precision != IPS_FP64 && precision != IPS_MIXED_FP32 && precision != IPS_MIXED_FP32_SLICES)
        return fail(IPS_E_INVALID_ARG, "unknown precision");
    if (d >= 2 && order != 4 && order != 6) return fail(IPS_E_INVALID_ARG, "order must be 4 or 6");
    for (int a = 0; a < d; ++a) {
        if (n[a] < 3) return fail(IPS_E_INVALID_ARG, "every n[i] must be >= 3");
        if (!(h[a] > 0.0) || !std::isfinite(h[a]))
            return fail(IPS_E_INVALID_ARG, "every h[i] must be finite and > 0");
        if (d >= 2 && order == 6 && n[a] < 8)
            return fail(IPS_E_INVALID_ARG, "order 6 needs n[i] >= 8 (extrapolation stencil)");
        const int maxN = d == 3 ? kMaxN3 : kMaxN12;
        if (2 * (n[a] - 1) > maxN)
            return fail(IPS_E_UNSUPPORTED, "n[i] - 1 must not exceed " + std::to_string(maxN / 2) +
                                               (d == 3 ? " in 3D" : " in 1D and 2D"));
    }
    if (d == 1 && precision != IPS_FP64)
        return fail(IPS_E_UNSUPPORTED, "d = 1 runs in FP64 only");
    if (d >= 2 && final_pass_lds(d, n, precision, tile_work_default()) > 160 * 1024)
        return fail(IPS_E_UNSUPPORTED, "n[0] too large for the final pass of this build");
    return IPS_OK;
}

// Host tables of one axis, computed in long double and rounded once.
std::vector<double> axis_tables(int M, double h)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    const int m1 = M - 1;
    std::vector<double> t((size_t)m1 * 7);
    const long double L = (long double)M * h;
    for (int k = 1; k < M; ++k) {
        const long double s = sinl(pi * k / (2.0L * M));
        t[k - 1] = (double)(-(4.0L / ((long double)h * h)) * s * s);
        const long double q = pi * k / L;
        t[m1 + k - 1] = (double)(q * q);
        for (int j = 1; j <= 5; ++j) {
            const long long r = ((long long)k * j) % (2LL * M);
            t[(size_t)(1 + j) * m1 + k - 1] = (double)sinl(pi * (long double)r / M);
        }
    }
    return t;
}

std::vector<cx<double>> twiddles(int N)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<cx<double>> w(N);
    for (int t = 0; t < N; ++t) {
        const long double a = 2.0L * pi * t / N;
        w[t] = {(double)cosl(a), (double)(-sinl(a))};
    }
    return w;
}

// Transform description and tile width of a pass along an axis (fd, tw).
void prep_pass(ips_plan p, PassArgs &a, const FftDesc &fd, const cx<double> *tw)
{
    a.fd = fd;
    a.tw = tw;
    a.twf = nullptr;
    for (int ax = 0; ax < p->d; ++ax)
        if (p->tw[ax] == tw) a.twf = p->twf[ax];
    if (a.W == 0) a.W = tile_width(fd.N, p->work, a.ncols);
}

// f32t: FP32 tiles between FP64 input and output
int run_pass(ips_plan p, PassArgs a, const FftDesc &fd, const cx<double> *tw, bool in_f32,
             bool out_f32, hipStream_t st, bool f32t = false)
{
    prep_pass(p, a, fd, tw);
    if (f32t && !in_f32 && !out_f32)
        IPS_HIP(launch_pass_f32t(a, st));
    else
        IPS_HIP(launch_pass(a, in_f32, out_f32, st));
    return IPS_OK;
}

// Tile width of the forward slot passes of rho: with FP32 tiles and
// transforms of 1024 points (513^3), twice the plan's budget, whose 8-column
// tiles read 64-byte runs of the strided rho rows (rho_y 1.43 -> 1.13 ms at
// 513^3; at 2M = 512 the default measured faster).  0 keeps the plan's default.
int rho_pass_width(ips_plan p, int N, int ncols, bool f32)
{
    if (!f32 || N < 1024 || N > kLdsMaxN || 2 * p->work > 4096) return 0;
    return tile_width(N, 2 * p->work, ncols);
}

// Independent passes (prepared) in one launch when their transforms fit the
// multi-pass kernel, else one launch each.
int run_passes(PassArgs *a, int n, bool in_f32, bool out_f32, hipStream_t st)
{
    bool fit = n > 1 && n <= kMultiPass;
    for (int i = 0; i < n; ++i) fit = fit && a[i].fd.N <= kLdsMaxN;
    if (fit) {
        IPS_HIP(launch_pass_multi(a, n, in_f32, out_f32, st));
        return IPS_OK;
    }
    for (int i = 0; i < n; ++i) IPS_HIP(launch_pass(a[i], in_f32, out_f32, st));
    return IPS_OK;
}

// Forward raw DST (IN_ZPAD -> S rows) or inverse (IN_SPECS -> real rows) of
// the last two (or one) axes of a stack of shell layers [nl][I_b][I_c]:
// the prepared pass of step 0 (along the contiguous axis) or step 1 (3D:
// along the lower axis).  Returns the number of steps.
int shell_dst_pass(ips_plan p, void *buf, int nl, int fam, bool inverse, int step, PassArgs &a)
{
    int ax[2], na = 0;
    for (int b = 0; b < p->d; ++b)
        if (b != fam) ax[na++] = b;
    const int last = ax[na - 1];
    const int64_t plane = na == 2 ? (int64_t)p->I[ax[0]] * p->I[ax[1]] : p->I[ax[0]];
    int axis, ncols, nbatch;
    int64_t rstride, cstride, bstride;
    if (na == 2 && step == 0) {
        // along the contiguous axis: rows stride 1, columns = lower axis
        axis = last, rstride = 1, cstride = p->I[last], ncols = p->I[ax[0]], nbatch = nl, bstride = plane;
    } else if (na == 2) {
        axis = ax[0], rstride = p->I[last], cstride = 1, ncols = p->I[last], nbatch = nl, bstride = plane;
    } else {
        axis = last, rstride = 1, cstride = plane, ncols = nl, nbatch = 1, bstride = 0;
    }
    a = PassArgs{};
    a.in = buf;
    a.out = buf;
    a.irs = a.ors = rstride;
    a.ics = a.ocs = cstride;
    a.ibs = a.obs = bstride;
    a.nrows_in = p->I[axis];
    a.ncols = ncols;
    a.nbatch = nbatch;
    a.in_mode = inverse ? IN_SPECS : IN_ZPAD;
    a.out_r0 = inverse ? 1 : p->M[axis] + 1;
    a.out_nrows = p->I[axis];
    a.scale = inverse ? 0.5 : 1.0;
    prep_pass(p, a, p->fd[axis], p->tw[axis]);
    return na;
}

int shell_dst(ips_plan p, void *buf, int nl, int fam, bool inverse, hipStream_t st, bool f32 = false)
{
    PassArgs a;
    const int nstep = shell_dst_pass(p, buf, nl, fam, inverse, 0, a);
    IPS_HIP(launch_pass(a, f32, f32, st));
    if (nstep == 2) {
        shell_dst_pass(p, buf, nl, fam, inverse, 1, a);
        IPS_HIP(launch_pass(a, f32, f32, st));
    }
    return IPS_OK;
}

// Shell layer transforms of all families: one launch per direction when the
// families are uniform (contiguous buffers of identical shape), else the
// families' passes of each step together in one multi-pass launch.
template <typename TS>
int shell_dst_all(ips_plan p, TS *const *arr, int nl, bool inverse, hipStream_t st)
{
    constexpr bool f32 = sizeof(TS) == 4;
    if (p->cube) return shell_dst(p, arr[0], nl * p->d, 0, inverse, st, f32);
    PassArgs a[3];
    int nstep = 1, rc;
    for (int step = 0; step < nstep; ++step) {
        for (int fam = 0; fam < p->d; ++fam) nstep = shell_dst_pass(p, arr[fam], nl, fam, inverse, step, a[fam]);
        if ((rc = run_passes(a, p->d, f32, f32, st))) return rc;
    }
    return IPS_OK;
}

// Regularised value of  integral over R^2 of 1/|x|  -  a b sum over x_j != 0
// of 1/|x_j|  for the lattice x_j = (m a, n b): the constant that makes the
// punctured trapezoidal rule third-order accurate at a 1/r singularity.
// Ewald split 1/r = erfc(s r)/r + erf(s r)/r: the first part is summed over
// the lattice directly, the second through Poisson summation over the
// reciprocal lattice (2 pi m/a, 2 pi n/b), where its transform is
// (2 pi/k) erfc(k/(2 s)); the removed k = 0 and r = 0 terms give
// 2 sqrt(pi)/s and 2 s a b / sqrt(pi).
double lattice_constant(double a, double b)
{
    const double pi = 3.141592653589793238462643383279502884;
    const double area = a * b, s = 1.5 / std::sqrt(area), reach = 12.0;
    const int mr = (int)std::ceil(reach / (s * a)), nr = (int)std::ceil(reach / (s * b));
    long double real = 0.0L;
    for (int m = -mr; m <= mr; ++m)
        for (int n = -nr; n <= nr; ++n) {
            if (m == 0 && n == 0) continue;
            const double r = std::hypot(m * a, n * b);
            real += (long double)(std::erfc(s * r) / r);
        }
    const int km = (int)std::ceil(s * reach * a / pi), kn = (int)std::ceil(s * reach * b / pi);
    long double rec = 0.0L;
    for (int m = -km; m <= km; ++m)
        for (int n = -kn; n <= kn; ++n) {
            if (m == 0 && n == 0) continue;
            const double k = std::hypot(2.0 * pi * m / a, 2.0 * pi * n / b);
            rec += (long double)(2.0 * pi / k * std::erfc(k / (2.0 * s)));
        }
    return (double)(2.0L * std::sqrt((long double)pi) / s - (long double)area * real - rec +
                    2.0L * s * area / std::sqrt((long double)pi));
}

// Sub-buffers carved out of one device block, 256-byte aligned; with a null
// base only the size is measured.
struct Carver {
    char *base = nullptr;
    size_t off = 0;
    template <typename T>
    void take(T **ptr, size_t bytes)
    {
        off = (off + 255) & ~(size_t)255;
        *ptr = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += bytes ? bytes : 8;
    }
};

void layout_adj(ips_plan p, Carver &c);

// The execution workspace of a plan (everything one solve writes besides phi):
// the sine-space volume B, the slot array A, the chunk partials, face values,
// shell layers, the final pass's row table and, for plans with ws_adj, the
// adjoint's buffers.  Assigns the plan's pointers from c.base.
void layout_ws(ips_plan p, Carver &c)
{
    const int d = p->d;
    if (d == 1) return;
    const int *I = p->I, *M = p->M, *N = p->N;
    size_t vol = 1, grid = 1;
    for (int a = 0; a < d; ++a) {
        vol *= (size_t)I[a];
        grid *= (size_t)p->n[a];
    }
    const size_t wsz = p->precision != IPS_FP64 ? sizeof(float) : sizeof(double);
    const size_t asz = p->precision == IPS_MIXED_FP32_SLICES ? sizeof(float) : sizeof(double);
    c.take(&p->B, vol * wsz);
    c.take(&p->rowtab, (d == 3 ? (size_t)I[2] : 1) * I[0] * 12 * sizeof(double));
    if (p->screen) {
        // no slice transforms or chunk partials: the face coefficients of the
        // screening charge and the surface node list instead
        size_t ts = 0;
        for (int fam = 0; fam < d; ++fam) {
            size_t f = 1;
            for (int b = 0; b < d; ++b)
                if (b != fam) f *= (size_t)I[b];
            ts += f;
        }
        double *bs;
        c.take(&bs, 2 * ts * sizeof(double));
        if (p->surf_fast) {
            for (int f = 0; f < 3; ++f) {
                int b, cc;
                face_axes(f, b, cc);
                const size_t face = (size_t)(M[b] + 1) * (M[cc] + 1);
                c.take(&p->FA[f], 2 * face * sizeof(double));
                c.take(&p->XH[f], 2 * (size_t)N[b] * N[cc] * sizeof(double));
                c.take(&p->PP[f], 2 * face * sizeof(double));
            }
            for (int pr = 0; pr < 3; ++pr) {
                int a, b, cc;
                pair_axes(pr, a, b, cc);
                c.take(&p->XA[pr], 2 * (size_t)(M[b] + 1) * N[cc] * sizeof(double));
                c.take(&p->XB[pr], 2 * (size_t)(M[a] + 1) * N[cc] * sizeof(double));
                const size_t G = (size_t)perp_groups(M, pr);
                c.take(&p->PA[pr], 4 * G * (M[b] + 1) * N[cc] * sizeof(double));
                c.take(&p->PB[pr], 4 * (size_t)(M[a] + 1) * N[cc] * sizeof(double));
                c.take(&p->QA[pr], 2 * (size_t)(M[b] + 1) * (M[cc] + 1) * sizeof(double));
                c.take(&p->QB[pr], 2 * (size_t)(M[a] + 1) * (M[cc] + 1) * sizeof(double));
            }
        } else {
            c.take(&p->src, 4 * 2 * ts * sizeof(double));
        }
        size_t os = 0;
        for (int fam = 0; fam < 3; ++fam) {
            p->S[fam] = nullptr;
            if (fam >= d || !c.base) continue;
            size_t f = 1;
            for (int b = 0; b < d; ++b)
                if (b != fam) f *= (size_t)I[b];
            p->S[fam] = bs + os;
            os += 2 * f;
        }
    }
    if (d == 3 && !p->screen) {
        const size_t a1 = (size_t)I[0] * I[1] * N[2], a2 = (size_t)I[0] * N[1] * I[2];
        c.take(&p->A, std::max(a1, a2) * asz);
    } else {
        p->A = nullptr;
    }
    // per-family sizes, one contiguous buffer per kind (families back to back)
    size_t fsz[3] = {0, 0, 0}, ssz[3] = {0, 0, 0};
    size_t tp = 0, tf = 0, ts = 0;
    for (int fam = 0; fam < d; ++fam) {
        fsz[fam] = 2;
        ssz[fam] = 1;
        for (int b = 0; b < d; ++b)
            if (b != fam) {
                fsz[fam] *= (size_t)N[b];
                ssz[fam] *= (size_t)I[b];
            }
        tp += fsz[fam] * p->nch[fam];
        tf += fsz[fam];
        ts += ssz[fam];
    }
    double *bp = nullptr, *bf = nullptr, *bg, *bpk, *bt = nullptr, *bd = nullptr, *bc = nullptr;
    if (!p->screen) {
        c.take(&bp, tp * sizeof(double));
        c.take(&bf, tf * sizeof(double));
    }
    c.take(&bg, 2 * ts * sizeof(double));
    c.take(&bpk, 6 * ts * sizeof(double));
    p->r6part = nullptr;
    if (p->order == 6) {
        c.take(&bt, 10 * ts * sizeof(double));
        c.take(&bd, 4 * ts * sizeof(double));
        c.take(&bc, 8 * ts * sizeof(double));
        const int ks = r6t_splits(p->geo);
        if (ks > 1) c.take(&p->r6part, (size_t)ks * 10 * ts * sizeof(double));
    }
    size_t op = 0, of = 0, os = 0;
    for (int fam = 0; fam < 3; ++fam) {
        p->part[fam] = p->F[fam] = p->G[fam] = p->P[fam] = p->T[fam] = p->D[fam] = p->C[fam] = nullptr;
        p->Tf[fam] = nullptr;
    }
    if (c.base)
        for (int fam = 0; fam < d; ++fam) {
            p->part[fam] = bp ? bp + op : nullptr;
            p->F[fam] = bf ? bf + of : nullptr;
            p->G[fam] = bg + 2 * os;
            p->P[fam] = bpk + 6 * os;
            if (bt) {
                p->T[fam] = bt + 10 * os;
                p->Tf[fam] = reinterpret_cast<float *>(bt) + 10 * os;
            }
            if (bd) p->D[fam] = bd + 4 * os;
            if (bc) p->C[fam] = bc + 8 * os;
            op += fsz[fam] * p->nch[fam];
            of += fsz[fam];
            os += ssz[fam];
        }
    if (d == 3) {
        c.take(&p->P1T, 6 * ssz[1] * sizeof(double));
        c.take(&p->P2T, 6 * ssz[2] * sizeof(double));
    }
    if (p->ws_adj) layout_adj(p, c);
}

// The adjoint's buffers: three interior volumes, two grids (order 6), face
// weights and their spectra, and one slice stack (3D).
void layout_adj(ips_plan p, Carver &c)
{
    const int d = p->d;
    const int *I = p->I, *M = p->M, *N = p->N;
    size_t vol = 1, grid = 1;
    for (int a = 0; a < d; ++a) {
        vol *= (size_t)I[a];
        grid *= (size_t)p->n[a];
    }
    c.take(&p->AX, vol * sizeof(double));
    c.take(&p->AY, vol * sizeof(double));
    if (p->order == 6) {
        c.take(&p->AX2, vol * sizeof(double));
        c.take(&p->AF, grid * sizeof(double));
        c.take(&p->AU, grid * sizeof(double));
    }
    size_t zmax = 0;
    for (int fam = 0; fam < d; ++fam) {
        int b, cc;
        kaxes(d, fam, b, cc);
        const size_t lf = 2 * (size_t)(M[b] + 1) * (d == 3 ? (size_t)(M[cc] + 1) : 1);
        const size_t lh = 2 * (size_t)N[b] * (d == 3 ? (size_t)N[cc] : 1);
        c.take(&p->LF[fam], lf * sizeof(double));
        c.take(&p->LH[fam], lh * sizeof(double));
        if (d == 3) zmax = std::max(zmax, (size_t)I[fam] * N[b] * I[cc]);
    }
    // order 6 also uses it as one grid-shaped scratch array (adjoint stencil)
    if (d == 3 && p->order == 6) zmax = std::max(zmax, grid);
    if (d == 3) c.take(&p->AZ, zmax * sizeof(double));
}

// Point the plan's buffers into `base` (size checked by the caller), or
// detach them (base = nullptr).
void bind_ws(ips_plan p, void *base)
{
    Carver c;
    c.base = static_cast<char *>(base);
    p->ws = base;
    if (base) {
        layout_ws(p, c);
        if (p->ws_adj) p->adj_ready = true;
    } else if (p->ws_adj) {
        p->adj_ready = false;
    }
}

size_t measure_ws(ips_plan p)
{
    Carver c;
    layout_ws(p, c);
    return p->d == 1 ? 0 : c.off;
}

int plan_build(ips_plan p, hipStream_t st)
{
    const int d = p->d;
    Geo &g = p->geo;
    g.d = d;
    g.pref = 1.0;
    for (int a = 0; a < 3; ++a) {
        g.M[a] = a < d ? p->M[a] : 1;
        g.h[a] = a < d ? p->h[a] : 1.0;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            g.c2[i][j] = (g.h[i] * g.h[i] + g.h[j] * g.h[j]) / 12.0;
            g.c4[i][j] = g.h[i] * g.h[i] * g.h[i] * g.h[i] / 240.0 +
                         g.h[i] * g.h[i] * g.h[j] * g.h[j] / 144.0;
        }
    for (int a = 0; a < d; ++a) g.pref *= 2.0 / p->M[a];

    for (int a = 0; a < d; ++a) {
        if (!factor_fft(p->N[a], p->fd[a])) return fail(IPS_E_UNSUPPORTED, "FFT length not factorable");
        std::vector<cx<double>> w = twiddles(p->N[a]);
        int rc = p->mem.alloc((void **)&p->tw[a], w.size() * sizeof(cx<double>));
        if (rc) return rc;
        IPS_HIP(hipMemcpy(p->tw[a], w.data(), w.size() * sizeof(cx<double>), hipMemcpyHostToDevice));
        if (p->N[a] > kLdsMaxN) {
            // long transforms read their twiddles from global memory: FP32 copy
            std::vector<cx<float>> wf(w.size());
            for (size_t t = 0; t < w.size(); ++t) wf[t] = {(float)w[t].x, (float)w[t].y};
            rc = p->mem.alloc((void **)&p->twf[a], wf.size() * sizeof(cx<float>));
            if (rc) return rc;
            IPS_HIP(hipMemcpy(p->twf[a], wf.data(), wf.size() * sizeof(cx<float>), hipMemcpyHostToDevice));
        }
        std::vector<double> t = axis_tables(p->M[a], p->h[a]);
        double *dt = nullptr;
        rc = p->mem.alloc((void **)&dt, t.size() * sizeof(double));
        if (rc) return rc;
        IPS_HIP(hipMemcpy(dt, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
        const int m1 = p->M[a] - 1;
        p->tab[a].lam = dt;
        p->tab[a].q = dt + m1;
        p->tab[a].s = dt + 2 * m1;
    }
    if (d == 1) return IPS_OK;

    const int *I = p->I, *M = p->M, *N = p->N;
    int rc;
    for (int fam = 0; fam < d; ++fam) {
        // chunking of the contraction over the face-normal axis (column-contraction kernel)
        int pen, nbatch;
        if (d == 3) {
            pen = fam == 0 ? 1 : 0;
            nbatch = fam == 2 ? N[1] : N[2];
        } else {
            pen = 1 - fam;
            nbatch = 1;
        }
        // a tile holds W/2 columns of the first half of the axis and their
        // mirrors: the chunks split the (I + 1)/2 first-half columns
        const int W = tile_width(N[pen], p->work, I[fam]);
        const int hc = (I[fam] + 1) / 2, Wh = W / 2;
        const int ncb = (hc + Wh - 1) / Wh;
        // about 4096 (2M <= 512) or 6144 blocks of 256 threads, a few tiles
        // each (more chunks give more blocks but more partials for the face
        // pass to sum); 256 blocks of 1024 for long transforms
        const int target = N[pen] > kLdsMaxN ? 256 : cc_block_target(N[pen]);
        int nch = std::max(1, std::min(ncb, (target + nbatch - 1) / nbatch));
        const int per = (ncb + nch - 1) / nch;
        p->chunk[fam] = per * Wh;
        p->nch[fam] = (hc + per * Wh - 1) / (per * Wh);
    }
    // uniform families: one launch covers the three (two in 2D) families
    p->cube = true;
    for (int fam = 1; fam < d; ++fam)
        if (M[fam] != M[0] || p->nch[fam] != p->nch[0]) p->cube = false;
    if (p->screen) {
        // singular corrections of the surface sums (targets inside a face)
        const double pi = 3.141592653589793238462643383279502884;
        for (int fam = 0; fam < d; ++fam) {
            if (d == 3) {
                const int b = fam == 0 ? 1 : 0, c = fam == 2 ? 1 : 2;
                p->tau[fam] = -lattice_constant(p->h[b], p->h[c]) / (4.0 * pi);
            } else {
                const double hb = p->h[1 - fam];
                p->tau[fam] = hb * std::log(hb / (2.0 * pi)) / (2.0 * pi);
            }
        }
        size_t ts = 0;
        for (int fam = 0; fam < d; ++fam) {
            size_t f = 1;
            for (int b = 0; b < d; ++b)
                if (b != fam) f *= (size_t)I[b];
            ts += f;
        }
        p->nsrc = (int64_t)(2 * ts);
        const int64_t n0 = p->n[0], n1 = p->n[1], n2 = d == 3 ? p->n[2] : 1;
        p->ntgt = 2 * n1 * n2 + 2 * (n0 - 2) * n2 + (d == 3 ? 2 * (n0 - 2) * (n1 - 2) : 0);
        if (!p->surf_fast) return IPS_OK; // no tables: direct surface sums
        // parallel faces of family f: G at in-plane offsets on the same face and
        // on the opposite one, even transforms along c then b
        for (int f = 0; f < 3; ++f) {
            int b, c;
            face_axes(f, b, c);
            const int64_t plane = (int64_t)(M[b] + 1) * (M[c] + 1);
            if ((rc = p->mem.alloc((void **)&p->KP[f], 2 * plane * sizeof(double)))) return rc;
            IPS_HIP(launch_par_sample(p->KP[f], f, M, p->h, st));
            PassArgs a{};
            a.in = a.out = p->KP[f];
            a.irs = a.ors = 1;
            a.ics = a.ocs = M[c] + 1;
            a.ibs = a.obs = plane;
            a.nrows_in = M[c] + 1;
            a.ncols = M[b] + 1;
            a.nbatch = 2;
            a.in_mode = IN_EVEN;
            a.out_r0 = 0;
            a.out_nrows = M[c] + 1;
            a.scale = 1.0;
            if ((rc = run_pass(p, a, p->fd[c], p->tw[c], false, false, st))) return rc;
            PassArgs b2 = a;
            b2.irs = b2.ors = M[c] + 1;
            b2.ics = b2.ocs = 1;
            b2.nrows_in = M[b] + 1;
            b2.ncols = M[c] + 1;
            b2.out_nrows = M[b] + 1;
            b2.W = 0;
            if ((rc = run_pass(p, b2, p->fd[b], p->tw[b], false, false, st))) return rc;
        }
        // perpendicular pairs (a, b): G at (i h_a, j h_b, dc h_c), even
        // transform along dc
        for (int pr = 0; pr < 3; ++pr) {
            int a, b, c;
            pair_axes(pr, a, b, c);
            const int64_t slab = (int64_t)(M[a] + 1) * (M[b] + 1);
            if ((rc = p->mem.alloc((void **)&p->KT[pr], (size_t)(M[c] + 1) * slab * sizeof(double)))) return rc;
            IPS_HIP(launch_perp_sample(p->KT[pr], a, b, c, M, p->h, st));
            PassArgs t{};
            t.in = t.out = p->KT[pr];
            t.irs = t.ors = slab;
            t.ics = t.ocs = 1;
            t.nrows_in = M[c] + 1;
            t.ncols = (int)slab;
            t.nbatch = 1;
            t.in_mode = IN_EVEN;
            t.out_r0 = 0;
            t.out_nrows = M[c] + 1;
            t.scale = 1.0;
            if ((rc = run_pass(p, t, p->fd[c], p->tw[c], false, false, st))) return rc;
        }
        return IPS_OK;
    }
    for (int fam = 0; fam < d; ++fam) {
        // kernel spectra: samples then even transforms along the in-face axes
        size_t ksz = (size_t)I[fam];
        for (int b = 0; b < d; ++b)
            if (b != fam) ksz *= (size_t)(M[b] + 1);
        if ((rc = p->mem.alloc((void **)&p->K[fam], ksz * sizeof(double)))) return rc;
        int kb, kc;
        kaxes(d, fam, kb, kc);
        IPS_HIP(launch_ksample(p->K[fam], d, fam, kb, kc, M, p->h, st));
        if (d == 2) {
            PassArgs a{};
            a.in = a.out = p->K[fam];
            a.irs = a.ors = 1;
            a.ics = a.ocs = M[kb] + 1;
            a.nrows_in = M[kb] + 1;
            a.ncols = I[fam];
            a.nbatch = 1;
            a.in_mode = IN_EVEN;
            a.out_r0 = 0;
            a.out_nrows = M[kb] + 1;
            a.scale = 1.0;
            if ((rc = run_pass(p, a, p->fd[kb], p->tw[kb], false, false, st))) return rc;
        } else {
            const int64_t plane = (int64_t)(M[kb] + 1) * (M[kc] + 1);
            PassArgs a{};
            a.in = a.out = p->K[fam];
            a.irs = a.ors = 1;
            a.ics = a.ocs = M[kc] + 1;
            a.ibs = a.obs = plane;
            a.nrows_in = M[kc] + 1;
            a.ncols = M[kb] + 1;
            a.nbatch = I[fam];
            a.in_mode = IN_EVEN;
            a.out_r0 = 0;
            a.out_nrows = M[kc] + 1;
            a.scale = 1.0;
            if ((rc = run_pass(p, a, p->fd[kc], p->tw[kc], false, false, st))) return rc;
            PassArgs b2{};
            b2.in = b2.out = p->K[fam];
            b2.irs = b2.ors = M[kc] + 1;
            b2.ics = b2.ocs = 1;
            b2.ibs = b2.obs = plane;
            b2.nrows_in = M[kb] + 1;
            b2.ncols = M[kc] + 1;
            b2.nbatch = I[fam];
            b2.in_mode = IN_EVEN;
            b2.out_r0 = 0;
            b2.out_nrows = M[kb] + 1;
            b2.scale = 1.0;
            if ((rc = run_pass(p, b2, p->fd[kb], p->tw[kb], false, false, st))) return rc;
        }
    }
    return IPS_OK;
}

struct StageScope {
    ips_plan p;
    int stage;
    hipStream_t st;
    hipError_t err = hipSuccess;
    hipEvent_t e1 = nullptr;
    static hipError_t get(ips_plan p, hipEvent_t *e)
    {
        if (p->ev_used < p->ev_pool.size()) {
            *e = p->ev_pool[p->ev_used++];
            return hipSuccess;
        }
        hipError_t r = hipEventCreate(e);
        if (r != hipSuccess) return r;
        p->ev_pool.push_back(*e);
        ++p->ev_used;
        return hipSuccess;
    }
    StageScope(ips_plan p_, int s_, hipStream_t st_) : p(p_), stage(s_), st(st_)
    {
        if (!p->timing) return;
        hipEvent_t e0;
        if ((err = get(p, &e0)) != hipSuccess) return;
        if ((err = get(p, &e1)) != hipSuccess) return;
        err = hipEventRecord(e0, st);
        p->ev_rec.emplace_back(stage, e0, e1);
    }
    ~StageScope()
    {
        if (p->timing && e1) (void)hipEventRecord(e1, st);
    }
};

#define IPS_CAT2(a, b) a##b
#define IPS_CAT(a, b) IPS_CAT2(a, b)
#define STAGE(id) StageScope IPS_CAT(stage_scope_, __LINE__)(p, (id), st)

// 3D surface sums by transforms (sigma already on the faces): face charges
// W sigma; slot spectra of every face over both face axes and of every face
// along each of its axes; the parallel-face products and the perpendicular
// transfers; the inverse transforms; g at every boundary node.
int surface_sums(ips_plan p, double *phi, hipStream_t st)
{
    const int *M = p->M, *N = p->N;
    int rc;
    SurfArgs s{};
    for (int a = 0; a < 3; ++a) {
        s.M[a] = M[a];
        s.h[a] = p->h[a];
        s.tau[a] = p->tau[a];
        s.sig[a] = p->S[a];
        s.FA[a] = p->FA[a];
        s.XH[a] = p->XH[a];
        s.KP[a] = p->KP[a];
        s.PP[a] = p->PP[a];
        s.XA[a] = p->XA[a];
        s.XB[a] = p->XB[a];
        s.PA[a] = p->PA[a];
        s.PB[a] = p->PB[a];
        s.QA[a] = p->QA[a];
        s.QB[a] = p->QB[a];
        s.KT[a] = p->KT[a];
        s.groups[a] = perp_groups(M, a);
    }
    IPS_HIP(launch_face_charge(s, st));
    // face f along its axis x (o the other face axis), slot q of side s and
    // node m of axis o to out[q ors + s obs + m ocs]
    auto along = [&](int f, int x, double *out, int64_t ors, int64_t ocs, int64_t obs) -> PassArgs {
        int b, c;
        face_axes(f, b, c);
        const int o = x == c ? b : c;
        PassArgs a{};
        a.in = p->FA[f];
        a.out = out;
        a.irs = x == c ? 1 : M[c] + 1;
        a.ics = x == c ? M[c] + 1 : 1;
        a.ibs = (int64_t)(M[b] + 1) * (M[c] + 1);
        a.ors = ors;
        a.ocs = ocs;
        a.obs = obs;
        a.nrows_in = M[x] + 1;
        a.ncols = M[o] + 1;
        a.nbatch = 2;
        a.in_mode = IN_ZPAD0;
        a.out_r0 = 0;
        a.out_nrows = N[x];
        a.scale = 1.0;
        prep_pass(p, a, p->fd[x], p->tw[x]);
        return a;
    };
    // back on the nodes along the shared axis x, the sum of ncopy partials:
    // in[N_x][ncopy][2][M_o + 1] -> out[2][M_o + 1][M_x + 1]
    auto back = [&](const double *in, double *out, int x, int o, int ncopy) -> PassArgs {
        PassArgs a{};
        a.in = in;
        a.out = out;
        a.irs = (int64_t)ncopy * 2 * (M[o] + 1);
        a.ics = 1;
        a.ibs = M[o] + 1;
        a.nsum = ncopy;
        a.sstride = 2 * (int64_t)(M[o] + 1);
        a.ors = 1;
        a.ocs = M[x] + 1;
        a.obs = (int64_t)(M[o] + 1) * (M[x] + 1);
        a.nrows_in = N[x];
        a.ncols = M[o] + 1;
        a.nbatch = 2;
        a.in_mode = IN_HERM;
        a.out_r0 = 0;
        a.out_nrows = M[x] + 1;
        a.scale = 1.0 / N[x];
        prep_pass(p, a, p->fd[x], p->tw[x]);
        return a;
    };
    // The passes of the three faces (or pairs) of each step are independent:
    // one multi-pass launch per step.
    PassArgs g1[3], g2[3];
    for (int f = 0; f < 3; ++f) {
        int b, c;
        face_axes(f, b, c);
        // along c into [2][N_b][N_c] (rows 0..M_b), then along b in place
        g1[f] = along(f, c, p->XH[f], 1, N[c], (int64_t)N[b] * N[c]);
        PassArgs &a = g2[f];
        a = PassArgs{};
        a.in = a.out = p->XH[f];
        a.irs = a.ors = N[c];
        a.ics = a.ocs = 1;
        a.ibs = a.obs = (int64_t)N[b] * N[c];
        a.nrows_in = M[b] + 1;
        a.ncols = N[c];
        a.nbatch = 2;
        a.in_mode = IN_ZPAD0;
        a.out_r0 = 0;
        a.out_nrows = N[b];
        a.scale = 1.0;
        prep_pass(p, a, p->fd[b], p->tw[b]);
    }
    if ((rc = run_passes(g1, 3, false, false, st))) return rc;
    if ((rc = run_passes(g2, 3, false, false, st))) return rc;
    for (int pr = 0; pr < 3; ++pr) {
        int a, b, c;
        pair_axes(pr, a, b, c);
        g1[pr] = along(a, c, p->XA[pr], 2 * (int64_t)(M[b] + 1), 1, M[b] + 1);
        g2[pr] = along(b, c, p->XB[pr], 2 * (int64_t)(M[a] + 1), 1, M[a] + 1);
    }
    if ((rc = run_passes(g1, 3, false, false, st))) return rc;
    if ((rc = run_passes(g2, 3, false, false, st))) return rc;
    IPS_HIP(launch_par_mul(s, st));
    for (int f = 0; f < 3; ++f) {
        int b, c;
        face_axes(f, b, c);
        // synthesis along b in place (rows 0..M_b), then along c into PP
        PassArgs &a = g1[f];
        a = PassArgs{};
        a.in = a.out = p->XH[f];
        a.irs = a.ors = N[c];
        a.ics = a.ocs = 1;
        a.ibs = a.obs = (int64_t)N[b] * N[c];
        a.nrows_in = N[b];
        a.ncols = N[c];
        a.nbatch = 2;
        a.in_mode = IN_HERM;
        a.out_r0 = 0;
        a.out_nrows = M[b] + 1;
        a.scale = 1.0 / N[b];
        prep_pass(p, a, p->fd[b], p->tw[b]);
        PassArgs &z = g2[f];
        z = PassArgs{};
        z.in = p->XH[f];
        z.out = p->PP[f];
        z.irs = 1;
        z.ics = N[c];
        z.ibs = (int64_t)N[b] * N[c];
        z.ors = 1;
        z.ocs = M[c] + 1;
        z.obs = (int64_t)(M[b] + 1) * (M[c] + 1);
        z.nrows_in = N[c];
        z.ncols = M[b] + 1;
        z.nbatch = 2;
        z.in_mode = IN_HERM;
        z.out_r0 = 0;
        z.out_nrows = M[c] + 1;
        z.scale = 1.0 / N[c];
        prep_pass(p, z, p->fd[c], p->tw[c]);
    }
    if ((rc = run_passes(g1, 3, false, false, st))) return rc;
    if ((rc = run_passes(g2, 3, false, false, st))) return rc;
    IPS_HIP(launch_perp(s, st));
    for (int pr = 0; pr < 3; ++pr) {
        int a, b, c;
        pair_axes(pr, a, b, c);
        g1[pr] = back(p->PA[pr], p->QA[pr], c, b, 2 * s.groups[pr]);
        g2[pr] = back(p->PB[pr], p->QB[pr], c, a, 2);
    }
    if ((rc = run_passes(g1, 3, false, false, st))) return rc;
    if ((rc = run_passes(g2, 3, false, false, st))) return rc;
    IPS_HIP(launch_surf_assemble(s, phi, st));
    return IPS_OK;
}

// Boundary values from the screening charge (d = 2, 3): the raw sine spectrum
// of rho_I over all axes into B, in the final pass's layout ([k2][k0][k1],
// 2D [k0][k1]); the face coefficients of sigma = d phi*/dn; sigma on the
// faces by inverse sine transforms over the in-face axes; the corrected
// surface sums at every boundary node of phi.
int screen_boundary(ips_plan p, const double *rho, double *phi, hipStream_t st)
{
    const int d = p->d;
    const int *I = p->I, *M = p->M;
    const int64_t *n = p->n;
    int rc;
    {
        STAGE(IPS_STAGE_RHO_Z);
        PassArgs a{};
        a.in_mode = IN_ZPAD;
        a.scale = 1.0;
        if (d == 3) {
            // along z: rho[x][y][z] -> B[kz][x][y]
            a.in = rho + n[1] * n[2] + n[2] + 1;
            a.out = p->B;
            a.irs = 1;
            a.ics = n[2];
            a.ibs = n[1] * n[2];
            a.ors = (int64_t)I[0] * I[1];
            a.ocs = 1;
            a.obs = I[1];
            a.nrows_in = I[2];
            a.ncols = I[1];
            a.nbatch = I[0];
            a.out_r0 = M[2] + 1;
            a.out_nrows = I[2];
            if ((rc = run_pass(p, a, p->fd[2], p->tw[2], false, false, st))) return rc;
            // along y, in place: B[kz][x][y] -> B[kz][x][ky]
            PassArgs b = a;
            b.in = p->B;
            b.irs = b.ors = 1;
            b.ics = b.ocs = I[1];
            b.ibs = b.obs = (int64_t)I[0] * I[1];
            b.nrows_in = I[1];
            b.ncols = I[0];
            b.nbatch = I[2];
            b.out_r0 = M[1] + 1;
            b.out_nrows = I[1];
            b.W = 0;
            if ((rc = run_pass(p, b, p->fd[1], p->tw[1], false, false, st))) return rc;
            // along x, in place: B[kz][x][ky] -> B[kz][kx][ky]
            PassArgs c = b;
            c.irs = c.ors = I[1];
            c.ics = c.ocs = 1;
            c.nrows_in = I[0];
            c.ncols = I[1];
            c.nbatch = I[2];
            c.out_r0 = M[0] + 1;
            c.out_nrows = I[0];
            c.W = 0;
            if ((rc = run_pass(p, c, p->fd[0], p->tw[0], false, false, st))) return rc;
        } else {
            // along y: rho[x][y] -> B[x][ky]; then along x in place
            a.in = rho + n[1] + 1;
            a.out = p->B;
            a.irs = 1;
            a.ics = n[1];
            a.ors = 1;
            a.ocs = I[1];
            a.nrows_in = I[1];
            a.ncols = I[0];
            a.nbatch = 1;
            a.out_r0 = M[1] + 1;
            a.out_nrows = I[1];
            if ((rc = run_pass(p, a, p->fd[1], p->tw[1], false, false, st))) return rc;
            PassArgs b = a;
            b.in = p->B;
            b.irs = b.ors = I[1];
            b.ics = b.ocs = 1;
            b.nrows_in = I[0];
            b.ncols = I[1];
            b.out_r0 = M[0] + 1;
            b.out_nrows = I[0];
            b.W = 0;
            if ((rc = run_pass(p, b, p->fd[0], p->tw[0], false, false, st))) return rc;
        }
    }
    STAGE(IPS_STAGE_SCREEN);
    ScreenArgs s{};
    s.d = d;
    s.pref = p->geo.pref;
    for (int a = 0; a < 3; ++a) {
        s.M[a] = a < d ? M[a] : 1;
        s.h[a] = a < d ? p->h[a] : 1.0;
        s.piL[a] = a < d ? 3.141592653589793238462643383279502884 / ((double)M[a] * p->h[a]) : 0.0;
        s.tau[a] = p->tau[a];
        if (a < d) s.tab[a] = p->tab[a];
        s.S[a] = p->S[a];
        s.sig[a] = p->S[a];
    }
    s.Y = static_cast<const double *>(p->B);
    s.src = p->src;
    s.nsrc = p->nsrc;
    s.ntgt = p->ntgt;
    IPS_HIP(launch_screen(s, phi, st));
    // sigma on the faces: inverse sine transforms over the in-face axes (the
    // families' face arrays are carved one after the other, as the shell layers)
    if ((rc = shell_dst_all(p, p->S, 2, true, st))) return rc;
    if (!p->surf_fast) {
        IPS_HIP(launch_screen_g(s, phi, st));
        return IPS_OK;
    }
    return surface_sums(p, phi, st);
}

int execute(ips_plan p, const double *rho, double *phi, hipStream_t st)
{
    const int d = p->d;
    const int *I = p->I, *M = p->M, *N = p->N;
    const int64_t *n = p->n;
    const bool f32 = p->precision != IPS_FP64;                  // sine passes of phi
    const bool f32s = p->precision == IPS_MIXED_FP32_SLICES;    // slice transforms of rho
    int rc;
    if (d == 1) {
        STAGE(IPS_STAGE_FINAL);
        IPS_HIP(launch_1d(rho, phi, M[0], p->h[0], p->fd[0], p->tw[0], p->tab[0], p->screen ? 1 : 0, st));
        return IPS_OK;
    }
    if (p->screen) {
        if ((rc = screen_boundary(p, rho, phi, st))) return rc;
    } else if (d == 3) {
        const int64_t s1 = n[2], s0 = n[1] * n[2];
        const double *rin = rho + s0 + s1 + 1;
        const int64_t vxy = (int64_t)I[0] * I[1];
        {
            // (1) zero-padded cos/sin transform of rho along z -> A[slot_z][x][y]
            STAGE(IPS_STAGE_RHO_Z);
            PassArgs a{};
            a.in = rin;
            a.out = p->A;
            a.irs = 1;
            a.ics = s1;
            a.ibs = s0;
            a.ors = vxy;
            a.ocs = 1;
            a.obs = I[1];
            a.nrows_in = I[2];
            a.ncols = I[1];
            a.nbatch = I[0];
            a.in_mode = IN_ZPAD;
            a.out_r0 = 0;
            a.out_nrows = N[2];
            a.scale = 1.0;
            a.W = rho_pass_width(p, N[2], a.ncols, f32s);
            if ((rc = run_pass(p, a, p->fd[2], p->tw[2], false, f32s, st))) return rc;
        }
        {
            // (2) transform along y, sum over x-slices: faces x = 0, M0;
            //     the S_y S_z part is B[kz][x][ky]
            STAGE(IPS_STAGE_CONV_X);
            CcArgs a{};
            a.in = p->A;
            a.irs = 1;
            a.ics = I[1];
            a.ibs = vxy;
            a.nrows_in = I[1];
            a.ncols = I[0];
            a.nbatch = N[2];
            a.Mo = M[2];
            a.cols_per_chunk = p->chunk[0];
            a.K = p->K[0];
            a.Kd = (int64_t)(M[2] + 1) * (M[1] + 1);
            a.Ko = M[1] + 1;
            a.part = p->part[0];
            a.Bout = p->B;
            a.Bf32 = f32;
            a.Bcs = I[1];
            a.Brs = 1;
            a.Bbs = vxy;
            a.W = tile_width(N[1], p->work, a.ncols);
            a.fd = p->fd[1];
            a.tw = p->tw[1];
            a.twf = p->twf[1];
            IPS_HIP(launch_cc(a, p->nch[0], f32s, f32s, st));
        }
        {
            // (3) transform along x, sum over y-slices: faces y = 0, M1
            STAGE(IPS_STAGE_CONV_Y);
            CcArgs a{};
            a.in = p->A;
            a.irs = I[1];
            a.ics = 1;
            a.ibs = vxy;
            a.nrows_in = I[0];
            a.ncols = I[1];
            a.nbatch = N[2];
            a.Mo = M[2];
            a.cols_per_chunk = p->chunk[1];
            a.interleave = 1; // pencils along x: strided rows
            a.K = p->K[1];
            a.Kd = (int64_t)(M[2] + 1) * (M[0] + 1);
            a.Ko = M[0] + 1;
            a.part = p->part[1];
            a.Bout = nullptr;
            a.W = tile_width(N[0], p->work, a.ncols);
            a.fd = p->fd[0];
            a.tw = p->tw[0];
            a.twf = p->twf[0];
            IPS_HIP(launch_cc(a, p->nch[1], f32s, f32s, st));
        }
        {
            // (4) zero-padded transform of rho along y -> C[x][slot_y][z] (reuses A)
            STAGE(IPS_STAGE_RHO_Y);
            PassArgs a{};
            a.in = rin;
            a.out = p->A;
            a.irs = s1;
            a.ics = 1;
            a.ibs = s0;
            a.ors = I[2];
            a.ocs = 1;
            a.obs = (int64_t)N[1] * I[2];
            a.nrows_in = I[1];
            a.ncols = I[2];
            a.nbatch = I[0];
            a.in_mode = IN_ZPAD;
            a.out_r0 = 0;
            a.out_nrows = N[1];
            a.scale = 1.0;
            a.W = rho_pass_width(p, N[1], a.ncols, f32s);
            if ((rc = run_pass(p, a, p->fd[1], p->tw[1], false, f32s, st))) return rc;
        }
        {
            // (5) transform along x, sum over z-slices: faces z = 0, M2
            STAGE(IPS_STAGE_CONV_Z);
            CcArgs a{};
            a.in = p->A;
            a.irs = (int64_t)N[1] * I[2];
            a.ics = 1;
            a.ibs = I[2];
            a.nrows_in = I[0];
            a.ncols = I[2];
            a.nbatch = N[1];
            a.Mo = M[1];
            a.cols_per_chunk = p->chunk[2];
            a.interleave = 1;
            a.K = p->K[2];
            a.Kd = (int64_t)(M[1] + 1) * (M[0] + 1);
            a.Ko = M[0] + 1;
            a.part = p->part[2];
            a.Bout = nullptr;
            a.W = tile_width(N[0], p->work, a.ncols);
            a.fd = p->fd[0];
            a.tw = p->tw[0];
            a.twf = p->twf[0];
            IPS_HIP(launch_cc(a, p->nch[2], f32s, f32s, st));
        }
        STAGE(IPS_STAGE_FACES);
        // (6) face spectra: sum of the chunk partials, inverse transform along the
        //     contiguous slot axis c, then along r; F[fam][face][slot_r][slot_c]
        const int fr[3] = {2, 2, 1}, fc[3] = {1, 0, 0};
        PassArgs fa[3], fb[3];
        const int nf = p->cube ? 1 : 3;
        for (int fam = 0; fam < nf; ++fam) {
            const int nfam = p->cube ? 3 : 1;
            const int r = fr[fam], c = fc[fam];
            const int64_t plane = (int64_t)N[r] * N[c];
            PassArgs &a = fa[fam];
            a = PassArgs{};
            a.in = p->part[fam];
            a.out = p->F[fam];
            a.irs = a.ors = 1;
            a.ics = a.ocs = N[c];
            a.ibs = (int64_t)p->nch[fam] * plane;
            a.obs = plane;
            a.nsum = p->nch[fam];
            a.sstride = plane;
            a.nrows_in = N[c];
            a.ncols = N[r];
            a.nbatch = 2 * nfam;
            a.in_mode = IN_HERM;
            a.out_r0 = 0;
            a.out_nrows = M[c] + 1;
            a.scale = 1.0 / N[c];
            // few faces: narrow tiles give enough blocks to fill the device
            a.W = tile_width(N[c], std::min(p->work, 512), a.ncols);
            prep_pass(p, a, p->fd[c], p->tw[c]);
            PassArgs &b = fb[fam];
            b = PassArgs{};
            b.in = b.out = p->F[fam];
            b.irs = b.ors = N[c];
            b.ics = b.ocs = 1;
            b.ibs = b.obs = plane;
            b.nrows_in = N[r];
            b.ncols = M[c] + 1;
            b.nbatch = 2 * nfam;
            b.in_mode = IN_HERM;
            b.out_r0 = 0;
            b.out_nrows = M[r] + 1;
            b.scale = 1.0 / N[r];
            // the second step reads no partials: the default tile budget
            // (compile-time stages) measured faster than narrow tiles
            b.W = tile_width(N[r], std::min(p->work, 2048), b.ncols);
            prep_pass(p, b, p->fd[r], p->tw[r]);
        }
        // the families' passes of each step together (one launch each when uniform)
        if ((rc = run_passes(fa, nf, false, false, st))) return rc;
        if ((rc = run_passes(fb, nf, false, false, st))) return rc;
        // (8) boundary values into phi; F[fam][face][j_r][j_c] -> strides of the in-face
        //     axes in increasing order
        BwriteArgs a{};
        a.geo = p->geo;
        for (int q = 0; q < 3; ++q) a.n[q] = n[q];
        for (int fam = 0; fam < 3; ++fam) {
            a.F[fam] = p->F[fam];
            a.scale[fam] = p->h[0] * p->h[1] * p->h[2];
            const int r = fr[fam], c = fc[fam];
            a.fs[fam][0] = (int64_t)N[r] * N[c];
            // lower in-face axis first
            const int lo = std::min(r, c);
            a.fs[fam][1] = lo == c ? 1 : N[c];
            a.fs[fam][2] = lo == c ? N[c] : 1;
        }
        a.phi = phi;
        IPS_HIP(launch_bwrite(a, st));
    } else {
        // d == 2: faces are lines
        const int64_t s0 = n[1];
        const double *rin = rho + s0 + 1;
        for (int fam = 0; fam < 2; ++fam) {
            STAGE(fam == 0 ? IPS_STAGE_CONV_X : IPS_STAGE_CONV_Z);
            const int pen = 1 - fam;
            CcArgs a{};
            a.in = rin;
            a.irs = fam == 0 ? 1 : s0;
            a.ics = fam == 0 ? s0 : 1;
            a.ibs = 0;
            a.nrows_in = I[pen];
            a.ncols = I[fam];
            a.nbatch = 1;
            a.Mo = 0;
            a.cols_per_chunk = p->chunk[fam];
            a.interleave = fam == 1;
            a.K = p->K[fam];
            a.Kd = M[pen] + 1;
            a.Ko = 0;
            a.part = p->part[fam];
            if (fam == 0) {
                a.Bout = p->B;
                a.Bf32 = f32;
                a.Bcs = I[1];
                a.Brs = 1;
                a.Bbs = 0;
            }
            a.W = tile_width(N[pen], p->work, a.ncols);
            a.fd = p->fd[pen];
            a.tw = p->tw[pen];
            a.twf = p->twf[pen];
            IPS_HIP(launch_cc(a, p->nch[fam], f32s, false, st));
        }
        STAGE(IPS_STAGE_FACES);
        for (int fam = 0; fam < 2; ++fam) {
            if (p->cube && fam > 0) break;
            const int nfam = p->cube ? 2 : 1;
            const int pen = 1 - fam;
            // the chunk partials of every face summed in parallel (a face line has
            // few columns, so a summing load inside the pass would leave most of
            // the GPU idle), then the inverse transform in place
            IPS_HIP(launch_reduce(p->part[fam], p->F[fam], N[pen], p->nch[fam], 2 * nfam, st));
            PassArgs a{};
            a.in = p->F[fam];
            a.out = p->F[fam];
            a.irs = a.ors = 1;
            a.ics = N[pen];
            a.ocs = N[pen];
            a.ibs = a.obs = 0;
            a.nrows_in = N[pen];
            a.ncols = 2 * nfam;
            a.nbatch = 1;
            a.in_mode = IN_HERM;
            a.out_r0 = 0;
            a.out_nrows = M[pen] + 1;
            a.scale = 1.0 / N[pen];
            if ((rc = run_pass(p, a, p->fd[pen], p->tw[pen], false, false, st))) return rc;
        }
        BwriteArgs a{};
        a.geo = p->geo;
        for (int q = 0; q < 3; ++q) a.n[q] = q < 2 ? n[q] : 1;
        for (int fam = 0; fam < 2; ++fam) {
            a.F[fam] = p->F[fam];
            a.fs[fam][0] = N[1 - fam];
            a.fs[fam][1] = 1;
            a.fs[fam][2] = 0;
            a.scale[fam] = p->h[0] * p->h[1];
        }
        a.phi = phi;
        IPS_HIP(launch_bwrite(a, st));
    }

    // ---- harmonic part: shell spectra ------------------------------------------------
    {
        STAGE(IPS_STAGE_SHELL_GT);
        GtArgs a{};
        a.geo = p->geo;
        for (int q = 0; q < 3; ++q) a.n[q] = q < d ? n[q] : 1;
        a.phi = phi;
        for (int fam = 0; fam < d; ++fam) a.G[fam] = p->G[fam];
        IPS_HIP(launch_gtilde(a, st));
        if ((rc = shell_dst_all(p, p->G, 2, false, st))) return rc;
    }
    ShellSpec sh{};
    PackArgs pk{};
    pk.geo = p->geo;
    for (int fam = 0; fam < d; ++fam) {
        sh.G[fam] = p->G[fam];
        sh.D[fam] = p->D[fam];
        sh.P[fam] = p->P[fam];
        pk.G[fam] = p->G[fam];
        pk.D[fam] = p->D[fam];
        pk.P[fam] = p->P[fam];
    }
    sh.P1T = p->P1T;
    sh.P2T = p->P2T;
    pk.P1T = p->P1T;
    pk.P2T = p->P2T;
    pk.p2t_f32 = f32;
    pk.withD = 0;
    IPS_HIP(launch_pack(pk, st));
    if (p->order == 6) {
        STAGE(IPS_STAGE_SHELL_R6);
        {
            R6Args a{};
            a.geo = p->geo;
            for (int q = 0; q < d; ++q) {
                a.tab[q] = p->tab[q];
                a.P[q] = p->P[q];
                a.T[q] = f32 ? (void *)p->Tf[q] : (void *)p->T[q];
            }
            a.t_f32 = f32;
            a.P1T = p->P1T;
            a.part = p->r6part;
            int64_t off = 0;
            for (int q = 0; q < d; ++q) {
                a.part_off[q] = off;
                off += (int64_t)r6t_splits(p->geo) * 10 * shell_size_host(p->geo, q);
            }
            IPS_HIP(launch_r6t(a, st));
        }
        // mixed modes: the R_spec layers and their inverse transforms in FP32
        if ((rc = f32 ? shell_dst_all(p, p->Tf, 10, true, st) : shell_dst_all(p, p->T, 10, true, st))) return rc;
        DcorrArgs a{};
        a.geo = p->geo;
        for (int q = 0; q < 3; ++q) a.n[q] = q < d ? n[q] : 1;
        a.phi = phi;
        a.rs_f32 = f32;
        for (int fam = 0; fam < d; ++fam) {
            a.RS[fam] = f32 ? (const void *)p->Tf[fam] : (const void *)p->T[fam];
            a.C[fam] = p->C[fam];
            a.D[fam] = p->D[fam];
        }
        IPS_HIP(launch_dcorr(a, st));
        if ((rc = shell_dst_all(p, p->D, 4, false, st))) return rc;
        pk.withD = 1;
        IPS_HIP(launch_pack(pk, st));
    }
    // ---- combination and inverse transforms ------------------------------------------
    {
        FinalArgs a{};
        a.buf = p->B;
        if (d == 3) {
            // B[kz][x][ky]: rows x, columns ky, batch kz
            a.irs = I[1];
            a.ics = 1;
            a.ibs = (int64_t)I[0] * I[1];
            a.ncols = I[1];
            a.nbatch = I[2];
            a.cax = 1;
            a.bax = 2;
        } else {
            a.irs = I[1];
            a.ics = 1;
            a.ibs = 0;
            a.ncols = I[1];
            a.nbatch = 1;
            a.cax = 1;
            a.bax = -1;
        }
        a.nrows_in = I[0];
        a.W = tile_width(N[0], N[0] > kLdsMaxN ? p->work : final_work(p->precision), a.ncols);
        a.order = p->order;
        a.mixed = f32;
        a.geo = p->geo;
        for (int q = 0; q < d; ++q) a.tab[q] = p->tab[q];
        a.sh = sh;
        a.fd = p->fd[0];
        a.tw = p->tw[0];
        a.twf = p->twf[0];
        a.rowtab = p->rowtab;
        a.group = final_group(a.W, f32 ? 4 : 8);
        a.pre = p->screen ? 1 : 0; // B already holds the spectrum along axis 0
        IPS_HIP(launch_final_rows(a, st));
        STAGE(IPS_STAGE_FINAL);
        IPS_HIP(launch_final(a, st));
    }
    if (d == 3) {
        {
            STAGE(IPS_STAGE_INV_Y);
            // B[kz][x][ky] -> B[kz][x][y]
            PassArgs a{};
            a.in = a.out = p->B;
            a.irs = a.ors = 1;
            a.ics = a.ocs = I[1];
            a.ibs = a.obs = (int64_t)I[0] * I[1];
            a.nrows_in = I[1];
            a.ncols = I[0];
            a.nbatch = I[2];
            a.in_mode = IN_SPECS;
            a.out_r0 = 1;
            a.out_nrows = I[1];
            a.scale = 0.5;
            if ((rc = run_pass(p, a, p->fd[1], p->tw[1], f32, f32, st))) return rc;
        }
        STAGE(IPS_STAGE_INV_Z);
        // B[kz][x][y] -> phi[x][y][z]
        PassArgs b{};
        b.in = p->B;
        b.out = phi + n[1] * n[2] + n[2] + 1;
        b.irs = (int64_t)I[0] * I[1];
        b.ics = 1;
        b.ibs = I[1];
        b.ors = 1;
        b.ocs = n[2];
        b.obs = n[1] * n[2];
        b.nrows_in = I[2];
        b.ncols = I[1];
        b.nbatch = I[0];
        b.in_mode = IN_SPECS;
        b.out_r0 = 1;
        b.out_nrows = I[2];
        b.scale = 0.5;
        if ((rc = run_pass(p, b, p->fd[2], p->tw[2], f32, false, st))) return rc;
    } else {
        STAGE(IPS_STAGE_INV_Z);
        PassArgs b{};
        b.in = p->B;
        b.out = phi + n[1] + 1;
        b.irs = 1;
        b.ics = I[1];
        b.ibs = 0;
        b.ors = 1;
        b.ocs = n[1];
        b.obs = 0;
        b.nrows_in = I[1];
        b.ncols = I[0];
        b.nbatch = 1;
        b.in_mode = IN_SPECS;
        b.out_r0 = 1;
        b.out_nrows = I[1];
        b.scale = 0.5;
        if ((rc = run_pass(p, b, p->fd[1], p->tw[1], f32, false, st))) return rc;
    }
    return IPS_OK;
}

// ---- adjoint ---------------------------------------------------------------------------

// Adjoint buffers of a plan whose workspace does not hold them: one block,
// allocated by the first adjoint call.
int adj_alloc(ips_plan p)
{
    if (p->adj_ready || p->d == 1) {
        p->adj_ready = true;
        return IPS_OK;
    }
    if (p->ws_adj) return fail(IPS_E_WORKSPACE, "the plan has no workspace bound");
    Carver c;
    layout_adj(p, c);
    void *blk = nullptr;
    int rc = p->adjmem.alloc(&blk, c.off);
    if (rc) return rc;
    c.base = static_cast<char *>(blk);
    c.off = 0;
    layout_adj(p, c);
    p->adj_ready = true;
    return IPS_OK;
}

// Raw DST-I of an interior field over all axes.  src points at node (1, 1, 1)
// of an array with strides sst[] (a grid or a packed interior); X receives
// the packed coefficients [k0][k1][k2].
int vol_fwd(ips_plan p, const double *src, const int64_t *sst, double *X, hipStream_t st, bool f32t)
{
    const int *I = p->I, *M = p->M;
    PassArgs a{};
    a.in_mode = IN_ZPAD;
    a.scale = 1.0;
    if (p->d == 3) {
        a.in = src;
        a.out = X;
        a.irs = sst[2];
        a.ics = sst[1];
        a.ibs = sst[0];
        a.ors = 1;
        a.ocs = I[2];
        a.obs = (int64_t)I[1] * I[2];
        a.nrows_in = I[2];
        a.ncols = I[1];
        a.nbatch = I[0];
        a.out_r0 = M[2] + 1;
        a.out_nrows = I[2];
        int rc = run_pass(p, a, p->fd[2], p->tw[2], false, false, st, f32t);
        if (rc) return rc;
        PassArgs b = a;
        b.in = X;
        b.irs = b.ors = I[2];
        b.ics = b.ocs = 1;
        b.ibs = b.obs = (int64_t)I[1] * I[2];
        b.nrows_in = I[1];
        b.ncols = I[2];
        b.nbatch = I[0];
        b.out_r0 = M[1] + 1;
        b.out_nrows = I[1];
        b.W = 0;
        if ((rc = run_pass(p, b, p->fd[1], p->tw[1], false, false, st, f32t))) return rc;
        PassArgs c = b;
        c.irs = c.ors = (int64_t)I[1] * I[2];
        c.ics = c.ocs = 1;
        c.ibs = c.obs = I[2];
        c.nrows_in = I[0];
        c.ncols = I[2];
        c.nbatch = I[1];
        c.out_r0 = M[0] + 1;
        c.out_nrows = I[0];
        c.W = 0;
        return run_pass(p, c, p->fd[0], p->tw[0], false, false, st, f32t);
    }
    a.in = src;
    a.out = X;
    a.irs = sst[1];
    a.ics = sst[0];
    a.ors = 1;
    a.ocs = I[1];
    a.nrows_in = I[1];
    a.ncols = I[0];
    a.nbatch = 1;
    a.out_r0 = M[1] + 1;
    a.out_nrows = I[1];
    int rc = run_pass(p, a, p->fd[1], p->tw[1], false, false, st, f32t);
    if (rc) return rc;
    PassArgs b = a;
    b.in = X;
    b.irs = b.ors = I[1];
    b.ics = b.ocs = 1;
    b.nrows_in = I[0];
    b.ncols = I[1];
    b.out_r0 = M[0] + 1;
    b.out_nrows = I[0];
    b.W = 0;
    return run_pass(p, b, p->fd[0], p->tw[0], false, false, st, f32t);
}

// Inverse of vol_fwd's coefficients (raw DST-I again, scaled by 1/2 per axis
// as the synthesis returns twice the sine sum): X is overwritten, the result
// goes to dst (node (1, 1, 1), strides dst_st[]).
int vol_inv(ips_plan p, double *X, double *dst, const int64_t *dst_st, hipStream_t st, bool f32t)
{
    const int *I = p->I, *M = p->M;
    PassArgs a{};
    a.in_mode = IN_SPECS;
    a.scale = 0.5;
    a.out_r0 = 1;
    if (p->d == 3) {
        a.in = a.out = X;
        a.irs = a.ors = (int64_t)I[1] * I[2];
        a.ics = a.ocs = 1;
        a.ibs = a.obs = I[2];
        a.nrows_in = I[0];
        a.ncols = I[2];
        a.nbatch = I[1];
        a.out_nrows = I[0];
        int rc = run_pass(p, a, p->fd[0], p->tw[0], false, false, st, f32t);
        if (rc) return rc;
        PassArgs b = a;
        b.irs = b.ors = I[2];
        b.ics = b.ocs = 1;
        b.ibs = b.obs = (int64_t)I[1] * I[2];
        b.nrows_in = I[1];
        b.ncols = I[2];
        b.nbatch = I[0];
        b.out_nrows = I[1];
        b.W = 0;
        if ((rc = run_pass(p, b, p->fd[1], p->tw[1], false, false, st, f32t))) return rc;
        PassArgs c = b;
        c.out = dst;
        c.irs = 1;
        c.ics = I[2];
        c.ibs = (int64_t)I[1] * I[2];
        c.ors = dst_st[2];
        c.ocs = dst_st[1];
        c.obs = dst_st[0];
        c.nrows_in = I[2];
        c.ncols = I[1];
        c.nbatch = I[0];
        c.out_nrows = I[2];
        c.W = 0;
        (void)M;
        return run_pass(p, c, p->fd[2], p->tw[2], false, false, st, f32t);
    }
    a.in = a.out = X;
    a.irs = a.ors = I[1];
    a.ics = a.ocs = 1;
    a.nrows_in = I[0];
    a.ncols = I[1];
    a.nbatch = 1;
    a.out_nrows = I[0];
    int rc = run_pass(p, a, p->fd[0], p->tw[0], false, false, st, f32t);
    if (rc) return rc;
    PassArgs b = a;
    b.out = dst;
    b.irs = 1;
    b.ics = I[1];
    b.ors = dst_st[1];
    b.ocs = dst_st[0];
    b.nrows_in = I[1];
    b.ncols = I[0];
    b.out_nrows = I[1];
    b.W = 0;
    return run_pass(p, b, p->fd[1], p->tw[1], false, false, st, f32t);
}

int execute_adjoint(ips_plan p, const double *w, double *out, hipStream_t st)
{
    const int d = p->d;
    const int *I = p->I, *M = p->M, *N = p->N;
    if (d == 1) {
        IPS_HIP(launch_adj_1d(w, out, M[0], p->h[0], p->fd[0], p->tw[0], p->tab[0], st));
        return IPS_OK;
    }
    int64_t gst[3] = {1, 1, 1}, pst[3] = {1, 1, 1};
    for (int a = d - 2; a >= 0; --a) {
        gst[a] = gst[a + 1] * p->n[a + 1];
        pst[a] = pst[a + 1] * I[a + 1];
    }
    int64_t off = 0;
    for (int a = 0; a < d; ++a) off += gst[a];
    AdjArgs aa{};
    aa.geo = p->geo;
    for (int a = 0; a < 3; ++a) aa.n[a] = a < d ? p->n[a] : 1;
    for (int a = 0; a < d; ++a) aa.tab[a] = p->tab[a];
    for (int fam = 0; fam < d; ++fam) {
        int b, c;
        kaxes(d, fam, b, c);
        aa.fb[fam] = b;
        aa.fc[fam] = c;
        aa.LF[fam] = p->LF[fam];
        aa.lf_size[fam] = 2 * (int64_t)(M[b] + 1) * (d == 3 ? (M[c] + 1) : 1);
    }
    const bool six = p->order == 6;
    // the mixed modes run the volume transforms in FP32 tiles (FP64 in HBM)
    const bool f32t = p->precision != IPS_FP64;
    int rc;
    // phi_star part and a = L0^-1 w_I from one forward transform
    if ((rc = vol_fwd(p, w + off, gst, p->AX, st, f32t))) return rc;
    IPS_HIP(launch_adj_spec(aa, p->AX, p->AY, st));
    if ((rc = vol_inv(p, p->AY, out + off, gst, st, f32t))) return rc;
    if ((rc = vol_inv(p, p->AX, p->AX, pst, st, f32t))) return rc;
    if (six) {
        // AZ (the slice stack of the boundary expansion, used later) is scratch here
        IPS_HIP(launch_adj_r6(aa, p->AX, p->AF, p->AU, p->AZ, st));
        if ((rc = vol_fwd(p, p->AU + off, gst, p->AX2, st, f32t))) return rc;
        IPS_HIP(launch_adj_spec(aa, p->AX2, nullptr, st));
        if ((rc = vol_inv(p, p->AX2, p->AX2, pst, st, f32t))) return rc;
    }
    IPS_HIP(launch_zero_boundary(aa, out, st));
    IPS_HIP(launch_adj_lambda(aa, w, p->AX, six ? p->AX2 : nullptr, six ? p->AU : nullptr, st));
    double vh = 1.0;
    for (int a = 0; a < d; ++a) vh *= p->h[a];
    for (int fam = 0; fam < d; ++fam) {
        const int b = aa.fb[fam], c = aa.fc[fam];
        // slot spectra of the two faces
        if (d == 3) {
            PassArgs a{};
            a.in = p->LF[fam];
            a.out = p->LH[fam];
            a.irs = 1;
            a.ics = M[c] + 1;
            a.ibs = (int64_t)(M[b] + 1) * (M[c] + 1);
            a.ors = 1;
            a.ocs = N[c];
            a.obs = (int64_t)N[b] * N[c];
            a.nrows_in = M[c] + 1;
            a.ncols = M[b] + 1;
            a.nbatch = 2;
            a.in_mode = IN_ZPAD0;
            a.out_r0 = 0;
            a.out_nrows = N[c];
            a.scale = 1.0;
            if ((rc = run_pass(p, a, p->fd[c], p->tw[c], false, false, st))) return rc;
            PassArgs b2{};
            b2.in = b2.out = p->LH[fam];
            b2.irs = b2.ors = N[c];
            b2.ics = b2.ocs = 1;
            b2.ibs = b2.obs = (int64_t)N[b] * N[c];
            b2.nrows_in = M[b] + 1;
            b2.ncols = N[c];
            b2.nbatch = 2;
            b2.in_mode = IN_ZPAD0;
            b2.out_r0 = 0;
            b2.out_nrows = N[b];
            b2.scale = 1.0;
            if ((rc = run_pass(p, b2, p->fd[b], p->tw[b], false, false, st))) return rc;
            // slices: product with the kernel spectra, synthesis along c, then along b
            ExpandArgs e{};
            e.d = 3;
            e.LH0 = p->LH[fam];
            e.LH1 = p->LH[fam] + (int64_t)N[b] * N[c];
            e.K = p->K[fam];
            e.Kd = (int64_t)(M[b] + 1) * (M[c] + 1);
            e.Kb = M[c] + 1;
            e.Ms = M[fam];
            e.Mb = M[b];
            e.out = p->AZ;
            e.ors = 1;
            e.ocs = I[c];
            e.obs = (int64_t)N[b] * I[c];
            e.ncols = N[b];
            e.nbatch = I[fam];
            e.W = tile_width(N[c], p->work / 2, N[b]);
            e.scale = 1.0 / N[c];
            e.accum = 0;
            e.fd = p->fd[c];
            e.tw = p->tw[c];
            IPS_HIP(launch_expand(e, st));
            PassArgs z{};
            z.in = p->AZ;
            z.out = out + off;
            z.irs = I[c];
            z.ics = 1;
            z.ibs = (int64_t)N[b] * I[c];
            z.ors = gst[b];
            z.ocs = gst[c];
            z.obs = gst[fam];
            z.nrows_in = N[b];
            z.ncols = I[c];
            z.nbatch = I[fam];
            z.in_mode = IN_HERM;
            z.out_r0 = 1;
            z.out_nrows = I[b];
            z.scale = vh / N[b];
            z.accum = 1;
            if ((rc = run_pass(p, z, p->fd[b], p->tw[b], false, false, st))) return rc;
        } else {
            PassArgs a{};
            a.in = p->LF[fam];
            a.out = p->LH[fam];
            a.irs = 1;
            a.ics = M[b] + 1;
            a.ors = 1;
            a.ocs = N[b];
            a.nrows_in = M[b] + 1;
            a.ncols = 2;
            a.nbatch = 1;
            a.in_mode = IN_ZPAD0;
            a.out_r0 = 0;
            a.out_nrows = N[b];
            a.scale = 1.0;
            if ((rc = run_pass(p, a, p->fd[b], p->tw[b], false, false, st))) return rc;
            ExpandArgs e{};
            e.d = 2;
            e.LH0 = p->LH[fam];
            e.LH1 = p->LH[fam] + N[b];
            e.K = p->K[fam];
            e.Kd = M[b] + 1;
            e.Kb = 0;
            e.Ms = M[fam];
            e.Mb = 0;
            e.out = out + off;
            e.ors = gst[b];
            e.ocs = gst[fam];
            e.obs = 0;
            e.ncols = I[fam];
            e.nbatch = 1;
            e.W = tile_width(N[b], p->work, I[fam]);
            e.scale = vh / N[b];
            e.accum = 1;
            e.fd = p->fd[b];
            e.tw = p->tw[b];
            IPS_HIP(launch_expand(e, st));
        }
    }
    return IPS_OK;
}

int flush_timing(ips_plan p)
{
    for (auto &r : p->ev_rec) {
        hipEvent_t e0 = std::get<1>(r), e1 = std::get<2>(r);
        IPS_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        IPS_HIP(hipEventElapsedTime(&ms, e0, e1));
        p->stage_ms[std::get<0>(r)] += ms;
        p->stage_calls[std::get<0>(r)] += 1;
    }
    p->ev_rec.clear();
    p->ev_used = 0;
    return IPS_OK;
}

void plan_free(ips_plan p)
{
    if (!p) return;
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != p->device) (void)hipSetDevice(p->device);
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    p->mem.release();
    p->wsmem.release();
    p->adjmem.release();
    if (cur != p->device) (void)hipSetDevice(cur);
    delete p;
}

// Plan cache of ips_solve / ips_solve_ex: least recently used plans beyond
// the capacity (IPS_SOLVE_CACHE plans, default 4) are destroyed, except those
// another thread is using.
using CacheKey = std::tuple<int, int, int64_t, int64_t, int64_t, double, double, double, int, int>;
struct CacheEnt {
    ips_plan p = nullptr;
    uint64_t last = 0; // use tick
    int users = 0;     // threads inside a solve with this plan
};
std::mutex g_cache_mu;
std::map<CacheKey, CacheEnt> g_cache;
uint64_t g_cache_tick = 0;

size_t cache_capacity()
{
    static const size_t cap = [] {
        const char *e = getenv("IPS_SOLVE_CACHE");
        const long v = e ? atol(e) : 4;
        return (size_t)(v < 1 ? 1 : v);
    }();
    return cap;
}

// Destroy idle entries, least recently used first, until at most `keep`
// remain (entries in use are skipped).  Call with g_cache_mu held.
void cache_trim(size_t keep)
{
    while (g_cache.size() > keep) {
        auto victim = g_cache.end();
        for (auto it = g_cache.begin(); it != g_cache.end(); ++it)
            if (it->second.users == 0 && (victim == g_cache.end() || it->second.last < victim->second.last))
                victim = it;
        if (victim == g_cache.end()) return;
        plan_free(victim->second.p);
        g_cache.erase(victim);
    }
}

} // namespace

// Plan with a given tile budget (arguments already validated).
int plan_create_work(ips_plan *out, int d, const int64_t *n, const double *h, int order,
                     int precision, unsigned flags, int work)
{
    g_alloc_seq = 0;
    ips_plan p = new (std::nothrow) ips_plan_s();
    if (!p) return fail(IPS_E_NO_MEMORY, "host allocation failed");
    p->d = d;
    p->order = d == 1 ? 4 : order;
    p->precision = precision;
    p->work = work;
    p->timing = (flags & IPS_FLAG_STAGE_TIMING) != 0;
    p->screen = (flags & IPS_FLAG_SCREENING) != 0;
    for (int a = 0; a < d; ++a) {
        p->n[a] = n[a];
        p->h[a] = h[a];
        p->M[a] = (int)(n[a] - 1);
        p->I[a] = p->M[a] - 1;
        p->N[a] = 2 * p->M[a];
    }
    if (p->screen && d == 3 && !(flags & IPS_FLAG_SCREEN_DIRECT)) p->surf_fast = perp_fits(p->M);
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return fail(IPS_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    int rc = plan_build(p, nullptr);
    if (rc == IPS_OK) {
        // execution workspace: measured, then owned by the plan unless the
        // caller brings it (IPS_FLAG_NO_WORKSPACE, ips_plan_set_workspace)
        p->ws_adj = (flags & IPS_FLAG_ADJOINT) != 0 && d > 1;
        p->ws_bytes = measure_ws(p);
        if (d == 1) {
            p->adj_ready = true;
        } else if (!(flags & IPS_FLAG_NO_WORKSPACE)) {
            void *blk = nullptr;
            rc = p->wsmem.alloc(&blk, p->ws_bytes);
            if (rc == IPS_OK) bind_ws(p, blk);
        }
    }
    if (rc == IPS_OK) {
        e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) rc = fail(IPS_E_DEVICE, std::string("plan build: ") + hipGetErrorString(e));
    }
    if (rc) {
        plan_free(p);
        return rc;
    }
    *out = p;
    return IPS_OK;
}

// Autotuner of the tile budget: every admissible budget is timed on a full
// solve of this geometry (two warm-up solves, then the best of three timed
// ones, HIP events on a private stream); the fastest wins.  Results are
// cached per (device, geometry, order, precision) for the life of the process.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int64_t, int64_t, int64_t, double, double, double, int, int>, int> g_tune;

int autotune_work(int d, const int64_t *n, const double *h, int order, int precision, int *best)
{
    int dev = 0;
    IPS_HIP(hipGetDevice(&dev));
    const auto key = std::make_tuple(dev, d, n[0], d > 1 ? n[1] : 0, d > 2 ? n[2] : 0, h[0],
                                     d > 1 ? h[1] : 0.0, d > 2 ? h[2] : 0.0, order, precision);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            *best = it->second;
            return IPS_OK;
        }
    }
    size_t cnt = 1;
    for (int a = 0; a < d; ++a) cnt *= (size_t)n[a];
    DevBuf mem;
    double *rho = nullptr, *phi = nullptr;
    int rc = mem.alloc((void **)&rho, cnt * sizeof(double));
    if (!rc) rc = mem.alloc((void **)&phi, cnt * sizeof(double));
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
        rc = fail(IPS_E_DEVICE, "autotune: hipStreamCreate failed");
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = fail(IPS_E_DEVICE, "autotune: hipEventCreate failed");
    if (!rc && launch_fill(rho, (int64_t)cnt, 1.0, st) != hipSuccess)
        rc = fail(IPS_E_DEVICE, "autotune: fill failed");
    int pick = tile_work_default();
    float pick_ms = 1e30f;
    const int cand[3] = {1024, 2048, 4096};
    for (int ci = 0; ci < 3 && !rc; ++ci) {
        if (final_pass_lds(d, n, precision, cand[ci]) > 160 * 1024) continue;
        ips_plan p = nullptr;
        rc = plan_create_work(&p, d, n, h, order, precision, 0, cand[ci]);
        if (rc) break;
        float tbest = 1e30f;
        for (int it = 0; it < 5 && !rc; ++it) {
            if (hipEventRecord(e0, st) != hipSuccess) rc = fail(IPS_E_DEVICE, "autotune: event");
            if (!rc) rc = execute(p, rho, phi, st);
            if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = fail(IPS_E_DEVICE, "autotune: event");
            if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = fail(IPS_E_DEVICE, "autotune: sync");
            float ms = 0.f;
            if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(IPS_E_DEVICE, "autotune: time");
            if (!rc && it >= 2) tbest = std::min(tbest, ms);
        }
        plan_free(p);
        if (!rc && tbest < pick_ms) {
            pick_ms = tbest;
            pick = cand[ci];
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    mem.release();
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = pick;
    }
    *best = pick;
    return IPS_OK;
}

// panel counts whose prime factors are 2, 3 and 5 (the fast FFT radices)
bool smooth235(int64_t m)
{
    if (m < 1) return false;
    for (int64_t q : {2, 3, 5})
        while (m % q == 0) m /= q;
    return m == 1;
}

// Extended plan: embed the caller's array in the zero extended array, solve
// (or apply the adjoint) there, restrict the result to the caller's nodes.
int execute_extended(ips_plan p, const double *in, double *out, hipStream_t st, bool adjoint)
{
    ips_plan q = p->inner;
    IPS_HIP(launch_embed(in, p->ext_in, p->d, p->n, q->n, p->ext_off, false, st));
    int rc;
    if (adjoint) {
        if ((rc = adj_alloc(q))) return rc;
        STAGE(IPS_STAGE_ADJOINT);
        rc = execute_adjoint(q, p->ext_in, p->ext_out, st);
    } else {
        rc = execute(q, p->ext_in, p->ext_out, st);
    }
    if (rc) return rc;
    IPS_HIP(launch_embed(p->ext_out, out, p->d, p->n, q->n, p->ext_off, true, st));
    return IPS_OK;
}

// Library-held scratch for ips_execute_static: one fixed device array per
// GPU (every device that loads the library holds it until the process ends).
// Host code never uses the array's name as an address: the device address
// of each GPU's copy comes from hipGetSymbolAddress with that GPU current.
constexpr size_t kStaticScratchBytes = (size_t)IPS_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's scratch array (looked up once per device).
int static_scratch(int dev, void **ptr)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(IPS_E_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *q = nullptr;
        hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !q) {
            (void)hipGetLastError();
            return fail(IPS_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = q;
    }
    *ptr = g_scratch_ptr[dev];
    return IPS_OK;
}

// A solve on a plain or an extended plan.
int execute_any(ips_plan p, const double *rho, double *phi, hipStream_t st)
{
    return p->inner ? execute_extended(p, rho, phi, st, false) : execute(p, rho, phi, st);
}

extern "C" {

const char *ips_status_string(int status)
{
    switch (status) {
    case IPS_OK: return "ok";
    case IPS_E_INVALID_ARG: return "invalid argument";
    case IPS_E_UNSUPPORTED: return "unsupported request";
    case IPS_E_NO_MEMORY: return "out of memory";
    case IPS_E_DEVICE: return "HIP runtime error";
    case IPS_E_WORKSPACE: return "workspace too small";
    default: return "unknown status";
    }
}

int ips_last_error_detail(char *buf, size_t len)
{
    if (!buf) return IPS_E_INVALID_ARG;
    if (len == 0) return IPS_OK;
    std::snprintf(buf, len, "%s", g_err.c_str());
    return IPS_OK;
}

int ips_plan_create(ips_plan *out, int d, const int64_t *n, const double *h, int order,
                    int precision, unsigned flags)
{
    if (!out) return fail(IPS_E_INVALID_ARG, "out must not be NULL");
    *out = nullptr;
    int rc = validate(d, n, h, order, precision, flags);
    if (rc) return rc;
    int work = tile_work_default();
    if ((flags & IPS_FLAG_AUTOTUNE) && d >= 2) {
        rc = autotune_work(d, n, h, order, precision, &work);
        if (rc) return rc;
    }
    return plan_create_work(out, d, n, h, order, precision, flags, work);
}

int ips_plan_workspace_size(ips_plan p, size_t *bytes)
{
    if (!p || !bytes) return fail(IPS_E_INVALID_ARG, "NULL argument");
    *bytes = p->inner ? p->inner->ws_bytes : p->ws_bytes;
    return IPS_OK;
}

int ips_plan_table_size(ips_plan p, size_t *bytes)
{
    if (!p || !bytes) return fail(IPS_E_INVALID_ARG, "NULL argument");
    *bytes = p->mem.bytes + p->adjmem.bytes + (p->inner ? p->inner->mem.bytes + p->inner->adjmem.bytes : 0);
    return IPS_OK;
}

int ips_plan_set_workspace(ips_plan p, void *dev_ptr, size_t bytes)
{
    if (!p) return fail(IPS_E_INVALID_ARG, "plan must not be NULL");
    if (p->inner) return ips_plan_set_workspace(p->inner, dev_ptr, bytes);
    if (p->d == 1) return IPS_OK; // the 1D solve needs no workspace
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || cur != p->device)
        return fail(IPS_E_INVALID_ARG, "plan belongs to another device than the current one");
    if (!dev_ptr) {
        if (bytes != 0) return fail(IPS_E_INVALID_ARG, "a NULL workspace must come with 0 bytes");
        // back to a plan-owned block
        if (p->wsmem.ptrs.empty()) {
            void *blk = nullptr;
            int rc = p->wsmem.alloc(&blk, p->ws_bytes);
            if (rc) return rc;
        }
        bind_ws(p, p->wsmem.ptrs[0]);
        return IPS_OK;
    }
    if (reinterpret_cast<uintptr_t>(dev_ptr) % 256 != 0)
        return fail(IPS_E_INVALID_ARG, "the workspace must be 256-byte aligned");
    if (bytes < p->ws_bytes)
        return fail(IPS_E_WORKSPACE, "workspace of " + std::to_string(bytes) + " bytes, the plan needs " +
                                         std::to_string(p->ws_bytes));
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, dev_ptr) != hipSuccess || attr.type == hipMemoryTypeHost ||
        attr.device != p->device) {
        (void)hipGetLastError();
        return fail(IPS_E_INVALID_ARG, "the workspace must be device memory of the plan's device");
    }
    // the plan's own block is released: the previous solves on it must have
    // completed (hipFree waits for the device)
    p->wsmem.release();
    bind_ws(p, dev_ptr);
    return IPS_OK;
}

int ips_extension(int d, const int64_t *n, const int64_t *margin, int64_t *n_ext, int64_t *offset)
{
    if (!n || !margin || !n_ext || !offset) return fail(IPS_E_INVALID_ARG, "NULL argument");
    if (d < 1 || d > 3) return fail(IPS_E_INVALID_ARG, "d must be 1, 2 or 3");
    for (int a = 0; a < d; ++a)
        if (n[a] < 3 || margin[a] < 0 || margin[a] > (int64_t)1 << 24 || n[a] > (int64_t)1 << 24)
            return fail(IPS_E_INVALID_ARG, "n[a] must be >= 3 and margin[a] >= 0");
    for (int a = 0; a < d; ++a) {
        const int64_t need = n[a] + 2 * margin[a];
        int64_t ne = need;
        while (!smooth235(ne - 1)) ++ne;
        n_ext[a] = ne;
        offset[a] = margin[a] + (ne - need) / 2;
    }
    return IPS_OK;
}

int ips_plan_create_extended(ips_plan *out, int d, const int64_t *n, const double *h, int order,
                             int precision, unsigned flags, const int64_t *margin)
{
    if (!out) return fail(IPS_E_INVALID_ARG, "out must not be NULL");
    *out = nullptr;
    int64_t ne[3] = {1, 1, 1}, off[3] = {0, 0, 0};
    int rc = ips_extension(d, n, margin, ne, off);
    if (rc) return rc;
    // the caller's grid: h and the flags are checked with it, the order
    // constraint applies to the extended grid
    if (!h) return fail(IPS_E_INVALID_ARG, "h must not be NULL");
    ips_plan inner = nullptr;
    rc = ips_plan_create(&inner, d, ne, h, order, precision, flags);
    if (rc) return rc;
    ips_plan p = new (std::nothrow) ips_plan_s();
    if (!p) {
        ips_plan_destroy(inner);
        return fail(IPS_E_NO_MEMORY, "host allocation failed");
    }
    p->d = d;
    p->order = order;
    p->precision = precision;
    p->device = inner->device;
    p->inner = inner;
    size_t cnt = 1;
    for (int a = 0; a < d; ++a) {
        p->n[a] = n[a];
        p->h[a] = h[a];
        p->ext_off[a] = off[a];
        cnt *= (size_t)ne[a];
    }
    if ((rc = p->mem.alloc((void **)&p->ext_in, cnt * sizeof(double))) ||
        (rc = p->mem.alloc((void **)&p->ext_out, cnt * sizeof(double)))) {
        ips_plan_destroy(p); // also destroys the inner plan
        return rc;
    }
    if (hipMemset(p->ext_in, 0, cnt * sizeof(double)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        ips_plan_destroy(p);
        return fail(IPS_E_DEVICE, "clearing the extended input failed");
    }
    *out = p;
    return IPS_OK;
}

int ips_execute(ips_plan p, const double *rho, double *phi, void *stream)
{
    if (!p) return fail(IPS_E_INVALID_ARG, "plan must not be NULL");
    if (!rho || !phi) return fail(IPS_E_INVALID_ARG, "rho and phi must not be NULL");
    size_t cnt = 1;
    for (int a = 0; a < p->d; ++a) cnt *= (size_t)p->n[a];
    const char *r0 = reinterpret_cast<const char *>(rho), *p0 = reinterpret_cast<const char *>(phi);
    if (r0 < p0 + cnt * sizeof(double) && p0 < r0 + cnt * sizeof(double))
        return fail(IPS_E_INVALID_ARG, "rho and phi must not overlap");
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || cur != p->device)
        return fail(IPS_E_INVALID_ARG, "plan belongs to another device than the current one");
    if (p->inner) {
        if (!p->inner->ws && p->d > 1) return fail(IPS_E_WORKSPACE, "the plan has no workspace bound");
        return execute_extended(p, rho, phi, static_cast<hipStream_t>(stream), false);
    }
    if (!p->ws && p->d > 1) return fail(IPS_E_WORKSPACE, "the plan has no workspace bound");
    return execute(p, rho, phi, static_cast<hipStream_t>(stream));
}

int ips_execute_static(ips_plan p, const double *rho, double *phi, void *stream)
{
    if (!p) return fail(IPS_E_INVALID_ARG, "plan must not be NULL");
    if (!rho || !phi) return fail(IPS_E_INVALID_ARG, "rho and phi must not be NULL");
    size_t cnt = 1;
    for (int a = 0; a < p->d; ++a) cnt *= (size_t)p->n[a];
    const char *r0 = reinterpret_cast<const char *>(rho), *p0 = reinterpret_cast<const char *>(phi);
    if (r0 < p0 + cnt * sizeof(double) && p0 < r0 + cnt * sizeof(double))
        return fail(IPS_E_INVALID_ARG, "rho and phi must not overlap");
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || cur != p->device)
        return fail(IPS_E_INVALID_ARG, "plan belongs to another device than the current one");
    ips_plan q = p->inner ? p->inner : p; // the plan whose workspace the solve uses
    if (q->ws_bytes > kStaticScratchBytes)
        return fail(IPS_E_WORKSPACE, "the plan needs " + std::to_string(q->ws_bytes) +
                                         " bytes of workspace, the static scratch holds " +
                                         std::to_string(kStaticScratchBytes));
    void *sp = nullptr;
    int rc = static_scratch(cur, &sp);
    if (rc) return rc;
    // run on the scratch, then give the plan its own binding back (kernel
    // arguments are fixed when a launch is enqueued)
    void *saved = q->ws;
    const bool saved_adj = q->adj_ready;
    if (q->d > 1) bind_ws(q, sp);
    if (p->inner)
        rc = execute_extended(p, rho, phi, static_cast<hipStream_t>(stream), false);
    else
        rc = execute(p, rho, phi, static_cast<hipStream_t>(stream));
    if (q->d > 1) {
        bind_ws(q, saved);
        q->adj_ready = saved_adj;
    }
    return rc;
}

int ips_execute_adjoint(ips_plan p, const double *phi_bar, double *rho_bar, void *stream)
{
    if (!p) return fail(IPS_E_INVALID_ARG, "plan must not be NULL");
    if (!phi_bar || !rho_bar) return fail(IPS_E_INVALID_ARG, "phi_bar and rho_bar must not be NULL");
    size_t cnt = 1;
    for (int a = 0; a < p->d; ++a) cnt *= (size_t)p->n[a];
    const char *r0 = reinterpret_cast<const char *>(phi_bar), *p0 = reinterpret_cast<const char *>(rho_bar);
    if (r0 < p0 + cnt * sizeof(double) && p0 < r0 + cnt * sizeof(double))
        return fail(IPS_E_INVALID_ARG, "phi_bar and rho_bar must not overlap");
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || cur != p->device)
        return fail(IPS_E_INVALID_ARG, "plan belongs to another device than the current one");
    if ((p->inner ? p->inner : p)->screen)
        return fail(IPS_E_UNSUPPORTED, "the screening variant has no adjoint");
    if (p->inner) return execute_extended(p, phi_bar, rho_bar, static_cast<hipStream_t>(stream), true);
    int rc = adj_alloc(p);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    STAGE(IPS_STAGE_ADJOINT);
    return execute_adjoint(p, phi_bar, rho_bar, st);
}

const char *ips_stage_name(int stage)
{
    static const char *names[IPS_STAGE_COUNT] = {
        "rho_z", "conv_x", "conv_y", "rho_y", "conv_z", "faces",
        "shell_gt", "shell_r6", "final", "inv_y", "inv_z", "adjoint", "screen"};
    if (stage < 0 || stage >= IPS_STAGE_COUNT) return "unknown";
    return names[stage];
}

int ips_plan_stage_time(ips_plan p, int stage, double *ms_total, int64_t *calls)
{
    if (!p || !ms_total || !calls) return fail(IPS_E_INVALID_ARG, "NULL argument");
    if (stage < 0 || stage >= IPS_STAGE_COUNT) return fail(IPS_E_INVALID_ARG, "bad stage");
    if (p->inner) return ips_plan_stage_time(p->inner, stage, ms_total, calls);
    int rc = flush_timing(p);
    if (rc) return rc;
    *ms_total = p->stage_ms[stage];
    *calls = p->stage_calls[stage];
    return IPS_OK;
}

int ips_plan_reset_stage_times(ips_plan p)
{
    if (!p) return fail(IPS_E_INVALID_ARG, "NULL argument");
    if (p->inner) return ips_plan_reset_stage_times(p->inner);
    int rc = flush_timing(p);
    if (rc) return rc;
    for (int i = 0; i < IPS_STAGE_COUNT; ++i) {
        p->stage_ms[i] = 0.0;
        p->stage_calls[i] = 0;
    }
    return IPS_OK;
}

int ips_plan_destroy(ips_plan p)
{
    if (!p) return IPS_OK;
    if (p->inner) {
        ips_plan_destroy(p->inner);
        p->inner = nullptr;
    }
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        for (auto it = g_cache.begin(); it != g_cache.end(); ++it)
            if (it->second.p == p) {
                g_cache.erase(it);
                break;
            }
    }
    plan_free(p);
    return IPS_OK;
}

int ips_solve_ex(int d, const int64_t *n, const double *h, const double *rho, int order, int precision,
                 double *phi)
{
    int rc = validate(d, n, h, order, precision, 0);
    if (rc) return rc;
    if (!rho || !phi) return fail(IPS_E_INVALID_ARG, "rho and phi must not be NULL");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(IPS_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    const CacheKey key = std::make_tuple(dev, d, n[0], d > 1 ? n[1] : 0, d > 2 ? n[2] : 0, h[0],
                                         d > 1 ? h[1] : 0.0, d > 2 ? h[2] : 0.0, d == 1 ? 4 : order, precision);
    ips_plan p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            p = it->second.p;
        } else {
            rc = ips_plan_create(&p, d, n, h, order, precision, 0);
            if (rc) return rc;
            it = g_cache.emplace(key, CacheEnt{p, 0, 0}).first;
        }
        it->second.users += 1;
        it->second.last = ++g_cache_tick;
        cache_trim(cache_capacity());
    }
    {
        // the enqueue of one solve must not interleave with another thread's
        // solve on the same plan (they share its workspace); the wait for the
        // device happens outside every lock
        std::lock_guard<std::mutex> plk(p->exec_mu);
        rc = ips_execute(p, rho, phi, nullptr);
    }
    if (rc == IPS_OK) {
        e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) rc = fail(IPS_E_DEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    }
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) it->second.users -= 1;
        cache_trim(cache_capacity());
    }
    return rc;
}

int ips_solve(int d, const int64_t *n, const double *h, const double *rho, int order, double *phi)
{
    return ips_solve_ex(d, n, h, rho, order, IPS_FP64, phi);
}

int ips_solve_release_cache(void)
{
    std::lock_guard<std::mutex> lk(g_cache_mu);
    cache_trim(0);
    return IPS_OK;
}

int ips_live_device_bytes(size_t *bytes)
{
    if (!bytes) return fail(IPS_E_INVALID_ARG, "NULL argument");
    const int64_t v = g_live_bytes.load();
    *bytes = (size_t)(v < 0 ? 0 : v);
    return IPS_OK;
}

int ips_solve_cache_size(size_t *plans)
{
    if (!plans) return fail(IPS_E_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(g_cache_mu);
    *plans = g_cache.size();
    return IPS_OK;
}

} // extern "C"

struct ips_batch_s {
    std::vector<ips_plan> plans;
    std::vector<int> order; // execution order: largest problems first
    bool eager = false;
    int device = 0;
    // graph of the last capture and the buffers it was captured with
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    hipGraphExec_t exec = nullptr;
    std::vector<const double *> rho_key;
    std::vector<double *> phi_key;
};

namespace {

// Branches of a batch graph (IPS_BATCH_STREAMS = 1..32 overrides the default,
// for measurements).  The speedup of the graph over eager launches is the
// concurrency of its branches (one branch runs as fast as eager launches);
// with the 4 hardware queues a HIP process has by default, 8 branches
// measured 2-3 % faster than 4, and raising the queue count made it slower.
int batch_streams()
{
    static const int v = [] {
        const char *e = getenv("IPS_BATCH_STREAMS");
        const int x = e ? atoi(e) : 0;
        return x >= 1 && x <= 32 ? x : 8;
    }();
    return v;
}

void batch_release_graph(ips_batch b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    b->rho_key.clear();
    b->phi_key.clear();
}

// Capture every problem's solve into one graph: the problems are spread over
// batch_streams() branches (fork from one stream, join back), so independent
// solves may run side by side on the device.
int batch_capture(ips_batch b, const double *const *rho, double *const *phi)
{
    const int nst = batch_streams();
    if (b->streams.empty()) {
        for (int k = 0; k < nst; ++k) {
            hipStream_t s = nullptr;
            IPS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            b->streams.push_back(s);
        }
        for (int k = 0; k < nst; ++k) {
            hipEvent_t e = nullptr;
            IPS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            b->events.push_back(e);
        }
    }
    hipStream_t s0 = b->streams[0];
    IPS_HIP(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal));
    int rc = IPS_OK;
    hipError_t e = hipEventRecord(b->events[0], s0);
    for (int k = 1; k < nst && e == hipSuccess; ++k) e = hipStreamWaitEvent(b->streams[k], b->events[0], 0);
    if (e != hipSuccess) rc = fail(IPS_E_DEVICE, std::string("batch capture fork: ") + hipGetErrorString(e));
    for (size_t j = 0; j < b->order.size() && !rc; ++j) {
        const int i = b->order[j];
        rc = execute_any(b->plans[i], rho[i], phi[i], b->streams[j % nst]);
    }
    for (int k = 1; k < nst && !rc; ++k) {
        e = hipEventRecord(b->events[k], b->streams[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s0, b->events[k], 0);
        if (e != hipSuccess) rc = fail(IPS_E_DEVICE, std::string("batch capture join: ") + hipGetErrorString(e));
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s0, &graph);
    if (!rc && e != hipSuccess) rc = fail(IPS_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    if (!rc) {
        e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            b->exec = nullptr;
            rc = fail(IPS_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (rc) {
        (void)hipGetLastError();
        return rc;
    }
    b->rho_key.assign(rho, rho + b->plans.size());
    b->phi_key.assign(phi, phi + b->plans.size());
    return IPS_OK;
}

} // namespace

extern "C" {

int ips_batch_create(ips_batch *out, int count, const int *d, const int64_t (*n)[3],
                     const double (*h)[3], int order, int precision, unsigned flags)
{
    if (!out) return fail(IPS_E_INVALID_ARG, "out must not be NULL");
    *out = nullptr;
    if (count <= 0 || !d || !n || !h) return fail(IPS_E_INVALID_ARG, "bad batch description");
    if ((flags & IPS_FLAG_BATCH_SMOOTH) && (flags & IPS_FLAG_SCREENING))
        return fail(IPS_E_UNSUPPORTED, "smooth batches take the volume sums only");
    ips_batch b = new (std::nothrow) ips_batch_s();
    if (!b) return fail(IPS_E_NO_MEMORY, "host allocation failed");
    b->eager = (flags & IPS_FLAG_BATCH_EAGER) != 0;
    (void)hipGetDevice(&b->device);
    // per-problem plans: no stage timing inside a batch
    const unsigned pflags =
        flags & ~(IPS_FLAG_STAGE_TIMING | IPS_FLAG_BATCH_EAGER | IPS_FLAG_NO_WORKSPACE | IPS_FLAG_BATCH_SMOOTH);
    const int64_t zero[3] = {0, 0, 0};
    std::vector<std::pair<int64_t, int>> sz;
    for (int i = 0; i < count; ++i) {
        ips_plan p = nullptr;
        int rc = (flags & IPS_FLAG_BATCH_SMOOTH)
                     ? ips_plan_create_extended(&p, d[i], n[i], h[i], order, precision, pflags, zero)
                     : ips_plan_create(&p, d[i], n[i], h[i], order, precision, pflags);
        if (rc) {
            for (ips_plan q : b->plans) ips_plan_destroy(q);
            delete b;
            return rc;
        }
        b->plans.push_back(p);
        int64_t c = 1;
        for (int a = 0; a < d[i]; ++a) c *= n[i][a];
        sz.emplace_back(-c, i);
    }
    std::stable_sort(sz.begin(), sz.end());
    for (auto &v : sz) b->order.push_back(v.second);
    *out = b;
    return IPS_OK;
}

int ips_batch_execute(ips_batch b, const double *const *rho, double *const *phi, void *stream)
{
    if (!b || !rho || !phi) return fail(IPS_E_INVALID_ARG, "NULL argument");
    const size_t cnt = b->plans.size();
    for (size_t i = 0; i < cnt; ++i) {
        if (!rho[i] || !phi[i]) return fail(IPS_E_INVALID_ARG, "NULL problem array");
        size_t m = 1;
        for (int a = 0; a < b->plans[i]->d; ++a) m *= (size_t)b->plans[i]->n[a];
        const char *r0 = reinterpret_cast<const char *>(rho[i]), *p0 = reinterpret_cast<const char *>(phi[i]);
        if (r0 < p0 + m * sizeof(double) && p0 < r0 + m * sizeof(double))
            return fail(IPS_E_INVALID_ARG, "rho and phi of a problem must not overlap");
    }
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || cur != b->device)
        return fail(IPS_E_INVALID_ARG, "batch belongs to another device than the current one");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (b->eager) {
        for (int i : b->order) {
            int rc = execute_any(b->plans[i], rho[i], phi[i], st);
            if (rc) return rc;
        }
        return IPS_OK;
    }
    const bool same = b->exec && std::equal(b->rho_key.begin(), b->rho_key.end(), rho) &&
                      std::equal(b->phi_key.begin(), b->phi_key.end(), phi);
    if (same) {
        IPS_HIP(hipGraphLaunch(b->exec, st));
        return IPS_OK;
    }
    // new buffers: solve directly on the caller's stream (which also sets every
    // kernel attribute outside any capture), then capture the graph that later
    // calls with these buffers replay
    batch_release_graph(b);
    for (int i : b->order) {
        int rc = execute_any(b->plans[i], rho[i], phi[i], st);
        if (rc) return rc;
    }
    return batch_capture(b, rho, phi);
}

int ips_batch_destroy(ips_batch b)
{
    if (!b) return IPS_OK;
    batch_release_graph(b);
    for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
    for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
    for (ips_plan p : b->plans) ips_plan_destroy(p);
    delete b;
    return IPS_OK;
}

} // extern "C"
