// Kernel argument blocks and launchers of the HIP solver (internal header).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_tile.h"

namespace ips {

// IN_ZPAD  : f_1..f_{M-1} at positions 1..M-1 of a zero-padded length-N sequence
// IN_ZPAD0 : f_0..f_M at positions 0..M (zeros at M+1..N-1)
// IN_EVEN  : f_0..f_M mirrored to length N
// IN_HERM  : slot rows C_0..C_M, S_1..S_{M-1} -> hermitian synthesis
// IN_SPECS : S rows only (C = 0) -> hermitian synthesis (inverse DST-I)
enum InMode { IN_ZPAD = 0, IN_EVEN = 1, IN_HERM = 2, IN_SPECS = 3, IN_ZPAD0 = 4 };

// Generic pencil pass: one transform along the tile rows, tile columns are a
// block of W consecutive columns, grid.y runs over a batch index.
struct PassArgs {
    const void *in;
    void *out;
    int64_t irs, ics, ibs; // input strides (elements) of row, column, batch
    int64_t ors, ocs, obs; // output strides
    int nrows_in;          // rows read (M-1 for IN_ZPAD/IN_SPECS, M+1 for IN_EVEN, N for IN_HERM)
    int ncols;             // columns in total
    int nbatch;
    int in_mode;
    int out_r0, out_nrows; // LDS rows [out_r0, out_r0 + out_nrows) are stored as rows 0..
    double scale;
    int W; // columns per block (even)
    FftDesc fd;
    const cx<double> *tw; // N twiddles exp(-2 pi i t / N)
    const cx<float> *twf; // the same in FP32 (transforms longer than 2048 in FP32)
    int nsum;             // IN_HERM: input element = sum of nsum copies (0/1: plain load)
    int64_t sstride;      // spacing of those copies
    int accum;            // add the result into the output instead of storing it
};

// Boundary convolution, contraction over the tile columns (faces normal to
// the column axis).  grid.x = chunks of columns, grid.y = batch entries.
struct CcArgs {
    const void *in;    // TI (double rho or T slot data)
    int64_t irs, ics, ibs;
    int nrows_in;      // M_p - 1
    int ncols;         // interior length of the contracted axis
    int nbatch;        // slots of the remaining in-face axis (1 if none)
    int Mo;            // M of that axis (slot -> wavenumber), 0 if none
    int cols_per_chunk; // first-half columns per chunk (a tile pairs column c with ncols-1-c)
    int interleave;     // chunk ch takes tiles ch, ch + nchunk, ... instead of a contiguous run
    const double *K;   // K[d][k_o][k_p], k_p contiguous (FP64 in every mode)
    int64_t Kd, Ko;
    double *part;      // FP64 chunk partials [2][nchunk][nbatch][2 M_p]
    void *Bout;        // optional S_p output: Bout[col*Bcs + (k_p-1)*Brs + (k_o-1)*Bbs],
                       // written for the sine slots k_o of the batch axis (all batches if Mo == 0)
    int64_t Bcs, Brs, Bbs;
    int Bf32;          // Bout holds float (else the transform type)
    int W;
    FftDesc fd;
    const cx<double> *tw;
    const cx<float> *twf;
};

// Per-axis tables of a plan (device pointers, index k-1 for k = 1..M-1).
struct AxisTabs {
    const double *lam;  // -(4/h^2) sin^2(pi k / 2M)       eigenvalue of D2
    const double *q;    // (pi k / L)^2                    continuous eigenvalue
    const double *s;    // s[(j-1)*(M-1) + k-1] = sin(pi k j / M), j = 1..5
};

struct Geo {
    int d;
    int M[3];
    double h[3];
    double c2[3][3]; // (h_i^2 + h_j^2)/12
    double c4[3][3]; // h_i^4/240 + h_i^2 h_j^2/144  (coefficient of D2_i D2_i D2_j)
    double pref;     // prod 2/M_i
};

// Shell spectra: g~ layers (2 per axis) and the deferred-correction layers
// (4 per axis, layers 1, 2, M-2, M-1).  Index [layer][k_b-1][k_c-1] over the
// two other axes in increasing order (3D) or [layer][k_b-1] (2D).
struct ShellSpec {
    const double *G[3];
    const double *D[3];
    // Parity-packed form used by the spectral kernels, [par][t][k_other] with
    // par = k_a & 1 and sg = +1 (odd k_a) or -1 (even k_a):
    //   t = 0: G_lo + sg G_hi          (multiplies sin(pi k_a / M_a))
    //   t = 1: D_1 + sg D_{M-1}        (multiplies sin(pi k_a / M_a))
    //   t = 2: D_2 + sg D_{M-2}        (multiplies sin(2 pi k_a / M_a))
    const double *P[3];
    // 3D: family 1 packed values transposed to [par][t][k2][k0] (k0 contiguous),
    // for the final pass which walks k0 at fixed k2
    const double *P1T;
    // 3D: family 2 packed values transposed to [par][t][k1][k0] (k0 contiguous),
    // for the final pass, whose lanes walk k0; stored in the final pass's
    // transform type (FP32 in the mixed modes)
    const void *P2T;
};

struct PackArgs {
    Geo geo;
    const double *G[3];
    const double *D[3];
    double *P[3];
    double *P1T; // 3D only
    void *P2T;   // 3D only: FP32 if p2t_f32, else FP64
    int p2t_f32;
    int withD;   // also pack the deferred-correction layers
};

struct FinalArgs {
    void *buf;  // B: raw DST of rho along the last d-1 axes; overwritten in place
    int64_t irs, ics, ibs;
    int cax, bax; // problem axes of the tile columns and of the batch (-1: none)
    int nrows_in; // M_0 - 1
    int ncols, nbatch;
    int W;
    int order;
    int mixed;   // buf holds float instead of double
    Geo geo;
    AxisTabs tab[3];
    ShellSpec sh;
    FftDesc fd;
    const cx<double> *tw;
    const cx<float> *twf;
    int group;      // neighbouring column blocks taken together (their rows share 128-byte lines)
    int pre;        // buf already holds the raw sine spectrum along axis 0 (no forward transform)
    void *rowtab;   // row table [nbatch][M0 - 1][12] (transform type) in global memory, written by
                    // launch_final_rows before the pass; both launchers reject a null table
};

// Boundary values from the screening charge (screen.hip).
struct ScreenArgs {
    int d;
    int M[3];
    double h[3];
    double piL[3];       // pi / L_a
    double pref;         // prod 2/M_a
    double tau[3];       // singular correction of a target inside a face of axis a
    AxisTabs tab[3];
    const double *Y;     // raw sine spectrum of rho_I, final-pass layout
    double *S[3];        // face coefficients, then (after the inverse transforms) sigma: [2][I_b][I_c]
    const double *sig[3];
    double *src;         // [4][nsrc]: x, y, z, W sigma
    int64_t nsrc, ntgt;  // surface nodes with sigma, boundary nodes
};

// Fast evaluation of the 3D surface sums (screen.hip).  Faces (axis f, side s),
// in-face axes (b, c) in increasing order; pairs pr = (0,1), (0,2), (1,2) of
// face axes (a, b) with the third axis c.
struct SurfArgs {
    int M[3];
    double h[3];
    double tau[3];
    const double *sig[3]; // sigma on the face interiors [2][I_b][I_c]
    double *FA[3];        // face charges W sigma on all face nodes [2][M_b + 1][M_c + 1]
    double *XH[3];        // their slot spectra over both in-face axes [2][2 M_b][2 M_c]
    const double *KP[3];  // kernel spectra of the same face and the opposite face [2][M_b + 1][M_c + 1]
    double *PP[3];        // parallel-face sums at the face nodes [2][M_b + 1][M_c + 1]
    // per pair: slot spectra along c of the charges of faces a and b (slot
    // major), the partial transfers to the other family, and the sums back on
    // the face nodes
    const double *XA[3], *XB[3]; // [2 M_c][2][M_b + 1], [2 M_c][2][M_a + 1]
    double *PA[3];               // targets on a: [2 M_c][2 groups][2][M_b + 1]
    double *PB[3];               // targets on b: [2 M_c][2][2][M_a + 1]
    double *QA[3], *QB[3];       // [2][M_b + 1][M_c + 1], [2][M_a + 1][M_c + 1]
    const double *KT[3];         // kernel spectra along c: KT[k][i][j] = FFT_c G(i h_a, j h_b, .)
    int groups[3];               // row groups per wavenumber (perp_groups)
};

// G samples of the tables: same face / opposite face of axis f ([2][M_b + 1][M_c + 1])
hipError_t launch_par_sample(double *out, int f, const int *M, const double *h, hipStream_t st);
// perpendicular pair (a, b), third axis c: out[dc][i][j] (zero at the origin)
hipError_t launch_perp_sample(double *out, int a, int b, int c, const int *M, const double *h, hipStream_t st);
hipError_t launch_face_charge(const SurfArgs &s, hipStream_t st);
hipError_t launch_par_mul(const SurfArgs &s, hipStream_t st);
// the perpendicular-pair kernel takes these sizes (face sides up to 3 NT nodes)
bool perp_fits(const int *M);
// row groups per wavenumber of pair pr (a launch runs (M_c + 1) x groups blocks)
int perp_groups(const int *M, int pr);
hipError_t launch_perp(const SurfArgs &s, hipStream_t st);
hipError_t launch_surf_assemble(const SurfArgs &s, double *phi, hipStream_t st);

// face coefficients of sigma from Y
hipError_t launch_screen(const ScreenArgs &a, double *phi, hipStream_t st);
// surface nodes and g at every boundary node of phi
hipError_t launch_screen_g(const ScreenArgs &a, double *phi, hipStream_t st);

// Sixth-order right-hand side on the depth-5 shell layers (see k_r6t).
struct R6Args {
    Geo geo;
    AxisTabs tab[3];
    const double *P[3]; // packed shell spectra (ShellSpec::P)
    const double *P1T;  // 3D: family 1 transposed (ShellSpec::P1T)
    void *T[3];         // [10][other axes] per axis: layers 1..5, then M-1..M-5
    int t_f32;          // T holds FP32 (mixed modes), else FP64
    int nblk[3];        // filled by the launcher
    // more than one split of the k_a sums (r6t_splits > 1, shells with few
    // positions): FP64 partials [axis][split][10][positions], axis ax at part_off[ax]
    double *part;
    int64_t part_off[3];
};

// splits of the k_a sums of k_r6t (1: none); the partial buffer holds
// splits * 10 * (sum of the shell sizes) doubles
int r6t_splits(const Geo &g);

struct DcorrArgs {
    Geo geo;
    int64_t n[3];
    const double *phi;     // grid with boundary values already written
    const void *RS[3];     // R_spec on the depth-5 shell layers [10][..][..]
    int rs_f32;            // RS holds FP32, else FP64
    double *C[3];          // R on the core layers 2..5, M-5..M-2: [8][..][..]
    double *D[3];          // outputs [4][..][..]
};

struct GtArgs {
    Geo geo;
    int64_t n[3];
    const double *phi;
    double *G[3]; // [2][..][..]
};

struct BwriteArgs {
    Geo geo;
    int64_t n[3];
    const double *F[3];   // face values after the inverse transforms
    int64_t fs[3][3];     // strides (face, row, col) of F[a]
    double scale[3];
    double *phi;
};

// Adjoint (rho_bar = A^T phi_bar), FP64.
struct AdjArgs {
    Geo geo;
    int64_t n[3];
    AxisTabs tab[3];
    double *LF[3];       // boundary weights per face family [2][M_b + 1][M_c + 1]
    int64_t lf_size[3];  // entries of LF[fam]
    int fb[3], fc[3];    // in-face axes (b, c) of each family, c contiguous (3D)
};

// Face-to-slice expansion (first transform), see k_expand.
struct ExpandArgs {
    int d;
    const double *LH0, *LH1; // slot spectra of the two faces
    const double *K;         // kernel spectra K_hat[dd][kb][kc] (2D: [dd][k])
    int64_t Kd, Kb;
    int Ms; // M of the face-normal axis
    int Mb; // M of the column axis (3D)
    double *out;
    int64_t ors, ocs, obs;
    int ncols, nbatch, W;
    double scale;
    int accum;
    FftDesc fd;
    const cx<double> *tw;
};

hipError_t launch_adj_spec(const AdjArgs &a, double *X, double *Y, hipStream_t st);
// T: 3D scratch of one grid-shaped array (unused in 2D)
hipError_t launch_adj_r6(const AdjArgs &a, const double *A, double *F, double *U, double *T, hipStream_t st);
hipError_t launch_adj_lambda(const AdjArgs &a, const double *w, const double *y1, const double *y2,
                             const double *U, hipStream_t st);
hipError_t launch_zero_boundary(const AdjArgs &a, double *out, hipStream_t st);
hipError_t launch_expand(const ExpandArgs &a, hipStream_t st);
hipError_t launch_adj_1d(const double *w, double *out, int M, double h, const FftDesc &fd,
                         const cx<double> *tw, const AxisTabs &tab, hipStream_t st);

// Raise a kernel's dynamic LDS limit above 64 KiB (once per size, cached).
void set_lds(const void *fn, size_t bytes);

hipError_t launch_pass(const PassArgs &a, bool in_f32, bool out_f32, hipStream_t st);
// FP64 input and output, FP32 tiles (the adjoint's volume transforms in the mixed modes)
hipError_t launch_pass_f32t(const PassArgs &a, hipStream_t st);

// Up to kMultiPass independent passes (generic widths, transforms up to 2048)
// in one launch; first[] is filled by the launcher.
constexpr int kMultiPass = 3;
struct MultiPassArgs {
    PassArgs p[kMultiPass];
    int first[kMultiPass + 1];
    int n;
};
hipError_t launch_pass_multi(const PassArgs *p, int n, bool in_f32, bool out_f32, hipStream_t st);
// in_f32: input data in FP32 (else FP64); f32: transform type
hipError_t launch_cc(const CcArgs &a, int nchunk, bool f32, bool in_f32, hipStream_t st);
// out[s][i] = sum over the chunks c of part[s][c][i]  (nset sets of nchunk rows of len)
hipError_t launch_reduce(const double *part, double *out, int64_t len, int nchunk, int nset, hipStream_t st);
hipError_t launch_bwrite(const BwriteArgs &a, hipStream_t st);
hipError_t launch_gtilde(const GtArgs &a, hipStream_t st);
hipError_t launch_pack(const PackArgs &a, hipStream_t st);
hipError_t launch_r6t(R6Args a, hipStream_t st);
hipError_t launch_dcorr(const DcorrArgs &a, hipStream_t st);
// Caller's block n at offset off inside the extended grid ne: embed (extract =
// false: dst is extended) or restrict (extract = true: src is extended).
hipError_t launch_embed(const double *src, double *dst, int d, const int64_t *n, const int64_t *ne,
                        const int64_t *off, bool extract, hipStream_t st);
// Row table of the final pass: once per solve, before launch_final.
hipError_t launch_final_rows(const FinalArgs &a, hipStream_t st);
hipError_t launch_final(const FinalArgs &a, hipStream_t st);
// K[dd][ib][ic] (3D) or K[dd][ib] (2D) for faces normal to axis a; (b, c) are
// the in-face axes in storage order (c contiguous).
hipError_t launch_ksample(double *out, int d, int a, int b, int c, const int *M, const double *h,
                          hipStream_t st);
// screen: end values from the screening charge instead of the direct sums
hipError_t launch_1d(const double *rho, double *phi, int M, double h, const FftDesc &fd,
                     const cx<double> *tw, const AxisTabs &tab, int screen, hipStream_t st);
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t st);
hipError_t launch_to_f32(const double *src, float *dst, int64_t n, hipStream_t st);

} // namespace ips
