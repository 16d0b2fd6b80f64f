/*
 * ipoisson.h -- C ABI of the MI355X infinite-domain Poisson solver.
 *
 * The solver evaluates phi(x) = integral over R^d of G(|x - s|) rho(s) ds at
 * every node of a uniform rectangular grid (d = 1, 2, 3), i.e. the solution
 * of Delta phi = rho in free space restricted to the box, following
 * C. R. Anderson, "High order accurate solution of Poisson's equation in
 * infinite domains for smooth functions" (arXiv 2108.11871):
 *
 *   phi = phi_star + phi_H                                   (Section 2)
 *   phi_star : sine-transform solve with zero boundary values (Section 3)
 *   g        : boundary values of phi, trapezoidal sum of G against rho
 *              evaluated through slice-wise FFT convolutions  (Section 4)
 *   phi_H    : 4th- or 6th-order discrete harmonic function with boundary
 *              values g (compact operator, deferred correction,
 *              cubic extrapolation)                            (Section 5)
 *   d = 1    : phi_H is the linear function through the two end values.
 *
 * Grid and layout
 *   n[i] nodes along axis i (n[i] = M_i + 1 panels), spacing h[i]; node
 *   (i0, ..., i_{d-1}) lies at a + (i0 h0, ..., i_{d-1} h_{d-1}); the result
 *   does not depend on the origin a.  Arrays are row-major with axis d-1
 *   contiguous: node (i0, i1, i2) is element (i0 * n1 + i1) * n2 + i2.
 *   All array arguments are DEVICE pointers (hipMalloc'd memory or the data
 *   of a GPU tensor) of n0 * ... * n_{d-1} doubles.
 *
 * Input contract
 *   rho values on boundary nodes are ignored.  The method assumes the
 *   support of rho keeps a positive distance from the boundary (Section 2);
 *   this is not checked, and accuracy degrades when it is violated.
 *   On output, phi holds g on every boundary node (faces, edges, corners)
 *   and phi_star + phi_H on every interior node.
 *
 * Errors
 *   Every call returns an ips_status.  Nothing aborts, exits or throws
 *   across the ABI.  On error the content of output arrays is unspecified.
 *   ips_last_error_detail() returns a message for the calling thread.
 *
 * Ownership and threading
 *   The caller owns rho and phi; the library never frees them and keeps no
 *   reference to them after the work enqueued by a call has completed.
 *   A plan owns its device workspace and tables.  One plan must not execute
 *   concurrently on two streams; different plans may.
 */
#ifndef IPOISSON_H
#define IPOISSON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ips_plan_s *ips_plan;
typedef struct ips_batch_s *ips_batch;

typedef enum {
    IPS_OK = 0,
    IPS_E_INVALID_ARG = -1, /* bad dimension, size, spacing, order, pointer */
    IPS_E_UNSUPPORTED = -2, /* valid request outside what this build handles */
    IPS_E_NO_MEMORY = -3,   /* device or host allocation failed */
    IPS_E_DEVICE = -4,      /* a HIP runtime call failed */
    IPS_E_WORKSPACE = -5    /* caller-supplied workspace too small */
} ips_status;

/* Arithmetic used by the transforms.  Input and output stay FP64.  In every
 * mode the boundary sums of Section 4 are accumulated in FP64 against FP64
 * kernel spectra (per tile, per chunk of slices and over the chunks), and the
 * inverse transforms of the face sums, g~, the core stencils, the cubic
 * extrapolation and the differences D = R - R_spec of the sixth-order step,
 * and the spectral symbols are FP64.  The mixed modes store the sine-space
 * volume in FP32, run its transforms in FP32, combine the spectrum in FP32
 * from those FP64 parts, and keep the sixth-order sine-series values on the
 * shell layers in FP32. */
typedef enum {
    IPS_FP64 = 0,              /* everything in FP64 */
    IPS_MIXED_FP32 = 1,        /* sine-transform passes of phi_star + phi_H in FP32 */
    IPS_MIXED_FP32_SLICES = 2  /* as 1, and the slice transforms of rho that feed the
                                  boundary sums in FP32 (each FP32 slot value is widened
                                  exactly and multiplied and summed in FP64) */
} ips_precision;

/*
 * ips_solve -- one blocking FP64 solve on the null stream of the current
 * device (ips_solve_ex with IPS_FP64).
 *   d      : 1, 2 or 3
 *   n      : d node counts, n[i] >= 3; for order 6 and d >= 2, n[i] >= 8
 *            (the extrapolation reaches five nodes in from the boundary)
 *   h      : d mesh widths, finite and > 0
 *   rho    : device array, n0*...*n_{d-1} doubles (boundary values ignored)
 *   order  : 4 or 6 (accuracy order of the harmonic part, Section 5);
 *            ignored for d = 1
 *   phi    : device array of the same size, must not overlap rho
 * Plans are cached per (device, d, n, h, order, precision): the cache keeps
 * the most recently used plans (4, or the value of the environment variable
 * IPS_SOLVE_CACHE read at the first call) and destroys the least recently
 * used idle ones beyond that.  Threads share the cache; solves of different
 * plans run concurrently, solves of one plan are enqueued one at a time, and
 * no lock is held while a call waits for the device.
 */
int ips_solve(int d, const int64_t *n, const double *h, const double *rho, int order,
              double *phi);

/* ips_solve with an ips_precision (errors as ips_solve; IPS_E_INVALID_ARG for
 * an unknown precision, IPS_E_UNSUPPORTED for a mixed mode with d = 1). */
int ips_solve_ex(int d, const int64_t *n, const double *h, const double *rho, int order,
                 int precision, double *phi);

/* Destroy every idle plan of the ips_solve cache (plans in use by another
 * thread stay).  Waits for their work (hipFree). */
int ips_solve_release_cache(void);

/* Number of plans in the ips_solve cache. */
int ips_solve_cache_size(size_t *plans);

/* Device bytes currently allocated by the library: tables and workspaces of
 * every live plan, batch and cached plan (caller-supplied workspaces are not
 * counted).  For memory accounting and leak checks. */
int ips_live_device_bytes(size_t *bytes);

/*
 * ips_plan_create -- build a reusable plan on the current device: FFT
 * descriptors, eigenvalue and sine tables, the Fourier transforms of the
 * Green's-function kernels used by the boundary convolutions (Section 4),
 * and all device workspace.  Arguments as ips_solve, plus:
 *   precision : an ips_precision value
 *   flags     : bitwise OR of IPS_FLAG_STAGE_TIMING, IPS_FLAG_ADJOINT,
 *               IPS_FLAG_AUTOTUNE and IPS_FLAG_NO_WORKSPACE (or 0)
 * On success *out receives the plan; release it with ips_plan_destroy.
 */
int ips_plan_create(ips_plan *out, int d, const int64_t *n, const double *h, int order,
                    int precision, unsigned flags);

/*
 * Device memory of a plan comes in two parts:
 *   tables    : twiddles, eigenvalue and sine tables, kernel spectra; built by
 *               ips_plan_create, owned by the plan, read-only afterwards;
 *   workspace : everything one solve writes besides phi (sine-space volume,
 *               slice transforms, chunk partial sums, face values, shell
 *               layers) and, for a plan created with IPS_FLAG_ADJOINT, the
 *               adjoint's buffers.  0 bytes for d = 1.
 * ips_plan_workspace_size gives the workspace bytes ips_plan_set_workspace
 * needs; ips_plan_table_size the bytes of tables held by the plan (the
 * adjoint buffers allocated by a first adjoint call and an extended plan's
 * two extended arrays included).  For an extended plan both refer to its
 * extended grid.
 */
int ips_plan_workspace_size(ips_plan p, size_t *bytes);
int ips_plan_table_size(ips_plan p, size_t *bytes);

/*
 * ips_plan_set_workspace -- let the plan run in caller-owned device memory.
 *   dev_ptr : device memory of the plan's device, 256-byte aligned, of at
 *             least ips_plan_workspace_size bytes; the caller keeps it valid
 *             and unused by others while work of this plan is enqueued or
 *             running.  NULL (with bytes = 0) returns the plan to a
 *             plan-owned workspace (allocated if needed).
 * Any plan-owned workspace is freed (hipFree, which waits for the device).
 * Several plans may share one buffer if their solves never overlap in time.
 * A plan created with IPS_FLAG_NO_WORKSPACE holds none until this call;
 * ips_execute on it returns IPS_E_WORKSPACE meanwhile.
 * Errors: IPS_E_WORKSPACE when bytes is too small (the plan is unchanged),
 * IPS_E_INVALID_ARG for a NULL plan, misaligned or host memory, or another
 * device.  d = 1 plans accept any buffer and use none.
 */
#define IPS_FLAG_NO_WORKSPACE 16u

int ips_plan_set_workspace(ips_plan p, void *dev_ptr, size_t bytes);

/*
 * ips_extension -- the enlarged grid of an automatically extended solve (host
 * only, no device work).  The method assumes that the support of rho lies at
 * least a distance sigma inside the box and that each panel count suits the
 * FFT; both are met by enlarging the box (Section 2, the assumptions on the
 * computational domain).  For each axis a, with the caller's mesh width kept:
 *   n_ext[a]  = the smallest n' >= n[a] + 2 margin[a] whose panel count n' - 1
 *               has no prime factor above 5;
 *   offset[a] = index of the caller's node 0 in the extended grid
 *               (margin[a] plus half the rounding, rounded down).
 * margin[a] = ceil(sigma / h[a]) nodes gives the distance sigma.
 * Errors: IPS_E_INVALID_ARG for d outside 1..3, n[a] < 3, margin[a] < 0 or any
 * NULL pointer.
 */
int ips_extension(int d, const int64_t *n, const int64_t *margin, int64_t *n_ext, int64_t *offset);

/*
 * ips_plan_create_extended -- a plan for the caller's grid n that solves on
 * the extended grid of ips_extension.  ips_execute on it places rho (all of
 * its nodes, boundary nodes included: they are interior nodes of the extended
 * box) into a zero extended array, solves there, and returns phi at the
 * caller's nodes; ips_execute_adjoint applies the transpose of that map
 * (embed, adjoint solve, restrict).  Arguments as ips_plan_create plus the d
 * margins (nodes added on each side before the rounding).  The two extended
 * arrays are part of the plan's workspace.  Batches do not take extended
 * plans.  Errors as ips_plan_create (the extended grid must meet its size
 * limits) and as ips_extension.
 */
int ips_plan_create_extended(ips_plan *out, int d, const int64_t *n, const double *h, int order,
                             int precision, unsigned flags, const int64_t *margin);

/*
 * ips_execute -- enqueue one solve on `stream` (a hipStream_t, NULL = null
 * stream).  Returns once the work is enqueued; it allocates nothing and
 * performs no host synchronisation, so it may be captured in a hipGraph.
 * rho and phi as in ips_solve; they must stay valid until the stream has
 * executed the work.
 */
int ips_execute(ips_plan p, const double *rho, double *phi, void *stream);

/*
 * ips_execute_static -- ips_execute without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The solve runs in a scratch array
 * that the library holds in device memory, one per GPU, of
 * IPS_STATIC_SCRATCH_BYTES bytes, instead of the plan's workspace; the
 * plan's own workspace binding is left as it was (a plan created with
 * IPS_FLAG_NO_WORKSPACE holds tables only).  The call itself allocates
 * nothing and performs no host synchronisation.
 *   p, rho, phi, stream : as ips_execute
 * Every call on one GPU shares that GPU's array and leaves its last contents
 * there; the solve writes every scratch value it reads, so nothing needs
 * clearing.  Calls whose work overlaps in time on one GPU (other streams,
 * other threads, other plans) race on the array: serialise them.
 * Errors: as ips_execute; IPS_E_WORKSPACE when the plan's workspace
 * (ips_plan_workspace_size) exceeds IPS_STATIC_SCRATCH_BYTES (3D grids up to
 * about 97^3 in FP64 fit); IPS_E_DEVICE if the array's address cannot be
 * obtained.
 */
#define IPS_STATIC_SCRATCH_BYTES (64u << 20)

int ips_execute_static(ips_plan p, const double *rho, double *phi, void *stream);

/*
 * ips_execute_adjoint -- enqueue rho_bar = A^T phi_bar, where A is the
 * linear map rho -> phi of the method (Sections 2-5) at the plan's grid and
 * order, i.e. the transpose of the FP64 solve.  FP64 plans run every step
 * in FP64.  Mixed plans run the sine transforms of the volume in FP32 tiles
 * (data in memory stay FP64; every other step FP64): the result then agrees
 * with the FP64 adjoint to a few FP32 roundings (about 3e-7 relative, as the
 * mixed forward solve).  The steps of the solve are transposed in
 * reverse order: the sine-transform solves are symmetric; the transfer of
 * boundary values (eq. harmonic4thOrderNH2D), the sixth-order stencils and
 * their cubic extrapolation (eqs. 6thOrderRelation2D/3D) are applied
 * transposed; the boundary sums of Section 4 become sums from the boundary
 * nodes over the interior, evaluated with the same kernel spectra.
 *   phi_bar : device array of the grid's size (all nodes, boundary included)
 *   rho_bar : device array of the same size, must not overlap phi_bar;
 *             its boundary entries are set to 0 (the solve ignores rho there)
 * Used for gradients: if J depends on phi, dJ/drho = A^T dJ/dphi.
 * Buffers: a plan created with IPS_FLAG_ADJOINT keeps them in its workspace;
 * otherwise the first adjoint call allocates them (later calls allocate
 * nothing).  About four interior volumes plus two grids (order 6) in FP64.
 */
#define IPS_FLAG_ADJOINT 2u

int ips_execute_adjoint(ips_plan p, const double *phi_bar, double *rho_bar, void *stream);

/*
 * Stage timing (diagnostics).  A plan created with IPS_FLAG_STAGE_TIMING
 * records a pair of HIP events around every stage of ips_execute on the
 * execution stream.  ips_plan_stage_time waits for the recorded events,
 * adds their elapsed times to the stage totals and returns the totals since
 * the last reset: *ms_total (milliseconds) and *calls (executions).
 */
#define IPS_FLAG_STAGE_TIMING 1u

typedef enum {
    IPS_STAGE_RHO_Z = 0,  /* cos/sin transform of rho along axis 2 (3D) */
    IPS_STAGE_CONV_X = 1, /* transform + convolution sum for the axis-0 faces */
    IPS_STAGE_CONV_Y = 2, /* same for the axis-1 faces (3D) */
    IPS_STAGE_RHO_Y = 3,  /* cos/sin transform of rho along axis 1 (3D) */
    IPS_STAGE_CONV_Z = 4, /* same for the axis-2 faces (3D); axis-1 faces (2D) */
    IPS_STAGE_FACES = 5,  /* chunk sums, inverse face transforms, boundary write */
    IPS_STAGE_SHELL_GT = 6, /* g~ and its sine transforms */
    IPS_STAGE_SHELL_R6 = 7, /* sixth-order right-hand side on the shell */
    IPS_STAGE_FINAL = 8,  /* spectral combination + inverse along axis 0 (1D: whole solve) */
    IPS_STAGE_INV_Y = 9,  /* inverse sine transform along axis 1 (3D) */
    IPS_STAGE_INV_Z = 10, /* inverse sine transform along the last axis into phi */
    IPS_STAGE_ADJOINT = 11, /* one whole ips_execute_adjoint */
    IPS_STAGE_SCREEN = 12,  /* screening charge and surface sums (IPS_FLAG_SCREENING;
                               its sine transforms of rho count as rho_z) */
    IPS_STAGE_COUNT = 13
} ips_stage;

const char *ips_stage_name(int stage);
int ips_plan_stage_time(ips_plan p, int stage, double *ms_total, int64_t *calls);
int ips_plan_reset_stage_times(ips_plan p);

/*
 * Boundary values from the screening charge (the James-type methods the
 * paper builds on, Sections 1 and 2) instead of the volume sums of Section 4.
 * A plan created with IPS_FLAG_SCREENING computes
 *   g(x) = surface integral of G(|x - s|) sigma(s) dS(s),  sigma = d phi_star / dn,
 * with sigma from the sine coefficients of phi_star (Section 3) and the surface
 * integral by the trapezoidal rule on each face (fourth-order Gregory weights
 * at the face edges, the target node left out, a third-order correction of
 * the 1/r or log r singularity at the target), then the harmonic part of
 * Section 5 as usual.  1D: the exact two-point sum.  FP64 only, no adjoint;
 * for d >= 2 every n[i] >= 7.  Its accuracy is that of the surface rule
 * (about second order), not the spectral accuracy of the volume sums.
 *
 * Evaluation of the 3D surface sums: by default, when every n[i] <= 768, as
 * convolutions -- the two faces of an axis by zero-padded 2D transforms over
 * the face axes, each pair of perpendicular face families by a transform along
 * their shared axis and, per wavenumber, a dense product over the other two
 * coordinates -- in O(n^3) work, with tables of about 3 n^3 doubles held by
 * the plan.  With IPS_FLAG_SCREEN_DIRECT too (and always in 2D or beyond that
 * size) by the direct sums over all surface nodes: O(boundary nodes^2) work,
 * no tables.  Both give the same sums up to rounding.
 */
#define IPS_FLAG_SCREENING 32u
#define IPS_FLAG_SCREEN_DIRECT 128u

/* Release a plan and its device memory (waits for nothing: the caller must
 * make sure no enqueued work still uses it). NULL is accepted. */
int ips_plan_destroy(ips_plan p);

/*
 * Tile autotuning.  A plan created with IPS_FLAG_AUTOTUNE times complete
 * solves of its geometry with every admissible LDS tile budget (1024, 2048
 * and 4096 complex elements per block) on scratch memory and keeps the
 * fastest; the choice is cached per (device, geometry, order, precision) for
 * the life of the process.  Without the flag the budget is 2048, or the
 * value of the environment variable IPS_TILE_WORK.
 */
#define IPS_FLAG_AUTOTUNE 4u

/*
 * ips_batch_create -- plans for `count` independent problems of possibly
 * different sizes and spacings, executed together (the batched form of the
 * solve of Sections 2-5; nothing is shared between problems).
 *   d[b], n[b][0..d[b]-1], h[b][0..d[b]-1] describe problem b
 *   order, precision : as ips_plan_create, for every problem
 *   flags : IPS_FLAG_ADJOINT, IPS_FLAG_AUTOTUNE and IPS_FLAG_SCREENING
 *           apply to every problem's plan (IPS_FLAG_STAGE_TIMING and
 *           IPS_FLAG_NO_WORKSPACE are ignored); IPS_FLAG_BATCH_EAGER makes
 *           ips_batch_execute launch the problems one after another on the
 *           caller's stream instead of through a graph; IPS_FLAG_BATCH_SMOOTH
 *           solves every problem on its extended grid with zero margin
 *           (ips_extension: each panel count rounded up to one with no prime
 *           factor above 5, as Section 2 prescribes for FFT-friendly panel
 *           counts) and returns phi at the caller's nodes -- the result is
 *           that of the enlarged box, not bit-identical to the plain solve;
 *           not combined with IPS_FLAG_SCREENING.
 */
#define IPS_FLAG_BATCH_EAGER 8u
#define IPS_FLAG_BATCH_SMOOTH 64u

int ips_batch_create(ips_batch *out, int count, const int *d, const int64_t (*n)[3],
                     const double (*h)[3], int order, int precision, unsigned flags);

/*
 * ips_batch_execute -- enqueue all problems of the batch on `stream`.
 *   rho[b], phi[b] : device arrays of problem b (host array of pointers);
 *                    rho[b] and phi[b] must not overlap
 * The first call (and any call with different array pointers) solves the
 * problems one after another on `stream` and then captures the same solves
 * into one HIP graph, spread over eight internal streams so that independent
 * problems can run side by side, largest first; later calls with the same
 * pointers replay that graph with a single launch on `stream`.  Capturing
 * creates the graph and, on first use, the internal streams; replays
 * allocate nothing.  One batch must not execute concurrently on two streams.
 */
int ips_batch_execute(ips_batch b, const double *const *rho, double *const *phi, void *stream);

int ips_batch_destroy(ips_batch b);

/* Static description of a status code. */
const char *ips_status_string(int status);

/* Copy the calling thread's last error message into buf (NUL-terminated,
 * truncated to len). Returns IPS_OK, or IPS_E_INVALID_ARG if buf is NULL. */
int ips_last_error_detail(char *buf, size_t len);

#ifdef __cplusplus
}
#endif

#endif /* IPOISSON_H */
