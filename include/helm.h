/*
 * helm.h -- C ABI of the MI355X (gfx950) FFT-based fast direct solver for the
 * separable finite-element Helmholtz problem
 *
 *     -Laplace(u) - omega^2 u = f   in [0, L_1] x ... x [0, L_d],  d = 2, 3,
 *     du/dn - i*omega*u = 0 on absorbing faces, du/dn = 0 on Neumann faces,
 *
 * discretised by bilinear (9-point) or trilinear (27-point) elements on a
 * uniform tensor mesh (Toivanen & Wolfmayr, "A fast Fourier transform based
 * direct solver for the Helmholtz problem", Section 2, eqs. (A2D), (A3D)).
 *
 * The solve is the three-step method of Section 3.1 (periodic auxiliary
 * problem along x_1, boundary partial solution, corrected periodic solve), in
 * 3D nested along x_2 as in Section 5: forward DFTs along the periodised axes,
 * batched complex tridiagonal solves along the last axis, inverse DFTs.
 *
 * Conventions shared by every entry point:
 *   - Arrays are complex128, interleaved (re, im) doubles, C-ordered
 *     [nrhs][n_1][n_2]([n_3]) with x_1 the slowest axis (the Kronecker
 *     ordering of eqs. (A2D), (A3D)).
 *   - Pointers named f, u, r are DEVICE pointers (memory of the current HIP
 *     device, e.g. torch tensors' data_ptr()); the caller owns them.
 *   - stream is a hipStream_t or NULL for the default stream.
 *   - Every function returns a status code (HELM_OK = 0, negative on error);
 *     no C++ exception crosses this boundary.
 *   - Tuning: a 3D plan times, at setup, the two block layouts of the line
 *     solves that reduce over the x_1 modes (each block one x_2 mode over
 *     many x_1 modes, or consecutive x_2 modes at one x_1 mode; both give
 *     the same sums) and keeps the faster; HELM_RED_L_LAYOUT=2 or 3 in the
 *     environment at setup fixes the choice instead (tests).  With
 *     helm_options.tune_cache set, this and the other measured choices
 *     (transform, boundary tables) are read from / appended to that file.
 */
#ifndef HELM_H
#define HELM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define HELM_OK            0
#define HELM_EINVAL       -1  /* bad argument: dimension, grid < 3, nrhs < 1, null pointer */
#define HELM_ENOMEM       -2  /* device or host allocation failed */
#define HELM_EDEVICE      -3  /* a HIP runtime call failed */
#define HELM_ESINGULAR    -4  /* the system is singular or degenerate (omega = 0 is always rejected) */
#define HELM_ENOCONV      -5  /* refinement did not reach tol within max_iter (u holds the last iterate) */
#define HELM_ENONFINITE   -6  /* f (or an intermediate residual) holds NaN or Inf */
#define HELM_EUNSUPPORTED -7  /* valid problem outside what this build implements */

/* Precision of the bulk transforms and tridiagonal sweeps. */
#define HELM_PREC_FP64   0  /* complex128 storage and arithmetic throughout */
#define HELM_PREC_MIXED  1  /* complex64 storage of the transforms and sweep inputs/outputs,
                               FP64 recurrence arithmetic, FP64 stencil residual and
                               FP64 solution update (iterative refinement) */

/* Solver options.  helm_default_options fills: precision = HELM_PREC_FP64,
 * tol = 1e-10, max_iter = 8, check = 1, transform = FFT, tune_cache = NULL,
 * boundary = AUTO, eigen = AUTO. */
/* Transform along the periodised axes (helm_options.transform):
 *   FFT   the fast method of Sections 4.2 / 5.2: DFTs of the periodic
 *         problem, three line passes and the boundary steps;
 *   DENSE diagonalisation with the full absorbing-boundary eigenvectors,
 *         u = (V (x) I) T^{-1} (V^T (x) I) f (eq. (A2Dinv); 3D with V_1 (x) V_2):
 *         two dense complex transforms on the matrix cores and one line pass;
 *         periodised lengths up to HELM_DENSE_MAX;
 *   AUTO  the plan times both at setup (one right-hand side, the plan's
 *         precision) and keeps the faster; with tune_cache set, decisions are
 *         read from and appended to that text file, keyed by the problem shape. */
#define HELM_TRANSFORM_AUTO  0
#define HELM_TRANSFORM_FFT   1
#define HELM_TRANSFORM_DENSE 2
#define HELM_DENSE_MAX 1024

/* Evaluation of the boundary steps in 3D (helm_options.boundary; 2D always
 * uses line sweeps).  Step 2 of the method (eqs. (step2-1)-(step2-3)) maps two
 * boundary vectors to w_k = sum_k' sum_j V^b[k,j] V^b[k',j] T_j^{-1} r_k', a
 * linear map that depends on the operator only:
 *   LINES   sweep the N/n_3 line systems for it in every solve (the inner
 *           Step 2 of the outer Steps 1 and 3, and the whole outer Step 2);
 *   TABLES  build that map once at setup as dense n_3 x n_3 blocks (per outer
 *           mode for the inner Step 2, per inner absorbing mode for the outer
 *           Step 2, the latter after the dense inner eigenvector transform of
 *           the two boundary planes) and apply it as a batched matrix product:
 *           5 of the 9 line sweeps of a 3D solve become products with
 *           64 n_3^2 (n_1 + n_2) bytes of tables
 *           (complex128; half that, complex64, for HELM_PREC_MIXED plans);
 *   AUTO    build the tables when they fit the memory budget (at most 32 GiB
 *           and a quarter of the free device memory) and use them for solves
 *           of at least as many right-hand sides as the plan measured them to
 *           pay for (timed at setup with 1 and 16 right-hand sides; cached in
 *           tune_cache when set).
 * Both give A^{-1} f up to rounding. */
#define HELM_BOUNDARY_AUTO   0
#define HELM_BOUNDARY_LINES  1
#define HELM_BOUNDARY_TABLES 2

/* Where the absorbing-boundary eigenpairs of eq. (EVP1a) are computed at setup
 * (helm_options.eigen; Section 6 notes that this eigen-solve dominates the
 * initialisation):
 *   HOST    the host root finder and extended-precision inverse iteration
 *           (OpenMP; helm_eig1d);
 *   DEVICE  the same method on the current HIP device, one thread per root
 *           (Aberth sweeps in FP64, inverse iteration in double-double
 *           arithmetic; helm_eig1d_device), with the whole eigenvectors, when
 *           the plan needs them, written straight to device memory;
 *   AUTO    DEVICE.
 * Both meet the same acceptance checks (normwise backward error below 1e-12
 * per pair, distinct eigenvalues); the eigenvalues agree to rounding. */
#define HELM_EIGEN_AUTO   0
#define HELM_EIGEN_HOST   1
#define HELM_EIGEN_DEVICE 2

typedef struct helm_options {
    int    precision; /* HELM_PREC_FP64 or HELM_PREC_MIXED */
    double tol;       /* target ||f - A u||_2 / ||f||_2 per right-hand side */
    int    max_iter;  /* maximum refinement steps after the first solve */
    int    check;     /* FP64 path: 1 = evaluate the FP64 residual after the solve and
                         refine while it exceeds tol; 0 = one plain solve, no residual.
                         The mixed path always checks. */
    int    transform; /* HELM_TRANSFORM_*; default FFT */
    const char* tune_cache; /* AUTO only: decision cache file, or NULL */
    int    boundary;  /* HELM_BOUNDARY_*; default AUTO */
    int    eigen;     /* HELM_EIGEN_*; default AUTO */
} helm_options;

void helm_default_options(helm_options* opt);

/* Opaque plan: owns the 1D spectral data, the device tables and its device
 * workspace. */
typedef struct helm_plan helm_plan;

/*
 * helm_setup -- build a plan for one operator (Sections 3.2, 4.1, 5.1).
 *   dim    2 or 3
 *   grid   host array of dim node counts n_j >= 3 (nodes 0..n_j-1)
 *   h      host array of dim mesh sizes h_j > 0 (the paper uses h_j = 1/(n_j - 1))
 *   omega  wavenumber (finite)
 *   abc    face mask: bit 2j = low face of axis j is absorbing, bit 2j+1 = high
 *          face; clear bits are Neumann faces.  Any combination is accepted
 *          on the periodised axes (x_1, and x_2 in 3D); the last axis needs
 *          at least one absorbing face (else its tridiagonal systems can be
 *          exactly singular).
 *   opt    options or NULL for the defaults
 *   out    receives the plan
 * Computes the 1D spectra: closed-form periodic spectra (eqs. (eigvectorsPer),
 * (eigvaluesPer)) on the host and the absorbing-boundary generalized
 * eigenpairs K V = M V Lambda^A (eq. (EVP1a), normalised as in eq. (EVPcondA))
 * on the current HIP device or the host (helm_options.eigen), and builds the
 * plan's device tables there.
 * Size limits of this build: the last (line) axis has at most 4097 nodes;
 * a periodised axis of n nodes needs a transform length (n itself for a power
 * of two, else a chirp-z length >= 2n - 1) of at most 2^18.
 * Errors: HELM_EINVAL, HELM_ESINGULAR (omega = 0: every absorbing face then
 * degenerates to a Neumann face and A annihilates the constants, so it is
 * rejected whatever the mask), HELM_EUNSUPPORTED (no absorbing face on the
 * last axis, or a length beyond the limits above), HELM_ENOCONV (the
 * eigen-setup of an axis found two coinciding eigenvalues: with both faces
 * absorbing and at most about 3 points per wavelength on that axis, the two
 * faces' boundary modes share one eigenvalue to rounding, and the plan does
 * not choose a basis of that eigenspace), HELM_ENOMEM, HELM_EDEVICE.
 */
int helm_setup(int dim, const int64_t* grid, const double* h, double omega,
               uint32_t abc, const helm_options* opt, helm_plan** out);

/*
 * helm_setup_general -- the same for the operator with a zeroth-order
 * coefficient of either sign and Robin (impedance) faces, the other separable
 * problems of Section 1: -Lap u - c u = f in the box, du/dn + g u = 0 on each
 * face (outward normal).  The Galerkin matrices are those of eqs. (A2D),
 * (A3D) with c in place of omega^2 and the corner entries of K_j
 * (eq. (matrixK)) equal to 1/h_j + g of the face; helm_setup is the case
 * c = omega^2, g = -i omega on absorbing faces (eq. (1st-order-abc)) and
 * g = 0 on Neumann faces.
 *   c      real zeroth-order coefficient (c < 0: modified Helmholtz, c = 0: Laplace)
 *   gamma  host array of 4 dim doubles: g of the low face of axis j at
 *          (gamma[4j], gamma[4j+1]) = (Re, Im), of the high face at
 *          (gamma[4j+2], gamma[4j+3])
 * Accepted coefficient sets (every line system of the method nonsingular):
 * some face of the last axis with Im g != 0 and no two faces with Im g of
 * opposite signs; or every g real and >= 0 with c < 0, or with c = 0 and
 * g > 0 on a face of the last axis.  Errors as helm_setup: HELM_EINVAL
 * (non-finite c or g, bad sizes), HELM_ESINGULAR (c = 0 and g = 0 on every
 * face: A annihilates the constants), HELM_EUNSUPPORTED (other coefficient
 * sets, where resonant line systems are possible; size limits).
 */
int helm_setup_general(int dim, const int64_t* grid, const double* h, double c,
                       const double* gamma, const helm_options* opt, helm_plan** out);

/*
 * helm_solve -- u = A^{-1} f for nrhs right-hand sides.
 *   f  device, read only, complex128 [nrhs][grid]
 *   u  device, written, complex128 [nrhs][grid]; must not overlap f
 * All kernels run on `stream`.  With checking (mixed precision, or FP64 with
 * opt.check = 1) the call synchronises `stream` to read the residual norms
 * (once per refinement step on the host loop, once per call on a captured
 * solve); a plain FP64 solve (check = 0) is fully asynchronous.  A call that
 * repeats the previous call's arguments (f, u, nrhs, stream) captures the
 * whole solve, with as many device-controlled refinement steps as the
 * previous call took, into a HIP graph that later repeats launch; if those
 * steps fall short of opt.tol the host loop continues and the next call
 * captures again.  Results and the report are those of the host loop.
 * Per-kernel profiling (helm_profile) always runs the host loop.  The plan's
 * workspace grows on demand for larger nrhs (dropping captured graphs); a plan
 * must not be used from two streams at once.
 * Errors: HELM_EINVAL, HELM_ENOMEM, HELM_EDEVICE, HELM_ENOCONV (u holds the
 * last iterate), HELM_ENONFINITE (f holds NaN/Inf).
 */
int helm_solve(helm_plan* p, const void* f, void* u, int nrhs, void* stream);

/*
 * helm_solve_static -- helm_solve for callers that cannot allocate device
 * memory: code under HIP stream capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, kernels, results and report as
 * helm_solve on the same plan, but the workspace of the solve is taken from a
 * device array of HELM_STATIC_SCRATCH_BYTES bytes that the library holds on
 * every GPU it runs on until the process ends, not from the plan's own
 * workspace, and nothing is allocated (no hipMalloc, hipFree or host
 * allocation: the plan builds every table it needs at setup).  The solve
 * always runs eagerly with the refinement loop on the host (no captured
 * graph; under a caller's stream capture only an unchecked FP64 solve can be
 * recorded, since checking reads the residual norms on the host), and
 * per-kernel profiling does not apply.
 * Limits: nrhs <= HELM_STATIC_MAX_RHS, and the workspace of the solve (about
 * three to four N x nrhs arrays of the plan's storage precision, plus
 * boundary planes and partial sums) at most HELM_STATIC_SCRATCH_BYTES;
 * larger solves return HELM_ENOMEM before any work is enqueued.
 * Sharing: every call on one GPU uses that GPU's one array, which keeps the
 * last call's contents (every kernel of a solve writes the workspace it later
 * reads, so nothing needs clearing); calls that overlap in time on one GPU
 * (two streams, two threads) race, and the caller must serialise them.
 * The current device must be the plan's (else HELM_EINVAL).
 * Errors: as helm_solve, and HELM_ENOMEM for sizes beyond the limits.
 */
#define HELM_STATIC_SCRATCH_BYTES (128u << 20)
#define HELM_STATIC_MAX_RHS 1024
int helm_solve_static(helm_plan* p, const void* f, void* u, int nrhs, void* stream);

/* Report of the last helm_solve on this plan. */
typedef struct helm_report {
    int    status;            /* status returned by the last solve */
    int    iterations;        /* refinement steps taken after the first solve */
    int    precision;         /* HELM_PREC_* used */
    int    nrhs;
    double rel_residual_max;  /* max over RHS of ||f - A u|| / ||f|| (FP64), -1 if unchecked */
    double rel_residual_first;/* same after the first solve, -1 if unchecked */
    int    transform;         /* HELM_TRANSFORM_FFT or _DENSE: the variant the plan runs */
    int    boundary;          /* HELM_BOUNDARY_LINES or _TABLES: how the boundary steps ran */
} helm_report;

int helm_report_get(const helm_plan* p, helm_report* out);

/*
 * helm_residual -- r = f - A u in FP64 with the matrix-free 9-/27-point
 * operator of eqs. (A2D)/(A3D), and per right-hand side
 * rel_res[k] = ||r_k||_2 / ||f_k||_2.
 *   u, f  device, complex128 [nrhs][grid]
 *   r     device complex128 [nrhs][grid], or NULL to compute the norms only
 *   rel_res host array of nrhs doubles (written after the stream is synchronised)
 */
int helm_residual(helm_plan* p, const void* u, const void* f, void* r,
                  double* rel_res, int nrhs, void* stream);

/*
 * Per-kernel timing.  With helm_profile(p, 1) every kernel launch of later
 * solves on this plan is bracketed by two HIP events recorded on the solve's
 * stream; helm_kernel_stats_get synchronises on the last event and returns,
 * per kernel function, the summed event time (ms), the number of launches and
 * the summed algorithmic bytes (the N-sized arrays each launch must read and
 * write once: 2 x element size per unknown for a transform pass, 1x, 0x or 2x
 * for the Step 1 / Step 2 / Step 3 line solves, 32 bytes for the FP64
 * residual; the table bytes for the boundary-table products).  reset != 0
 * clears the accumulators afterwards.
 */
#define HELM_NKERNELS 9
typedef struct helm_kernel_stats {
    double ms[HELM_NKERNELS];
    double bytes[HELM_NKERNELS];
    int    calls[HELM_NKERNELS];
} helm_kernel_stats;

int helm_profile(helm_plan* p, int on);
int helm_kernel_stats_get(helm_plan* p, helm_kernel_stats* out, int reset);
/* Name of kernel slot k (the device function timed in that slot), or NULL. */
const char* helm_kernel_name(int k);

/* Release the plan and its device memory (synchronises the device first). */
void helm_destroy(helm_plan* p);

/*
 * Batches: many independent problems (uneven grids, omega, precision) solved
 * by one graph launch.  The method is applied to every problem unchanged
 * (Sections 4.2, 5.2); batching is a scheduling layer above it.
 *
 * helm_batch_create -- group `count` distinct plans (same device; a plan may
 *   belong to one batch at a time and must not be solved on its own while the
 *   batch runs).  Each plan's workspace is sized for max_nrhs right-hand
 *   sides now.  The batch owns side streams but not the plans.
 *   Errors: HELM_EINVAL, HELM_ENOMEM, HELM_EDEVICE.
 *
 * helm_batch_solve -- u[i] = A_i^{-1} f[i] for every plan i, nrhs[i] <= max_nrhs
 *   right-hand sides each, same layout and ownership as helm_solve.  On the
 *   first call, or when any pointer, count or the stream differs from the
 *   previous call, it solves each problem once eagerly on `stream` (this also
 *   sets the refinement depth: one step more than those inputs needed, at
 *   least 2, at most the plan's max_iter), then captures every problem's
 *   complete solve into one graph, the problems on parallel branches, and
 *   instantiates it.  Every call then launches that graph on `stream` and
 *   returns without synchronising.  Checked plans (mixed precision, or
 *   opt.check) refine under device control: a residual check kernel stops
 *   the refinement of a problem by raising a flag that makes its remaining
 *   launches return at once.
 *   Errors: HELM_EINVAL, HELM_ENOMEM, HELM_EDEVICE, or the status of a
 *   failing eager solve.
 *
 * helm_batch_report_get -- report of problem i from the last batch solve
 *   (synchronises the stream of that solve).  status HELM_ENOCONV if the
 *   captured refinement depth did not reach tol, HELM_ENONFINITE for NaN/Inf.
 */
typedef struct helm_batch helm_batch;
int helm_batch_create(helm_plan* const* plans, int count, int max_nrhs, helm_batch** out);
int helm_batch_solve(helm_batch* b, const void* const* f, void* const* u, const int* nrhs,
                     void* stream);
int helm_batch_report_get(helm_batch* b, int i, helm_report* out);
/* Release the batch (synchronises the device first); the plans stay valid. */
void helm_batch_destroy(helm_batch* b);

/* Static description of a status code. */
const char* helm_strerror(int code);

/*
 * helm_eig1d -- host-only FP64 generalized eigenpairs of the 1D pencil
 * (K, M) of eqs. (matrixK), (matrixM): K v_l = lambda_l M v_l (eq. (EVP1a)),
 * normalised v_l^T M v_l = 1 (eq. (EVPcondA), plain transpose).
 *   n       nodes (>= 3), h mesh size, omega wavenumber
 *   abc_lo, abc_hi  1 = absorbing face, 0 = Neumann face
 *   lam     host, 2n doubles: eigenvalues (interleaved complex), sorted by real part
 *   vb      host, 4n doubles: boundary rows [2][n] complex: vb[0][l] = v_l(0),
 *           vb[1][l] = v_l(n-1); the common sign of a column is arbitrary
 * Runs no device code.  Errors: HELM_EINVAL, HELM_ENOCONV (root finder or
 * refinement failed, or two eigenvalues coincide to 1e-9 relative, as the
 * two boundary modes of a doubly absorbing axis do at about 3 points per
 * wavelength and below), HELM_ENOMEM.
 */
int helm_eig1d(int64_t n, double h, double omega, int abc_lo, int abc_hi,
               double* lam, double* vb);

/*
 * helm_eig1d_device -- the same eigenpairs, computed on the current HIP device
 * by the method of HELM_EIGEN_DEVICE (Aberth-Ehrlich sweeps on
 * det(K - lambda M) in FP64, then inverse iteration per root with the
 * complex-symmetric Rayleigh quotient in double-double arithmetic, at least
 * three steps and up to eight until the quotient settles to 1e-26).
 * Arguments and output layout as helm_eig1d (host arrays; the call
 * synchronises).  Allocates device memory for its workspace (at most 4 GiB
 * plus O(n) bytes) and frees it before returning.
 * Errors: HELM_EINVAL (n < 3 or n > 2^20, h <= 0, non-finite omega, null
 * arrays), HELM_ENOCONV, HELM_ENOMEM, HELM_EDEVICE.
 */
int helm_eig1d_device(int64_t n, double h, double omega, int abc_lo, int abc_hi,
                      double* lam, double* vb);

#ifdef __cplusplus
}
#endif

#endif /* HELM_H */
