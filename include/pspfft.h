/*
 * pspfft.h -- C ABI of an MI355X (gfx950) implementation of the isolated
 * Poisson solve of Budiardja & Cardall, "Parallel FFT-based Poisson Solver for
 * Isolated Three-dimensional Systems" (arXiv:1106.0557, PSPFFT).
 *
 * The operation (Sec. 2.1).  Given a source S on an nx x ny x nz mesh with
 * constant spacings (hx, hy, hz), the library returns the potential
 *
 *     Phi_i = sum_{i' in mesh} G(i - i') S_{i'},
 *     G(p,q,r) = -hx hy hz / (4 pi sqrt(hx^2 p^2 + hy^2 q^2 + hz^2 r^2)),  (p,q,r) != 0,
 *     G(0,0,0) = -hx hy hz / (4 pi min(hx, hy, hz)),
 *
 * i.e. Eq. (greens2) evaluated at integer index offsets with the self-cell value
 * of Eq. (greens_function), which solves del^2 Phi = S with Phi -> 0 at infinity
 * (Eq. (poisson)) to discretisation error.  It is evaluated with Hockney's mesh
 * doubling (Sec. 2.1, Fig. 1): S is zero-padded to (2nx)(2ny)(2nz), transformed,
 * multiplied by the transform of the doubled Green's function, transformed back,
 * and the active octant is kept.  The transform of G is computed once, when the
 * plan is created (Sec. 2.2.2: computed at initialisation and stored permanently).
 *
 * Layout.  S and Phi are dense arrays of nx*ny*nz reals in the plan's precision,
 * x fastest: element (x, y, z) is at index (z*ny + y)*nx + x.  This is the
 * paper's convention of the first array dimension being x (Sec. 3.2).  A torch
 * tensor of shape (nz, ny, nx), contiguous, has this layout.
 *
 * Memory.  Every data pointer (S, Phi, workspace memory, Green's-function
 * output buffers) is a device pointer on the current HIP device.  The library
 * never takes ownership of caller memory.  Plans own their Green's-function
 * spectrum, twiddle tables and one default workspace.
 *
 * Streams.  Solve calls only enqueue work on the given stream and return
 * without synchronising; the caller keeps S and Phi alive until the stream has
 * passed that point.  Plan creation and destruction are synchronous.
 *
 * Errors.  Every call returns a pspfft_status.  Argument checks happen before
 * any work is enqueued; a failed check leaves nothing enqueued and nothing
 * allocated.  A failed kernel launch returns PSPFFT_ERR_DEVICE.  Failures are
 * also reported as messages of level PSPFFT_CONSOLE_ERROR (see Messages).
 *
 * Supported sizes.  Each of nx, ny, nz may be any 2^a 3^b 5^c from 1 to 2048
 * (2n <= 4096 points per doubled line), in both precisions.  Sizes 2^a * o with
 * o in {1, 3, 5, 9} and n >= 8, 10, 12, 18 (x: twice that, the packed real
 * transform having length n), up to 2048 (FP32) or 1152 (FP64) for y and z and
 * 4096 or 2304 for x, run on compile-time radix-family kernels; the other sizes
 * on a generic line kernel (slower; a plan that uses it reports a warning).
 * Rows nx of 2560, 3072 and 4096 (FP32) or 2304 (FP64) are also accepted.
 * Other sizes return PSPFFT_ERR_UNSUPPORTED_SIZE.
 * S and Phi must be aligned to two reals (8 bytes FP32, 16 bytes FP64).
 */
#ifndef PSPFFT_H
#define PSPFFT_H

#include <stddef.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pspfft_plan_s *pspfft_plan_t;           /* immutable after creation */
typedef struct pspfft_workspace_s *pspfft_workspace_t; /* mutable per-in-flight-solve buffer */

typedef enum {
    PSPFFT_OK = 0,
    PSPFFT_ERR_INVALID_ARGUMENT = 1, /* null pointer, non-finite or non-positive h, bad count */
    PSPFFT_ERR_UNSUPPORTED_SIZE = 2, /* mesh size outside the supported set */
    PSPFFT_ERR_OUT_OF_MEMORY = 3,    /* device allocation failed; nothing leaked */
    PSPFFT_ERR_DEVICE = 4,           /* a HIP call or kernel launch failed */
    PSPFFT_ERR_NOT_IMPLEMENTED = 5
} pspfft_status;

/* Arithmetic precision of a plan; stands in for the paper's compile-time real
 * kind KR (Sec. 3.2).  FP32 plans compute every pass in FP32 with twiddles and
 * Green's-function spectrum generated in FP64 and rounded once. */
typedef enum { PSPFFT_FP32 = 0, PSPFFT_FP64 = 1 } pspfft_precision;

/* The five passes of one solve (Sec. 2.2.2: x transforms, transpose, y
 * transforms, transpose, z transforms with the multiply by the Green's-function
 * transform, then the reverse sequence).  On one GPU the transposes become
 * strided column passes over the workspace.  A fused plan (pspfft_plan_fused)
 * does the x and y transforms of each z plane in one kernel: its
 * PSPFFT_PASS_X_FWD also covers Y_FWD, its PSPFFT_PASS_X_INV also covers
 * Y_INV, and its two y passes do nothing. */
typedef enum {
    PSPFFT_PASS_X_FWD = 0,  /* zero-padded real-to-complex transforms along x     */
    PSPFFT_PASS_Y_FWD = 1,  /* transforms along y, upper half of the input zero   */
    PSPFFT_PASS_Z_CONV = 2, /* forward z transform, multiply by G~, inverse z      */
    PSPFFT_PASS_Y_INV = 3,  /* inverse transforms along y, only y < ny kept        */
    PSPFFT_PASS_X_INV = 4   /* inverse complex-to-real along x, only x < nx kept   */
} pspfft_pass;

/*
 * Create a solver for an nx x ny x nz mesh with spacings h[0..2] = (hx, hy, hz)
 * (Sec. 3.2, Create: CellWidth and nTotalCells; the communicator has no analogue
 * on one GPU).  Computes the transform of the doubled Green's function
 * (Eq. (greens_function)) in FP64 on the device, scales it by
 * 1/((2nx)(2ny)(2nz)) and keeps it resident in the plan's precision.
 * Synchronous.  *out receives the plan on success and is untouched on failure.
 */
pspfft_status pspfft_plan_create(int nx, int ny, int nz, const double h[3], pspfft_precision prec,
                                 pspfft_plan_t *out);

/*
 * Messages (Sec. 3.2, the optional VerbosityOption of Create): levels in
 * increasing verbosity.  The library prints messages of the level in force and
 * below to stderr, each line prefixed "[pspfft <kind>]", or hands them to the
 * callback set with pspfft_set_log_callback.  The process-wide level is
 * PSPFFT_CONSOLE_ERROR unless the environment variable PSPFFT_LOG says
 * error | warn | info1 | info2, or pspfft_set_verbosity changes it; a plan
 * created with PSPFFT_PLAN_VERBOSITY(level) uses that level for its own
 * messages.
 *   ERROR    every failed call, with its reason
 *   WARNING  conditions that cost speed (an axis on the generic line kernel)
 *   INFO_1   one line per plan created (size, form of the passes, resident
 *            bytes, workspace bytes) and per plan destroyed
 *   INFO_2   the stage plan of each axis, and every kernel launch
 */
typedef enum {
    PSPFFT_CONSOLE_ERROR = 0,
    PSPFFT_CONSOLE_WARNING = 1,
    PSPFFT_CONSOLE_INFO_1 = 2,
    PSPFFT_CONSOLE_INFO_2 = 3
} pspfft_verbosity;

/* Set the process-wide level; an unknown level returns PSPFFT_ERR_INVALID_ARGUMENT. */
pspfft_status pspfft_set_verbosity(pspfft_verbosity level);
pspfft_verbosity pspfft_get_verbosity(void);

/* Receiver of messages: level, the text (no newline; valid during the call) and
 * the user pointer given to pspfft_set_log_callback.  May be called from any
 * thread that calls the library, one message at a time (under a library lock:
 * the receiver must not call back into the library). */
typedef void (*pspfft_log_fn)(pspfft_verbosity level, const char *message, void *user);
/* Send messages to fn instead of stderr; NULL goes back to stderr. */
pspfft_status pspfft_set_log_callback(pspfft_log_fn fn, void *user);

/* Plan options for pspfft_plan_create_ex. */
typedef enum {
    PSPFFT_PLAN_DEFAULT = 0,
    /* Always run the five separate passes, even where the x and y transforms
     * of a plane could share one kernel. */
    PSPFFT_PLAN_FIVE_PASS = 1
} pspfft_plan_flags;
/* Option bits 4..6: the plan's own message level (the paper's VerbosityOption
 * argument of Create), PSPFFT_PLAN_VERBOSITY(PSPFFT_CONSOLE_INFO_1) and so on. */
#define PSPFFT_PLAN_VERBOSITY_SHIFT 4
#define PSPFFT_PLAN_VERBOSITY(level) ((unsigned)((level) + 1) << PSPFFT_PLAN_VERBOSITY_SHIFT)

/*
 * As pspfft_plan_create, with options (a bitwise or of pspfft_plan_flags and
 * at most one PSPFFT_PLAN_VERBOSITY; unknown bits return
 * PSPFFT_ERR_INVALID_ARGUMENT).  By default a plan fuses
 * the x and y transforms of each z plane when nx == ny = E*K (E in
 * {16, 20, 24, 36}, K a power of two dividing the power-of-two part of E, so at
 * most two stages) and the plane of x spectra fits in the 160 KB of LDS: FP32
 * up to n = 128, FP64 up to n = 80.  Both forms compute the same potential to
 * rounding; the fused one moves 2ny nz (nx+1) fewer complex values per solve.
 */
pspfft_status pspfft_plan_create_ex(int nx, int ny, int nz, const double h[3], pspfft_precision prec,
                                    unsigned flags, pspfft_plan_t *out);

/* 1 if the plan runs fused x-y plane kernels, 0 otherwise (and for NULL). */
int pspfft_plan_fused(pspfft_plan_t plan);

/*
 * 1 if the plan keeps its spectrum kz-fastest, 0 otherwise (and for NULL).
 * That is the case where the z pass keeps each line within one wavefront,
 * which reads its spectrum values in contiguous runs: z lines of three stages
 * E, M, K with 16, 32 or 64 threads per line (2 nz = 16*16*2, 36*4*4, 24*8*4,
 * 16*16*4 or 24*8*8, that is nz = 256, 288, 384, 512 or 768), four-stage FP32
 * lines of 32 or 64 threads (nz = 576, 1152, 320, 640), the FP32 32-family's
 * 2048-point lines (nz = 1024), each where a z line's block of NB*2ny*nx
 * positions stays below 4 GB; and z lines on the generic kernel (nz outside
 * the radix families), whose lanes of a line walk consecutive kz.
 * pspfft_plan_green exports the same octant either way.
 */
int pspfft_plan_spectrum_kz_fastest(pspfft_plan_t plan);

/*
 * Workspace layout, for code that reads a workspace between passes (tests,
 * debugging).  A workspace of this plan holds, in the plan's complex type,
 *   W  = [nz / B][2 ny][B][nx]  then, 256-byte aligned,  Wn = [nz][2 ny],
 * where B = pspfft_workspace_ztile(plan) (a power of two up to 16 dividing nz):
 * the value at (z, ky, kx < nx) is W[z / B][ky][z % B][kx] and the one at kx = nx
 * is Wn[z][ky].  Grouping B z planes keeps each z line of the z pass within
 * nz / B memory regions.  After the forward x and y passes it holds the
 * transform along x and y of the zero-padded source for z < nz; after the z pass
 * the same after the convolution.  Returns 0 for NULL.
 */
int pspfft_workspace_ztile(pspfft_plan_t plan);

/* Release a plan and everything it owns (Sec. 3.2, Destroy).  The memory is
 * freed with hipFree, which waits for the work already queued on the device,
 * so kernels still reading the plan finish first; destroying a plan therefore
 * waits for every stream of the device: destroy plans when the device is idle
 * (a server's plan cache at shutdown).  Workspaces created for the plan must be
 * destroyed first.  NULL returns PSPFFT_ERR_INVALID_ARGUMENT. */
pspfft_status pspfft_destroy(pspfft_plan_t plan);

/*
 * Phi = potential of S (Sec. 3.2, Solve).  S and Phi: device arrays of nx*ny*nz
 * reals in the plan's precision, layout as above.  S == Phi is allowed (the
 * paper overwrites the source with the potential).  Uses the plan's default
 * workspace, allocated by the first call (PSPFFT_ERR_OUT_OF_MEMORY if that
 * fails), so solves on one plan serialise on that workspace: concurrent solves
 * need a workspace each (pspfft_solve_ws).  Enqueues five kernels, or three for
 * a fused plan.
 */
pspfft_status pspfft_solve(pspfft_plan_t plan, const void *S, void *Phi, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid allocation): as
 * pspfft_solve, with the workspace in a library-owned device array of
 * PSPFFT_NOALLOC_MAX_BYTES (128 MiB) instead of the plan's default workspace.
 * The call allocates no device memory and creates no HIP objects; the caller
 * creates the plan beforehand and passes S and Phi as for pspfft_solve.  Every
 * GPU the library runs on holds one such array from the time the library's
 * device code is loaded there until the process ends; the array of the current
 * device (which must be the plan's) is used.  Meshes whose workspace
 * (pspfft_workspace_bytes) exceeds PSPFFT_NOALLOC_MAX_BYTES return
 * PSPFFT_ERR_UNSUPPORTED_SIZE with an error message (FP32 192^3 and FP64 160^3
 * fit, FP32 256^3 does not).  Nothing in the array has to start at zero (every pass writes
 * what the next one reads).  All calls on one GPU share its array: calls that
 * overlap in time on that GPU (different streams, or different host threads
 * without ordering) race and give wrong results.
 */
#define PSPFFT_NOALLOC_MAX_BYTES ((size_t)128 << 20)
pspfft_status pspfft_solve_noalloc(pspfft_plan_t plan, const void *S, void *Phi, hipStream_t stream);

/* Allocate a workspace for one in-flight solve of this plan
 * (pspfft_workspace_bytes bytes of device memory, owned by the workspace). */
pspfft_status pspfft_workspace_create(pspfft_plan_t plan, pspfft_workspace_t *out);

/* Wrap caller-owned device memory (at least pspfft_workspace_bytes bytes,
 * 256-byte aligned) as a workspace.  The memory stays the caller's. */
pspfft_status pspfft_workspace_wrap(pspfft_plan_t plan, void *memory, size_t bytes,
                                    pspfft_workspace_t *out);

/* Release a workspace handle, and its memory unless it was wrapped (hipFree,
 * after the work queued on the device). */
pspfft_status pspfft_workspace_destroy(pspfft_workspace_t ws);

/* As pspfft_solve, with an explicit workspace created for the same plan. */
pspfft_status pspfft_solve_ws(pspfft_plan_t plan, pspfft_workspace_t ws, const void *S, void *Phi,
                              hipStream_t stream);

/*
 * Solve `count` independent problems.  plans[i], ws[i], S[i], Phi[i] describe
 * problem i; plans may differ in size and precision; each ws[i] must belong to
 * plans[i] and be distinct from every other ws[j].  Every argument is checked
 * before anything is enqueued.  The problems of one plan go through the five
 * passes together, one launch per pass (at most 32 problems per launch); when
 * the batch holds several plans, each plan's problems run on a stream of the
 * library's own (8 per device, default priority), side by side, forked from and
 * joined back into `stream` by events: the batch is ordered after the work
 * queued on `stream` before the call and before the work queued after it, as
 * if it ran on `stream`.  Results do not depend on what else is in the batch:
 * every problem is cut into the same tiles whatever its neighbours.  A launch
 * whose problems' workspaces together exceed 256 MB (about the device's
 * Infinity Cache) streams its line data through nontemporal loads and stores
 * in the z pass and the inverse plane pass; the arithmetic and the results are
 * the same.
 */
pspfft_status pspfft_solve_batched(int count, const pspfft_plan_t *plans, const pspfft_workspace_t *ws,
                                   const void *const *S, void *const *Phi, hipStream_t stream);

/*
 * Run a single pass of the solve for `count` problems (same argument meaning as
 * pspfft_solve_batched).  Running PSPFFT_PASS_X_FWD .. PSPFFT_PASS_X_INV in
 * order on the same stream equals pspfft_solve_batched.  Used by schedulers that
 * let problems join at pass granularity, and to time passes separately.  S is
 * read only by PSPFFT_PASS_X_FWD and Phi written only by PSPFFT_PASS_X_INV.
 */
pspfft_status pspfft_pass_batched(pspfft_pass pass, int count, const pspfft_plan_t *plans,
                                  const pspfft_workspace_t *ws, const void *const *S, void *const *Phi,
                                  hipStream_t stream);

/* Device bytes a plan keeps resident (Green's-function spectrum, twiddles,
 * plan tables, and the default workspace once pspfft_solve has allocated it).
 * 0 for NULL. */
size_t pspfft_plan_bytes(pspfft_plan_t plan);

/* Device bytes a plan of this size keeps resident once created, before its
 * first pspfft_solve (spectrum octant, twiddle tables, plan table): what
 * pspfft_plan_bytes returns for it.  Host-side arithmetic only; 0 for an
 * unsupported size.  Lets a scheduler count a plan in its memory budget before
 * creating it. */
size_t pspfft_plan_resident_bytes(int nx, int ny, int nz, pspfft_precision prec);

/* Bytes of one workspace: 2 ny nz (nx + 1) complex values of the precision.
 * 0 for an unsupported size. */
size_t pspfft_workspace_bytes(int nx, int ny, int nz, pspfft_precision prec);

/* Algorithmic HBM bytes one pass moves for one problem of this plan: the
 * values it must read and write once each (zero halves never touched).  Used
 * for effective-bandwidth reports.  0 for NULL, an unknown pass, or a y pass of
 * a fused plan (its x passes then count the fused traffic). */
size_t pspfft_pass_bytes(pspfft_plan_t plan, pspfft_pass pass);

/* Size, spacings and precision of a plan (any output pointer may be NULL). */
pspfft_status pspfft_plan_info(pspfft_plan_t plan, int dims[3], double h[3], pspfft_precision *prec);

/*
 * Copy the plan's Green's-function spectrum to `dst` (device memory of
 * (nz+1)(ny+1)(nx+1) reals in the plan's precision): dst[(kz*(ny+1) + ky)*(nx+1)
 * + kx] = DFT(doubled G)(kx, ky, kz) / ((2nx)(2ny)(2nz)) for kx <= nx, ky <= ny,
 * kz <= nz.  The transform is real and even in each axis, so this octant holds
 * all of it.  Enqueued on `stream`.
 */
pspfft_status pspfft_plan_green(pspfft_plan_t plan, void *dst, hipStream_t stream);

/* Static, human-readable description of a status code. */
const char *pspfft_status_string(pspfft_status s);

#ifdef __cplusplus
}
#endif

#endif /* PSPFFT_H */
