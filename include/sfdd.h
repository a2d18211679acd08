/*
 * sfdd.h - C ABI of the overlapping-Schwarz optical-flow solver for MI355X.
 *
 * Method: Gilliocq-Hirtz & Belhachmi, "A massively parallel multi-level
 * approach to a domain decomposition method for the optical flow estimation
 * with varying illumination".  The library solves the P1 finite-element
 * discretisation (Section 2.2) of the Euler-Lagrange system of functional
 * (BW2) (Section 1), Horn-Schunck regularisation with a per-element alpha and
 * the Gennert-Negahdaripour illumination unknown m, by additive Schwarz with
 * overlapping rectangular subdomains and Dirichlet transmission (Section 3.2,
 * equation (schwarz)), each subdomain solved directly by a block
 * factorisation of its banded matrix over the grid lines; alpha is adapted
 * with the residual indicator of Section 2.3.
 *
 * Conventions shared by every call:
 *   - W x H nodes, one per pixel centre; node (x, y), x = column, y = row.
 *   - Each pixel square (x,y)-(x+1,y+1) is cut by its (x,y)-(x+1,y+1)
 *     diagonal into T0 = {(x,y),(x+1,y),(x+1,y+1)} and T1 = {(x,y),(x+1,y+1),(x,y+1)}.
 *   - Frames I0, I1:    double [B][H][W], row-major.
 *   - alpha, eta:       double [B][H-1][W-1][2], last index T0/T1.
 *   - U, F, residuals:  double [B][3][H][W], field planes u1 (x-flow),
 *                       u2 (y-flow), m (illumination derivative m_t).
 *   - All array pointers are DEVICE pointers (HIP memory on the context's
 *     device) unless a parameter says "host".  The caller owns them; the
 *     library never frees or retains caller pointers past a call.
 *   - Work is enqueued on the stream given to sf_create.  Calls that return
 *     host scalars synchronise that stream before returning.
 *   - Return value: SF_OK (0), a negative error (nothing useful was
 *     computed) or a positive numerical status (outputs are written).
 *   - A context is not thread-safe; use one context per host thread/stream.
 */
#ifndef SFDD_H
#define SFDD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define SF_OK              0
#define SF_ERR_INVALID    (-1)  /* bad argument or configuration             */
#define SF_ERR_HIP        (-2)  /* a HIP runtime call failed                  */
#define SF_ERR_OOM        (-3)  /* device allocation failed                   */
#define SF_ERR_STATE      (-4)  /* calls out of order (e.g. solve before factor) */
#define SF_ERR_DEVICE     (-5)  /* a device-side wait gave up (see sf_error_detail) */
#define SF_NOT_SPD          1   /* a subdomain matrix is not positive definite */
#define SF_NOT_CONVERGED    2   /* max_sweeps reached above rtol; U is written */
#define SF_NONFINITE        3   /* NaN/Inf in the inputs or in a residual norm */

#define SF_SIGMA_MAX 16.0

/* factor_precision */
#define SF_FP64      0          /* subdomain factors stored and applied in FP64 */
#define SF_FP32      1          /* inverse Schur tiles computed in FP64, stored in
                                   FP32 and applied in FP64 arithmetic: an inexact
                                   local solve whose error the Schwarz iteration on
                                   FP64 residuals removes (iterative refinement);
                                   the iteration converges to the same solution  */
#define SF_FP32_FACTOR 2        /* the factorisation itself in FP32 arithmetic
                                   (FP32 MFMA), tiles stored in FP32 and applied
                                   in FP64 arithmetic as with SF_FP32; a
                                   subdomain whose FP32 factorisation meets a
                                   pivot <= pivot_tol x its diagonal entry of A
                                   is factored again in FP64 arithmetic         */

typedef struct sf_config {
    int32_t width;            /* W >= 2 nodes                                    */
    int32_t height;           /* H >= 2 nodes                                    */
    int32_t batch;            /* B >= 1 independent frame pairs                   */
    int32_t parts_x;          /* tiles across, 1 <= parts_x <= W                  */
    int32_t parts_y;          /* tiles down,   1 <= parts_y <= H                  */
    int32_t overlap;          /* delta >= 0: nodes shared by neighbouring boxes   */
    double  lambda;           /* regularisation of m (> 0), constant (Section 2.3) */
    double  sigma;            /* Gaussian presmoothing of the frames, 0 = off,
                                 at most SF_SIGMA_MAX (Section 1: f = K_sigma * I;
                                 sampled Gaussian |k| <= ceil(3 sigma), normalised,
                                 rows then columns, clamp to edge)              */
    int32_t factor_precision; /* SF_FP64 or SF_FP32                               */
    int32_t band_tile;        /* sweep workgroups per chain of a subdomain; 0 = auto */
    double  rho;              /* Gaussian K_rho of the data term (Section 1,
                                 functionals (BW), (BW2)): A_rho = K_rho * (a a^T),
                                 F = -K_rho * (a f_t); 0 = off, at most
                                 SF_SIGMA_MAX.  Read as the sampled normalised
                                 Gaussian (|k| <= ceil(3 rho)) over whole-pixel
                                 shifts of the element data, clamp to edge per
                                 axis, integrated exactly (rho = 0: the plain
                                 data term)                                     */
    double  pivot_tol;        /* SF_FP32_FACTOR: relative pivot threshold of the
                                 FP32 factorisation (0 = default 1e-5)          */
    int32_t deferred_status;  /* 0: sf_assemble and sf_factor_subdomains wait
                                 for the stream and return the input check and
                                 pivot status themselves.  1: they only enqueue
                                 (no host synchronisation, capturable in a HIP
                                 graph); that status is collected by the next
                                 call that reads the context's results (solve,
                                 residual, rhs, indicator, alpha update,
                                 adjoint) or by sf_sync, which returns it.  The
                                 FP64 refactorisation of SF_FP32_FACTOR
                                 subdomains with a rejected pivot runs there.  */
} sf_config;

typedef struct sf_context sf_context;

/* Create a context for one geometry (Section 3.1: tile (p,q) owns nodes
 * [floor(pW/Px), floor((p+1)W/Px)) x [floor(qH/Py), floor((q+1)H/Py));
 * its box extends every side interior to the image by floor(delta/2)
 * (left/top) or ceil(delta/2) (right/bottom) nodes).  `stream` is a
 * hipStream_t (NULL = default stream).  Allocates all device storage the
 * geometry needs (factors: about 4*m*(m+32) bytes per grid line of every
 * subdomain, m = 3 x the shorter box side).  On success *out owns it.       */
int sf_create(const sf_config* cfg, void* stream, sf_context** out);

/* Release everything the context owns (NULL is accepted). */
void sf_destroy(sf_context* ctx);

/* Section 1 and 2.2: copy I0, I1 and alpha into the context and build the
 * right-hand side F_i = -int f_t a phi_i, a = (f_x, f_y, -f), f = K_sigma * I0
 * (P1), f_t = K_sigma * (I1 - I0) (P1), integrated exactly (with rho > 0,
 * -int (K_rho * (f_t a)) phi_i, and the smoothed data term of A).  Returns SF_NONFINITE if a frame
 * value is not finite and SF_ERR_INVALID if an alpha is not finite or <= 0.
 * Makes previous factors stale.                                             */
int sf_assemble(sf_context* ctx, const double* I0, const double* I1, const double* alpha);

/* Wait for the context's stream and collect a status that sf_assemble or
 * sf_factor_subdomains left pending (deferred_status = 1): their return
 * value as it would have been without deferral (SF_OK if nothing pends).  */
int sf_sync(sf_context* ctx);

/* Bound every device-side wait of the context's later launches (the factor's
 * and the sweep's exchanges between workgroups) to `polls` unsuccessful polls
 * (default 2^20, about a second); a launch whose wait exceeds it stops every
 * workgroup and its call returns SF_ERR_DEVICE (sf_error_detail: subdomain).
 * After SF_ERR_DEVICE from the factorisation the context is back to
 * assembled; from a solve, U holds a partial update and the factors stay
 * usable.  polls < 0 gives SF_ERR_INVALID.                                  */
int sf_set_wait_limit(sf_context* ctx, int64_t polls);

/* Section 3.2, local problems: factor every subdomain matrix A_i = A[S_i,S_i]
 * (ordering: lines along the shorter box side, 3 unknowns per node, band
 * half-width 3*ms+5).  Block LDL^T over the lines: S_t = A_tt -
 * B_t S_{t-1}^{-1} B_t^T with S_0 = A_00; every S_t is inverted (SPD
 * pivots checked) and stored as S_t^{-1}.  Returns SF_NOT_SPD (with
 * sf_error_detail) if a pivot is not positive.                              */
int sf_factor_subdomains(sf_context* ctx);

/* Section 3.2, equation (schwarz), restricted additive form: from the
 * initial guess in U, repeat r = F - A U, relres = ||r||/||F|| (per pair);
 * stop a pair when relres <= rtol or after max_sweeps sweeps; otherwise
 * U[O_i] += (A_i^{-1} r[S_i])[O_i] for every subdomain i (O_i its owned
 * nodes).  U [B][3][H][W] is read and overwritten.  sweeps [B] and relres
 * [B] are HOST arrays (either may be NULL).  A pair with F = 0 gets
 * U = 0 after 0 sweeps.  Returns SF_NOT_CONVERGED if a pair stopped on
 * max_sweeps above rtol (U still written), SF_NONFINITE on a NaN norm.
 * A sweep or factor launch may take the device's whole co-resident
 * capacity, so the calls that run them (this one, sf_schwarz_solve_graph,
 * sf_autotune, sf_adjoint, sf_subdomain_solve, and sf_factor_subdomains
 * unless deferred_status = 1) hold a per-device lock of the process until
 * their streams have drained: those of different contexts on one device run
 * one at a time.  A deferred factorisation only enqueues and takes no lock:
 * order it before other contexts' work on the device with events.         */
int sf_schwarz_solve(sf_context* ctx, double* U, double rtol, int32_t max_sweeps,
                     int32_t* sweeps, double* relres);

/* sf_schwarz_solve with the launches of every 4 iterations (residual and
 * convergence test, sweep) replayed from one captured HIP graph: the same
 * kernels in the same order, so U, sweeps and relres equal those of
 * sf_schwarz_solve bit for bit.  The graph runs on a private stream of the
 * context (created on the first call: default priority, non-blocking) that
 * waits for the work queued on the context's stream, which in turn waits
 * for the graph's; the iteration index and the sweep's tag base live on the
 * device for the replays.  Iterations beyond the last whole chunk of 4 run
 * as ordinary launches.  Converged pairs make later replays' kernels exit at
 * once.  Arguments, outputs and return codes as sf_schwarz_solve; calls on
 * one context must not overlap.                                            */
int sf_schwarz_solve_graph(sf_context* ctx, double* U, double rtol, int32_t max_sweeps,
                           int32_t* sweeps, double* relres);

/* Autotuning of the sweep's launch shape: with current factors, time
 * `trials` RAS sweeps for every number of workgroups per chain that changes
 * the block rows each one owns (clamped to what fits co-resident), keep the
 * fastest and return it in *band_tile (HOST, may be NULL).  U [B][3][H][W]
 * (device) is the iterate of the timing sweeps and is overwritten.  A shape
 * only reorders the partial sums inside a row, so later solves agree with
 * earlier ones to rounding.  SF_ERR_STATE without current factors.         */
int sf_autotune(sf_context* ctx, double* U, int32_t trials, int32_t* band_tile);

/* Gradients of a loss L(U) of the discrete solution (Section 2.2, A U = F)
 * with respect to the frames and alpha, by the adjoint method.  The adjoint
 * state P solves A P = G, G = dL/dU (A is symmetric), with the same
 * factors and RAS iteration as sf_schwarz_solve (stop at
 * ||G - A P|| <= rtol ||G|| or max_sweeps; a pair with G = 0 gets P = 0).
 * Then, with p = a.P, e = a.U + f_t and a = (f_x, f_y, -f):
 *   dalpha_K = -|K| (grad P1.grad U1 + grad P2.grad U2)
 *   dI1_n    = -int p phi_n
 *   dI0_n    = -int (grad phi_n.(P1,P2) - phi_n P3) e
 *                   + p (grad phi_n.(U1,U2) - phi_n U3 - phi_n)
 * (the frame integrals by a degree-4 exact triangle rule).  U, G, P are
 * [B][3][H][W] device arrays; P holds the initial iterate on entry (zeros
 * are a fine start) and the adjoint state on return.  dI0, dI1 [B][H][W] and
 * dalpha [B][H-1][W-1][2] are device outputs, any may be NULL.  sweeps and
 * relres [B] are HOST arrays or NULL.  Needs current factors
 * (SF_ERR_STATE otherwise); SF_ERR_INVALID when the context presmooths
 * (sigma > 0) or smooths the data term (rho > 0).  Returns SF_NOT_CONVERGED (gradients still written) like
 * sf_schwarz_solve.                                                       */
int sf_adjoint(sf_context* ctx, const double* U, const double* G, double* P,
               double* dI0, double* dI1, double* dalpha,
               double rtol, int32_t max_sweeps, int32_t* sweeps, double* relres);

/* Section 2.3: residual indicator eta_K (flow components, alpha weights,
 * element residual + half the flux jumps) and the decrease rule
 * alpha <- max(alpha / (1 + kappa max(eta/||eta||_inf - eta_thr, 0)), alpha_th)
 * with ||eta||_inf per pair.  alpha [B][H-1][W-1][2] is overwritten with
 * the new values, which also replace the context's copy; factors become
 * stale (call sf_factor_subdomains before the next solve; F is unchanged).
 * eta_max [B] is a HOST array or NULL.                                     */
int sf_update_alpha(sf_context* ctx, const double* U, double* alpha,
                    double kappa, double eta_thr, double alpha_th, double* eta_max);

/* Detail of the last SF_NOT_SPD / SF_ERR_DEVICE status: pair, subdomain
 * index (row-major tile order within the pair) and local row.  Host outputs,
 * any may be NULL.  Returns the status it describes.                       */
int sf_error_detail(const sf_context* ctx, int32_t* pair, int32_t* subdomain, int64_t* row);

/* Static text for a status code. */
const char* sf_status_string(int status);

/* Static text: SHA-256 (hex) of the sources the library was built from (the
 * names and bytes of csrc/ and include/ files, sorted), so that a caller can
 * refuse a library built from other sources than it expects.               */
const char* sf_build_digest(void);

/* ---- diagnostics (same math, exposed for verification) ------------------ */

/* Copy F [B][3][H][W] (valid after sf_assemble) into `F`.                   */
int sf_rhs(sf_context* ctx, double* F);

/* r = F - A U for U [B][3][H][W]; rnorm2 [B] HOST (||r||^2) or NULL.       */
int sf_residual(sf_context* ctx, const double* U, double* r, double* rnorm2);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * r = F - A U and ||r||^2 as sf_residual (same kernels, equal bit for bit),
 * with the block partials and norms held in a static device array of the
 * library (SF_NOALLOC_SCRATCH_BYTES per device, kept until the process
 * ends) instead of context storage; the call allocates nothing.  The array
 * holds B * ceil(W H / 256) + B doubles of this context; larger contexts get
 * SF_ERR_INVALID.  rnorm2 [B] is HOST or NULL (NULL: no synchronisation).
 * All contexts on one device share the array: calls that overlap on one
 * device (other threads or streams) race.                                  */
#define SF_NOALLOC_SCRATCH_BYTES (1 << 20)
int sf_residual_noalloc(sf_context* ctx, const double* U, double* r, double* rnorm2);

/* eta_K of sf_update_alpha without changing alpha; eta [B][H-1][W-1][2].   */
int sf_indicator(sf_context* ctx, const double* U, double* eta);

/* Host-only: device memory (bytes) that sf_create would allocate for cfg
 * (factors, workspace and field arrays, not counting allocation rounding or
 * the small graph-replay buffers); *bytes is HOST.  It grows linearly with
 * cfg->batch, so a driver can split many pairs into waves that fit the
 * device (a batch of tens of full-HD pairs needs several times its HBM).   */
int sf_memory_bytes(const sf_config* cfg, int64_t* bytes);

/* Host-only geometry plan (no device needed): returns the number of
 * subdomains of `cfg` (or a negative error) and, if geom != NULL, fills
 * geom[10*i .. 10*i+9] (HOST) with pair, box x0, x1, y0, y1, owned x0, x1,
 * y0, y1 and the lines-are-columns flag of subdomain i (same order as the
 * context uses: pair-major, then row-major tiles).                          */
int sf_plan(const sf_config* cfg, int32_t* geom);

/* Kernel timing with HIP events recorded on the context stream around every
 * launch of the sweep, factor and residual kernels (off by default; adds
 * one event pair per launch).  ms[4] / launches[4] (HOST, may be NULL)
 * receive the totals so far for classes 0 sweep, 1 factor, 2 residual +
 * stop test, 3 other.  enable: 1 = reset and start, 0 = reset and stop,
 * -1 = only read.                                                          */
int sf_profile(sf_context* ctx, int32_t enable, double* ms, int64_t* launches);

/* Section 3.1: the split parts_x x parts_y = nparts of a width x height image
 * whose parts have the largest area / perimeter, with a part of
 * w = width / parts_x by h = height / parts_y pixels (real-valued) having area
 * w h and perimeter 2 (w + h); ties go to the larger parts_x.  Host-only, no
 * device needed.  Outputs (HOST, any may be NULL): parts_x, parts_y, ratio.
 * SF_ERR_INVALID if no split of at most one part per pixel column / row
 * exists.                                                                  */
int sf_choose_split(int32_t width, int32_t height, int32_t nparts, int32_t* parts_x, int32_t* parts_y,
                    double* ratio);

/* Number of subdomains over all pairs (B * parts_x * parts_y).             */
int sf_num_subdomains(const sf_context* ctx);

/* With SF_FP32_FACTOR: the number of subdomains that the last
 * sf_factor_subdomains factored again in FP64 arithmetic because their FP32
 * factorisation met a pivot below the threshold (0 otherwise).            */
int sf_factor_fallbacks(const sf_context* ctx);

/* geom[13] (HOST): pair, box x0, x1, y0, y1 (half-open), owned x0, x1, y0,
 * y1, lines-are-columns flag, sweep workgroups per chain, chains (1: lines
 * eliminated top to bottom; 2: from both ends towards the middle line) and
 * the middle line k (nt - 1 with one chain).                               */
int sf_subdomain_geometry(const sf_context* ctx, int32_t sub, int32_t* geom);

/* x = A_i^{-1} b for subdomain `sub` from its factors; b and x hold
 * 3*bw*bh doubles in the local ordering 3*(t*ms + s) + c (line t, position s
 * along the line, field c).  Device pointers, may not alias.               */
int sf_subdomain_solve(sf_context* ctx, int32_t sub, const double* b, double* x);

#ifdef __cplusplus
}
#endif
#endif /* SFDD_H */
