/*
 * fewha.h -- C ABI of libfewha, an MI355X (gfx950) implementation of the hot
 * path of FEWHA, the Finite Element Wavelet Hybrid Algorithm for atmospheric
 * tomography (Stadler & Ramlau, arXiv 2202.11945).
 *
 * The library solves, for every frame, the wavelet-domain MAP system
 * (eq. fewha / eq. M):
 *     M c = b,  M = W^{-T} A^T C_hat^{-1} A W^{-1} + alpha D,
 *               b = W^{-T} A^T C_hat^{-1} s,
 * with a fixed number of Jacobi-preconditioned CG iterations (eq. precond),
 * warm-started from the previous frame (Sec. 3.3, Algorithm 1, open loop),
 * and returns the layers W^{-1} c and the DM commands (F = I when the layers
 * sit at the DM altitudes, Sec. 4.1).
 *
 * Conventions shared by every call:
 *  - Sensor g has N_g x N_g subapertures of pitch d = D / N_g; its corners are
 *    x_j = -D/2 + j d (j = 0..N_g), row index i = y, column index j = x.
 *  - Slopes of sensor g: [s^x over its active subapertures in row-major
 *    order; s^y in the same order] (Sec. 2); sensors concatenated in the
 *    order given to fewha_set_wfs.  s^x, s^y are phase differences across a
 *    subaperture (rad), the average slope of the bilinear wavefront (Sec. 2).
 *  - Layer l: n_l x n_l nodes (n_l = 2^J_l, Sec. 3.1), row-major (rows = y),
 *    on a centred square domain of side L shared by all layers; the node
 *    spacing is delta_l = L / n_l.  Layers are concatenated in order.
 *  - Wavelet coefficients: periodic Daubechies-3, Mallat layout per layer,
 *    the same n_l x n_l footprint; W_l = delta_l W.
 *  - All float* compute arguments are DEVICE pointers owned by the caller;
 *    the library never frees them.  Compute calls are asynchronous on the
 *    context's stream (fewha_set_stream; default: the null stream).
 *  - Argument and state errors are returned before anything is enqueued.
 *    A device error is returned as FEWHA_EDEVICE by the call that sees it.
 *    No C++ exception crosses this interface.
 *  - Numerical breakdown: M is symmetric positive definite (Sec. 3.1), so a
 *    PCG step meets p^T M p <= 0 with a nonzero residual, or a non-finite or
 *    negative inner product, only on non-finite or overflowing inputs.  The
 *    step then leaves its iterate unchanged (alpha = 0; a zero residual with
 *    p = 0 is exact convergence, not a breakdown) and sets a flag of the
 *    context (or batch); the next compute call on it, once that work has
 *    finished, returns FEWHA_ENUMERIC without enqueuing anything and clears
 *    the flag: results of the earlier calls are not valid.
 *  - A context is not thread-safe; distinct contexts may be used from
 *    distinct threads.
 */
#ifndef FEWHA_H
#define FEWHA_H

#ifdef __cplusplus
extern "C" {
#endif

#define FEWHA_API __attribute__((visibility("default")))

typedef struct fewha_ctx fewha_ctx;
typedef struct fewha_batch fewha_batch;

typedef enum {
  FEWHA_OK = 0,
  FEWHA_EINVAL = -1,   /* bad argument (null pointer, size, range)          */
  FEWHA_ENOMEM = -2,   /* host or device allocation failed                  */
  FEWHA_EDEVICE = -3,  /* HIP runtime error                                 */
  FEWHA_ESTATE = -4,   /* call not valid in the context's current state     */
  FEWHA_EGEOM = -5,    /* geometry rejected (footprint leaves a layer, ...)  */
  FEWHA_ENUMERIC = -6  /* numerical breakdown in earlier work (see below)    */
} fewha_status;

enum { FEWHA_NGS = 0, FEWHA_LGS = 1 };

/* One Shack-Hartmann wavefront sensor and its guide star (Sec. 2, Table 4). */
typedef struct {
  int kind;            /* FEWHA_NGS or FEWHA_LGS                                   */
  int n_subap;         /* N: N x N subapertures, (N+1)^2 corners; 1..4096          */
  double theta_x;      /* guide-star direction (rad)                               */
  double theta_y;
  double H;            /* LGS altitude (m), > every layer altitude; NGS: ignored   */
  double sigma;        /* slope noise std (rad): C_g = sigma^2 I (eq. NGS-noise)   */
  double launch_x;     /* LGS laser launch position in the pupil (m), used for the */
  double launch_y;     /*   spot elongation of eq. (LGS-noise)                     */
  int tt_removal;      /* LGS: 1 = C_hat_g^{-1} = (I-T) C_g^{-1} (I-T) (Sec. 3.2)  */
  const unsigned char* mask; /* host N*N row-major active flags, or NULL for the
                                annulus rule: active iff the subaperture centre
                                lies in [sqrt(obstruction) D/2, D/2]. Copied.     */
} fewha_wfs_desc;

/* One reconstruction layer (Sec. 2 layered model, Table 2). */
typedef struct {
  double h;            /* altitude (m), >= 0                                       */
  int n;               /* grid side, power of two, 8..2048                         */
  int levels;          /* wavelet decomposition depth; n >> levels in [1, 128]     */
  double cn2;          /* fractional turbulence weight gamma_l (> 0)               */
} fewha_layer_desc;

/* One deformable mirror for the fitting step (Sec. 4.1, Table 3); see fewha_set_fitting. */
typedef struct {
  double h;            /* conjugation altitude (m)                                 */
  int n_act;           /* n_act x n_act actuators, bilinear influence              */
  double pitch;        /* actuator spacing (m); the grid is centred on the axis    */
} fewha_dm_desc;

/* ---- context set-up (host only; no device work until fewha_finalize) ---- */

/* Create a context for HIP device `device`, or a host-only context when
 * device < 0 (set-up and table queries only; compute calls then return
 * FEWHA_ESTATE).  *out receives the context; FEWHA_EDEVICE if the device
 * cannot be selected. */
FEWHA_API fewha_status fewha_create(fewha_ctx** out, int device);

/* Stream (a hipStream_t passed as void*) on which compute calls enqueue. */
FEWHA_API fewha_status fewha_set_stream(fewha_ctx* ctx, void* hip_stream);

/* Telescope diameter D (m) and obstructed area fraction in [0, 1). */
FEWHA_API fewha_status fewha_set_pupil(fewha_ctx* ctx, double D, double obstruction);

/* G >= 1 sensors, copied. Sec. 2: A = [Gamma_g P_g]. */
FEWHA_API fewha_status fewha_set_wfs(fewha_ctx* ctx, int G, const fewha_wfs_desc* wfs);

/* L >= 1 layers on a common square domain of side domain_side (m). */
FEWHA_API fewha_status fewha_set_layers(fewha_ctx* ctx, int L, const fewha_layer_desc* layers,
                                        double domain_side);

/* Prior and preconditioner (eq. fewha, eq. precond): regularisation weight
 * alpha > 0; Fried parameter r0 (m) and outer scale L0 (m) of the diagonal
 * prior D; preconditioner threshold tau >= 0 (J = diag(data) + alpha max(D, tau)).
 * D, per coefficient at level block size 2^j, is the inverse of the von Karman
 * spectrum 0.023 gamma_l r0^{-5/3} ((2^j/L)^2 + L0^{-2})^{-11/6}. */
FEWHA_API fewha_status fewha_set_prior(fewha_ctx* ctx, double alpha, double r0, double L0, double tau);

/* LGS spot elongation (eq. LGS-noise): alpha_eta >= 0 (0 = no elongation),
 * sodium-layer FWHM (m), non-elongated spot FWHM f (rad, > 0). */
FEWHA_API fewha_status fewha_set_noise(fewha_ctx* ctx, double alpha_eta, double na_fwhm, double spot_fwhm);

/* Gain of Algorithm 1's control lines, in [0, 1]: open loop
 * a <- (1-gain) a + gain a~; closed loop (fewha_set_loop) see there. */
FEWHA_API fewha_status fewha_set_control(fewha_ctx* ctx, double gain);

/* Open (closed = 0, the default) or closed loop (closed = 1), Algorithm 1.
 * Closed loop, with the two-step delay: the slopes passed to a frame were
 * measured with the commands a^(i-1) (the state's a_prev) on the mirrors,
 * so the frame reconstructs from the pseudo-open-loop slopes
 * s + Gamma a^(i-1), Gamma being the mirrors' slope response (A, since with
 * F = I the mirrors are the reconstruction layers), and applies
 * a^(i+1) = a^(i) + gain (a~ - a^(i-1)).  F = I only: FEWHA_EINVAL at
 * fewha_finalize with fewha_set_fitting. */
FEWHA_API fewha_status fewha_set_loop(fewha_ctx* ctx, int closed);

/* Augmented PCG (Sec. 3.3; Algorithm 1's augPCG line): every frame's PCG
 * reuses the previous frame's first `keep` search directions W = P^(i) and
 * their images A W = Q^(i) = M P^(i) (keep in [0, 4]; 0 = plain PCG, the
 * default).  The paper defines the method by reference to another paper;
 * this is the deflated CG of Saad, Yeung, Erhel & Guyomarc'h (2000) with
 * the Jacobi preconditioner: the warm-start iterate and residual are
 * projected so that W^T r_0 = 0 (x_0 = c + W G^{-1} W^T r_0,
 * r_0 <- r_0 - A W G^{-1} W^T r_0, G = W^T A W), and each direction is
 * p_j = J^{-1} r_j + beta p_{j-1} - W G^{-1} (A W)^T J^{-1} r_j.  G is
 * factored by Cholesky in double precision; a direction with a non-positive
 * pivot is dropped.  The state grows by 2 keep N_c + 4 floats: after
 * [c | b | r | a_prev | a] come the keep directions, their images and the
 * count of valid ones (an all-zero state has none: the first frame is the
 * plain PCG).  Not available in fewha_reconstruct_noalloc. */
FEWHA_API fewha_status fewha_set_augmentation(fewha_ctx* ctx, int keep);

/* Noise level from photon counts (eq. NGS-noise, eq. LGS-noise): sigma_g^2 =
 * 1 / n_photons[g], the photons per subaperture and frame of sensor g (> 0),
 * replacing the sigma of fewha_set_wfs (call after it; G = its count). */
FEWHA_API fewha_status fewha_set_photons(fewha_ctx* ctx, int G, const double* n_photons);

/* DM fitting (Sec. 4.1: with the layers away from the DM altitudes, fitting
 * the mirrors is an additional minimisation problem).  The commands a (the
 * concatenated n_act x n_act grids of the n_dm DMs, bilinear influence,
 * centred actuator grids) minimise
 *     sum_k |M (B_k a - P_k phi)|^2 + eps |a|^2,
 * phi = W^{-1} c the reconstructed layers, over n_dirs directions
 * dirs_xy[2k], dirs_xy[2k+1] (rad); P_k, B_k propagate layers and DMs to the
 * corners of an n_fit x n_fit subaperture grid on the pupil (no cone effect),
 * M keeps the corners of its active subapertures (the pupil's annulus rule);
 * eps = eps_rel * mean(diag(sum_k B_k^T M B_k)).  Solved by fit_iters CG
 * iterations from a = 0 after every reconstruction; the control update of
 * Algorithm 1 then uses the fitted commands.  Without this call F = I (DM
 * commands = layers).  FEWHA_EGEOM at finalize if a direction leaves a DM. */
FEWHA_API fewha_status fewha_set_fitting(fewha_ctx* ctx, int n_dm, const fewha_dm_desc* dms, int n_dirs,
                                         const double* dirs_xy, int n_fit, int fit_iters, double eps_rel);

/* Validate the geometry and build every table: sensor masks, bilinear
 * propagation tables, the prior D and the exact Jacobi diagonal J
 * (eq. precond).  On a device context, upload the tables and allocate the
 * device work space.  FEWHA_EGEOM if a sensor footprint leaves a layer
 * (no periodic wrap in P) or a size is unsupported. */
FEWHA_API fewha_status fewha_finalize(fewha_ctx* ctx);

/* Sizes after finalize (any pointer may be NULL):
 *   n_coeff     = N_c = sum_l n_l^2 (wavelet coefficients = layer nodes)
 *   n_slopes    = sum_g 2 |M_g|
 *   n_layer_pts = N_c
 *   n_act       = number of DM commands (= N_c when F = I, else sum of n_act^2)
 *   n_state     = 3 N_c + 2 n_act (layout of the reconstruct state below),
 *                 plus 2 keep N_c + 4 with fewha_set_augmentation. */
FEWHA_API fewha_status fewha_sizes(const fewha_ctx* ctx, long* n_coeff, long* n_slopes,
                                   long* n_layer_pts, long* n_act, long* n_state);

/* Host copies of set-up tables, for inspection and tests (after finalize):
 *   FEWHA_TABLE_FILTER  : the 6 db3 lowpass taps                      (6)
 *   FEWHA_TABLE_PRIOR   : D per coefficient                           (N_c)
 *   FEWHA_TABLE_PRECOND : J per coefficient (eq. precond)             (N_c)
 *   FEWHA_TABLE_MASK    : active flags of every sensor, concatenated  (sum N_g^2)
 * `n` is the capacity of `out` (host); FEWHA_EINVAL if too small. */
enum { FEWHA_TABLE_FILTER = 0, FEWHA_TABLE_PRIOR = 1, FEWHA_TABLE_PRECOND = 2, FEWHA_TABLE_MASK = 3 };
FEWHA_API fewha_status fewha_get_table(const fewha_ctx* ctx, int which, double* out, long n);

/* ---- compute (device pointers, asynchronous on the context stream) ---- */

/* slopes = A phi (eq. atmo, s_g = Gamma_g P_g phi): layers (N_c floats, FE
 * domain) -> slopes (n_slopes floats). */
FEWHA_API fewha_status fewha_apply_A(fewha_ctx* ctx, const float* layers, float* slopes);

/* layers = A^T slopes (plain transpose, no noise weighting). */
FEWHA_API fewha_status fewha_apply_AT(fewha_ctx* ctx, const float* slopes, float* layers);

/* Mc = M c (eq. M), wavelet domain, N_c floats each. */
FEWHA_API fewha_status fewha_apply_M(fewha_ctx* ctx, const float* c, float* Mc);

/* b = W^{-T} A^T C_hat^{-1} s (right-hand side of eq. fewha). */
FEWHA_API fewha_status fewha_rhs(fewha_ctx* ctx, const float* slopes, float* b);

/* One time step of Algorithm 1 (open loop, F = I, plain warm restart):
 *   b' = rhs(slopes); r0 = (b' - b) + r; c <- PCG(c, r0, J, iters);
 *   phi = W^{-1} c; a_prev <- a; a <- (1-gain) a + gain phi.
 * state (in/out, n_state floats, 16-byte aligned) = [c | b | r | a_prev | a]; an all-zero
 * state starts a sequence (c = 0, r0 = b').  layers_out (N_c) and dm_out
 * (n_act) may be NULL.  iters in [0, 256].  With fewha_set_fitting the DM
 * commands are the fitted ones instead of phi.  PCG inner products and the
 * alpha/beta recurrences are computed in double precision. */
FEWHA_API fewha_status fewha_reconstruct(fewha_ctx* ctx, const float* slopes, float* state,
                                         float* layers_out, float* dm_out, int iters);

/* Restart from the true residual every `every` frames (0 = never, the
 * default): frame f (counted from 0 by the context's calls to
 * fewha_reconstruct / fewha_reconstruct_streamed) with f > 0 and f a
 * multiple of `every` takes r0 = b' - M c instead of Algorithm 1's
 * recurrence r0 = (b' - b) + r, which equals it in exact arithmetic but
 * accumulates rounding over a long sequence; it costs one more application
 * of M.  fewha_set_frame_count sets the count (e.g. when a sequence resumes
 * from a saved state in a new context). */
FEWHA_API fewha_status fewha_set_refresh(fewha_ctx* ctx, int every);
FEWHA_API fewha_status fewha_set_frame_count(fewha_ctx* ctx, long frames);

/* fewha_reconstruct for slopes in HOST memory that arrive sensor group by
 * sensor group (pipelining, Sec. 4.3): the sensors are split into `chunks`
 * contiguous groups (1 <= chunks <= min(G, 64)); each group's slopes are
 * copied to the device on a copy stream of the context, and the frame takes
 * in each group (slope buffer, tip/tilt partial sums) as soon as its copy is
 * done.  In closed loop the mirrors' part of the pseudo-open-loop slopes,
 * Gamma a^(i-1), needs no measurement and runs while the copies are in
 * flight.  Results are bitwise those of fewha_reconstruct on the same
 * slopes in device memory.  host_slopes (n_slopes floats; pinned memory
 * lets the copies run asynchronously) must stay valid and unchanged until
 * the frame's work on the context stream has completed. */
FEWHA_API fewha_status fewha_reconstruct_streamed(fewha_ctx* ctx, const float* host_slopes, float* state,
                                                  float* layers_out, float* dm_out, int iters, int chunks);

/* fewha_reconstruct without any allocation in the call, for callers that
 * cannot allocate device memory: code under HIP graph capture, tight
 * real-time serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * kernels and results (bitwise) as fewha_reconstruct; the frame's work
 * buffers (layers, adjoint, slopes, corner grids, search directions,
 * M p, inner-product slots) and the per-call pointer table live in one
 * static device array of the library (16 MiB, one copy per device, held
 * until the process ends) instead of the context's work space.  The call
 * makes no device or host allocation.  Every call on a device shares that
 * array, which keeps the last call's contents (every buffer is written
 * before it is read within a frame, so nothing needs clearing): calls that
 * overlap on one device (other streams, other threads, other contexts) race
 * and must be ordered by the caller.  FEWHA_EINVAL if the context's frame
 * needs more than 16 MiB of work buffers (about 2.9 MB for the 39 m
 * MAORY-like system, 8.6 MB for 9 layers of up to 256 x 256) or uses the
 * DM fitting step, augmentation or the true-residual restart. */
FEWHA_API fewha_status fewha_reconstruct_noalloc(fewha_ctx* ctx, const float* slopes, float* state,
                                                 float* layers_out, float* dm_out, int iters);

/* ---- converged solves and the implicit backward ---- */

/* Solve M x = rhs (eq. fewha, wavelet domain) to a relative residual
 * ||rhs - M x||_2 / ||rhs||_2 <= rtol.  Mixed-precision iterative refinement:
 * x = 0, then sweeps of { r = rhs - M x evaluated in double precision;
 * M d = r by the preconditioned CG of Algorithm 1 in FP32 (run to a
 * reduction of its J^{-1}-weighted residual, checked every 16 iterations);
 * x += d }, the iterate accumulated in double precision and rounded to float
 * once at the end.  The preconditioner is Jacobi plus a coarse-level
 * correction (fewha_set_solve_coarse).  rhs and x: N_c floats, device.
 * max_iters in [0, 2^24] bounds the total CG iterations; iters_done and
 * rel_res (host, may be NULL) receive that total and the final residual
 * ratio of the double-precision iterate (the sweeps also stop when one no
 * longer halves it).  Synchronizes the context stream after every sweep and
 * CG check.  A zero rhs returns x = 0 after 0 iterations.  FEWHA_ESTATE on a
 * context with augmentation (fewha_set_augmentation). */
FEWHA_API fewha_status fewha_solve(fewha_ctx* ctx, const float* rhs, float* x, int max_iters,
                                   double rtol, int* iters_done, double* rel_res);

/* Preconditioner of the converged solves (fewha_solve, fewha_solve_map and
 * their batched forms; the frame path keeps Algorithm 1's Jacobi PCG):
 *   z = J^{-1} r + Z E^{-1} Z^T r,   E = Z^T M Z,
 * with Z selecting the top-left side x side block of every layer's Mallat
 * coefficients (the coarsest levels; side halved until a problem has at
 * most 1024 such unknowns).  side: 0 (Jacobi only) or a power of two up to
 * 64; default 16.  The first solve after a change builds E with one
 * application of M per coarse unknown (the instances of one context in a
 * batch share the work) and inverts it on the host in double precision; a
 * system whose E is not positive definite keeps Jacobi.  It allocates
 * device memory of about 4 m^2 bytes per distinct system plus 4 N_c bytes
 * per problem (m = coarse unknowns). */
FEWHA_API fewha_status fewha_set_solve_coarse(fewha_ctx* ctx, int side);

/* As fewha_solve for rhs = W^{-T} A^T C_hat^{-1} slopes + W^{-T} g_layers
 * (either may be NULL): the MAP solution of eq. fewha for given slopes
 * (g_layers = NULL), or the adjoint solve M lambda = W^{-T} dL/dphi
 * (slopes = NULL).  The right-hand side is formed inside the double-precision
 * residual, never rounded to float.  slopes: n_slopes floats, g_layers: N_c
 * floats, x: N_c floats, all device. */
FEWHA_API fewha_status fewha_solve_map(fewha_ctx* ctx, const float* slopes, const float* g_layers,
                                       float* x, int max_iters, double rtol, int* iters_done,
                                       double* rel_res);

/* layers = W^{-1} coef = delta_l^{-1} W_l^T coef_l for every layer (Sec. 3.1:
 * W orthogonal, so W^{-1} = delta^{-1} W^T).  N_c floats each, device. */
FEWHA_API fewha_status fewha_apply_Winv(fewha_ctx* ctx, const float* coef, float* layers);

/* coef = W^{-T} layers = delta_l^{-1} W_l layers_l (the adjoint of
 * fewha_apply_Winv).  N_c floats each, device. */
FEWHA_API fewha_status fewha_apply_WinvT(fewha_ctx* ctx, const float* layers, float* coef);

/* Parameter gradients of a loss L(phi) of the reconstructed layers
 * phi = W^{-1} c*, c* = M^{-1} b(s) the exact solution of eq. fewha, through
 * the implicit-function theorem.  Inputs (device): slopes s (n_slopes
 * floats), coef = c* (N_c), lam = lambda = M^{-1} W^{-T} dL/dphi (N_c, the
 * adjoint solve; M is symmetric).  Output (device, 1 + 2L doubles):
 *   grads[0]       = dL/dalpha   = -lambda^T D c*
 *   grads[1 + l]   = dL/dgamma_l =  alpha lambda_l^T D_l c*_l / gamma_l
 *   grads[1 + L + l] = dL/dh_l   =  <dA_l W^{-1} lambda, C_hat^{-1}(s - A phi)>
 *                                 - <C_hat^{-1} A W^{-1} lambda, dA_l phi>
 * with dA_l = dA/dh_l (propagation P_g of Sec. 2, LGS cone factor 1 - h/H,
 * differentiated in h; on a grid line the average of the two one-sided
 * derivatives) and D the diagonal prior (Sec. 3.1), scaling as 1/gamma_l.
 * Only the dependence through c* is included: a loss that itself depends on
 * the heights adds its own explicit term.  FEWHA_EGEOM when a derivative
 * stencil would leave its layer.  Inner products are accumulated in double
 * precision and summed in a fixed order (deterministic). */
FEWHA_API fewha_status fewha_param_grads(fewha_ctx* ctx, const float* slopes, const float* coef,
                                         const float* lam, double* grads);

/* ---- batches: many independent problems per launch ---- */

/* Group n finalized device contexts (same device; geometries may differ)
 * into a batch whose every stage is one launch over all problems.  The
 * contexts must outlive the batch. */
FEWHA_API fewha_status fewha_batch_create(fewha_batch** out, fewha_ctx* const* ctxs, int n);
FEWHA_API fewha_status fewha_batch_set_stream(fewha_batch* b, void* hip_stream);

/* fewha_reconstruct for every problem k with slopes[k], state[k],
 * layers_out[k], dm_out[k] (host arrays of device pointers; the last two
 * may be NULL or hold NULLs).  use_graph = 1 replays a HIP graph of the
 * whole step (captured on first use for this iteration count). */
FEWHA_API fewha_status fewha_batch_reconstruct(fewha_batch* b, const float* const* slopes,
                                               float* const* state, float* const* layers_out,
                                               float* const* dm_out, int iters, int use_graph);

/* The true-residual restart schedule of a batch (as fewha_set_refresh, one
 * count for the batch's calls to fewha_batch_reconstruct). */
FEWHA_API fewha_status fewha_batch_set_refresh(fewha_batch* b, int every);
FEWHA_API fewha_status fewha_batch_set_frame_count(fewha_batch* b, long frames);
/* The converged solves' preconditioner of a batch (as fewha_set_solve_coarse). */
FEWHA_API fewha_status fewha_batch_set_solve_coarse(fewha_batch* b, int side);

/* Batched forms of the calls above: one entry of each host array of device
 * pointers per problem (same layouts and rules).  The batched solves iterate
 * until every problem meets rtol (the worst ratio in rel_res); in
 * fewha_batch_solve_map either array may be NULL. */
FEWHA_API fewha_status fewha_batch_solve(fewha_batch* b, const float* const* rhs, float* const* x,
                                         int max_iters, double rtol, int* iters_done,
                                         double* rel_res);
FEWHA_API fewha_status fewha_batch_solve_map(fewha_batch* b, const float* const* slopes,
                                             const float* const* g_layers, float* const* x,
                                             int max_iters, double rtol, int* iters_done,
                                             double* rel_res);
FEWHA_API fewha_status fewha_batch_apply_Winv(fewha_batch* b, const float* const* coef,
                                              float* const* layers);
FEWHA_API fewha_status fewha_batch_apply_WinvT(fewha_batch* b, const float* const* layers,
                                               float* const* coef);
FEWHA_API fewha_status fewha_batch_param_grads(fewha_batch* b, const float* const* slopes,
                                               const float* const* coef, const float* const* lam,
                                               double* const* grads);

/* Stage identifiers for fewha_batch_time_stage. */
enum {
  FEWHA_STAGE_IDWT_RES = 0, FEWHA_STAGE_IDWT_GLOB = 1, FEWHA_STAGE_P_GAMMA = 2,
  FEWHA_STAGE_GAMMA_T = 3, FEWHA_STAGE_P_T = 4, FEWHA_STAGE_FDWT_GLOB = 5,
  FEWHA_STAGE_FDWT_RES = 6, FEWHA_STAGE_UPDATE = 7, FEWHA_STAGE_COUNT = 8
};

/* Average device time (microseconds) of `reps` back-to-back launches of one
 * PCG-iteration stage over the whole batch, measured with HIP events on the
 * batch stream, in the launch configuration used by batch_reconstruct.
 * Must follow at least one fewha_batch_reconstruct (uses its buffers).
 * Also returns the stage's launch geometry (workgroups). */
FEWHA_API fewha_status fewha_batch_time_stage(fewha_batch* b, int stage, int reps, double* avg_us,
                                              long* workgroups);

FEWHA_API void fewha_batch_destroy(fewha_batch* b);

/* ---- tuning: launch shapes chosen per plan (by an autotuner or by hand) ---- */

/* dwt_resident: side of the largest transform block kept in one workgroup's
 * LDS by the resident DWT kernels (32, 64 or 128; 0 = default 128).  Levels
 * above it run as tiled passes over global memory, one launch per level.
 * Smaller values trade LDS work per workgroup for more workgroups and more
 * launches.  It must be at least every layer's coarsest block (n >> levels),
 * else FEWHA_EINVAL when the plan is built.
 * pt_rows: node rows per thread of the propagation adjoint P^T (4 or 8;
 * 0 = default 4); a tile is 64 node columns by 4 * pt_rows rows.  More rows
 * put more independent loads in flight per thread, at more registers.
 * streams: batches only (a context takes 0 or 1).  fewha_batch_reconstruct
 * runs the batch as this many contiguous parts of its problem list (1 to 4,
 * at most the number of problems; 0 = default 1), each part on a stream of
 * the library's own, forked from and joined back to the batch's stream by
 * events, so that the stages of one part overlap those of another.  Results
 * are identical to one part.  The parts' plans are built with the batch and
 * take device memory of their own (about that of the batch plan).  Every
 * other batch call runs the whole batch on the batch's stream.
 * res_split: the resident inverse levels run as one workgroup per (problem,
 * layer) (0 = default, or 1) or as four (4), each synthesizing the levels
 * below the top one itself and the top level for one quadrant of the
 * output, so that a launch spreads over more compute units; 4 needs every
 * layer's resident side to be at least 16 with at least one resident level
 * (else FEWHA_EINVAL when the plan is built).
 * pt_split: 1 = the propagation adjoint's tiles are 4 node rows x 64
 * columns and each tile's sensor list is split over its 4 waves (sensor i
 * to wave i mod 4, the partial sums added in a fixed order), a quarter of
 * the serial chain of sensors per wave; for launches with few tiles, such
 * as one problem's frame.  Needs pt_rows 0 or 4.  0 = default (off).
 * glob_fuse: 1 = a layer with two or more global levels (side above twice
 * dwt_resident) runs its last two inverse levels in one launch: each output
 * tile synthesizes the part of the inner level it needs itself (about 27 %
 * more inner-level work, one launch fewer per inverse transform).  0 =
 * default (off).
 * reserved: zero. */
typedef struct {
  int dwt_resident;
  int pt_rows;
  int streams;
  int res_split;
  int pt_split;
  int glob_fuse;
  int reserved[2];
} fewha_tuning;

/* Tuning of a context's own plan; before fewha_finalize. */
FEWHA_API fewha_status fewha_set_tuning(fewha_ctx* ctx, const fewha_tuning* t);

/* fewha_batch_create with the batch plan's tuning (NULL = defaults). */
FEWHA_API fewha_status fewha_batch_create_tuned(fewha_batch** out, fewha_ctx* const* ctxs, int n,
                                                const fewha_tuning* t);

/* Last error message of a context (never NULL). */
FEWHA_API const char* fewha_last_error(const fewha_ctx* ctx);
FEWHA_API const char* fewha_batch_last_error(const fewha_batch* b);

FEWHA_API void fewha_destroy(fewha_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* FEWHA_H */
