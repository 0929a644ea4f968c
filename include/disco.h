/*
 * disco.h — C ABI of the MI355X (gfx950) library for the dense registration objective
 * of Ruehaak et al., "Estimation of Large Motion in Lung CT by Integrating Regularized
 * Keypoint Correspondences into Dense Deformable Registration" (arXiv 1807.00467).
 *
 * The library evaluates the joint objective of eq. 11 without the lung-boundary term,
 *     J(u) = D(u) + alpha S(u) + gamma Vhat(u) + delta K(u),
 * its gradient with respect to the control-grid displacement u, and matrix-free
 * Gauss-Newton products, and runs one Gauss-Newton step (Jacobi-preconditioned CG plus
 * Armijo backtracking).  The paper obtains the same quantities with matrix-free
 * derivative rules (Sec. II-D, II-D3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Volumes have N = (Nx, Ny, Nz) voxels (x fastest) of spacing h = (hx, hy, hz) mm and
 *   are float32 arrays [Nz][Ny][Nx].  Voxel (i,j,k) has its centre at ((i+1/2)hx, ...).
 * - The deformation is y(x) = x + u(x), u trilinear (first-order B-spline) on a node
 *   grid with 4 voxels per cell and axis (Sec. II-D1, II-D3): n_a = N_a/4 + 1 nodes per
 *   axis at p * 4 h_a.  Every N_a must be a positive multiple of 4.
 * - Node fields (u, v, gradients, diagonals, Hv) are float32 SoA [3][nz][ny][nx]
 *   (component x, then y, then z), in mm (or the matching derived unit).
 * - All array arguments are DEVICE pointers on the context's device, owned by the
 *   caller, 4-byte aligned, not aliased with each other unless stated, and must stay
 *   valid until the work queued on the stream has finished.  Exceptions (host
 *   pointers) are stated per call.
 * - Scalar results (double, int32_t) are written to DEVICE memory so that calls can be
 *   recorded in a HIP graph; nothing synchronises the stream unless stated.
 * - `stream` is a hipStream_t (NULL = the null stream).  One context per stream at a
 *   time; a context is not thread safe.
 * - Return value: DISCO_OK or a negative error code detected on the host before any
 *   work is queued (nothing is written then), or DISCO_ERR_HIP - hipError_t when a HIP
 *   call failed.  Numerical outcomes (fold, CG breakdown, line-search failure) are
 *   reported through device status words, never through the return value.
 */
#ifndef DISCO_H
#define DISCO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* host-detected errors */
#define DISCO_OK 0
#define DISCO_ERR_ARG (-1)       /* null pointer, bad enum, bad count */
#define DISCO_ERR_SHAPE (-2)     /* N_a not a positive multiple of 4, keypoint outside the box, misaligned pointer */
#define DISCO_ERR_STATE (-3)     /* images not set, or ngf_hessvec / gn_hessvec before a linearisation */
#define DISCO_ERR_NONFINITE (-4) /* a scalar parameter is NaN/inf or out of its range */
#define DISCO_ERR_NOMEM (-5)     /* device allocation failed */
#define DISCO_ERR_LIMIT (-6)     /* input larger than the static scratch of the no-allocation entry point */
#define DISCO_ERR_HIP (-100)     /* returned as DISCO_ERR_HIP - (int)hipError_t */

/* numerical status bits (device int32 status words) */
#define DISCO_STATUS_FOLD 1          /* some coefficient d of eq. 8 is <= 0: Vhat = +inf (eq. 9) */
#define DISCO_STATUS_PCG_BREAKDOWN 2 /* p^T H p <= 0 in the CG solve */
#define DISCO_STATUS_LS_FAIL 4       /* no Armijo step accepted within ls_max trials */

/* storage of the image-gradient volumes and of the per-voxel GN vectors */
#define DISCO_STORAGE_FP32 0
#define DISCO_STORAGE_FP16 1 /* half precision with a per-volume power-of-two scale */

/* gn_pcg_step flags */
#define DISCO_FLAG_LS_DEVICE 1 /* line search fully on the device (fixed ls_max trials, graph capturable) */

/* which buffer disco_copy_buffer copies */
#define DISCO_BUF_GRAD_R 0 /* grad R, float32 [Nz][Ny][Nx][3] */
#define DISCO_BUF_GRAD_T 1 /* grad T, float32 [Nz][Ny][Nx][3] */
#define DISCO_BUF_SCACHE 2 /* s_v of the last linearisation, float32 [Nz][Ny][Nx][3] */

/* slots of the report written by gn_pcg_step (doubles) */
#define DISCO_REP_J 0        /* J(u) at the start of the step */
#define DISCO_REP_D 1
#define DISCO_REP_S 2
#define DISCO_REP_V 3
#define DISCO_REP_K 4
#define DISCO_REP_GNORM 5    /* |grad J(u)| */
#define DISCO_REP_T 6        /* accepted step length (0 if none) */
#define DISCO_REP_PCG_ITERS 7
#define DISCO_REP_PCG_RES 8  /* final CG residual norm */
#define DISCO_REP_GTP 9      /* g^T p */
#define DISCO_REP_J_NEW 10   /* J at the accepted point (or last trial) */
#define DISCO_REP_D_NEW 11
#define DISCO_REP_S_NEW 12
#define DISCO_REP_V_NEW 13
#define DISCO_REP_K_NEW 14
#define DISCO_REP_LS_TRIALS 15
#define DISCO_REP_B 16       /* lung-boundary term B(u) (eq. 6; 0 without masks) */
#define DISCO_REP_B_NEW 17
#define DISCO_REP_SIZE 18

typedef struct {
    int32_t n[3]; /* voxels Nx, Ny, Nz (multiples of 4) */
    double h[3];  /* spacing in mm */
} disco_geom;

typedef struct {
    double eta;       /* NGF edge parameter (eq. 1), HU/mm, > 0 */
    double alpha;     /* curvature weight (eq. 11), >= 0 */
    double gamma;     /* volume-change weight (eq. 11), >= 0 */
    double delta;     /* keypoint weight (eq. 11), >= 0 */
    double tau;       /* optional damping tau I added to the GN matrix, >= 0 */
    double armijo_c1; /* Armijo constant, in (0, 1) */
    double pcg_tol;   /* stop CG when |r| <= pcg_tol |g| (0: run pcg_iters) */
    int32_t pcg_iters; /* CG iterations, >= 1 */
    int32_t ls_max;    /* maximum number of line-search trials (t = 1, 1/2, ...), >= 1 */
    int32_t flags;     /* DISCO_FLAG_* */
    double beta;       /* lung-boundary weight (eq. 6, eq. 11), >= 0; used only with masks set */
} disco_params;

/* L-BFGS settings (Sec. II-D3) */
typedef struct {
    double tau;       /* H0 = alpha C_H L^T L + tau I, > 0 */
    double curv_eps;  /* a pair (s, y) is used only if s^T y > curv_eps |s| |y|, >= 0 */
    double h0_tol;    /* stop the H0 solve at |r| <= h0_tol |q| (0: run h0_iters), >= 0 */
    int32_t m;        /* history length, 1..8 */
    int32_t h0_iters; /* CG iterations of the H0 solve, >= 1 */
} disco_lbfgs;

typedef struct disco_ctx disco_ctx;
typedef void *disco_stream; /* hipStream_t */

/* Create a context for one image pair geometry on the current HIP device.  storage is
   DISCO_STORAGE_FP32 or DISCO_STORAGE_FP16.  Allocates the derived volumes (grad R,
   grad T, per-voxel GN vectors: 3 x 12 B per voxel in FP32, 3 x 8 B in FP16, whose three
   halfs are padded to one aligned 8-byte word) and small workspaces.  The volume may hold
   at most (2^32 - 1) / 3 voxels in FP32 and (2^32 - 1) / 4 in FP16 (DISCO_ERR_SHAPE
   otherwise).  *out receives the context (NULL on error). */
int disco_create(const disco_geom *geom, int32_t storage, disco_ctx **out);

/* Free a context (synchronises the device first).  NULL is ignored. */
void disco_destroy(disco_ctx *ctx);

/* Set the fixed image R and moving image T (device float32 [Nz][Ny][Nx]) and build
   their central-difference gradient volumes with replicated borders (the gradients of
   eq. 1).  Invalidates the linearisation. */
int disco_set_images(disco_ctx *ctx, const float *R, const float *T, disco_stream stream);

/* disco_set_images for callers that cannot allocate device memory (code under HIP graph
   capture, serving loops, harnesses that forbid hipMalloc): the same result, bitwise, with
   no allocation in the call.  With FP16 storage the scale search keeps its per-tile
   maxima (one double per 64 x 16 x 16 voxel tile) in a static device array of 128 KB
   instead of a buffer the context allocates at its first disco_set_images call, so
   volumes of more than 2^14 tiles (ceil(Nx/64) ceil(Ny/16) ceil(Nz/16) > 16384, e.g.
   beyond 512 x 512 x 1024) are rejected with DISCO_ERR_LIMIT before anything is queued;
   FP32 storage needs no scratch and has no such limit.  Every call on a device shares that device's array: calls that overlap on
   one device (different streams or host threads) race.  The array is held until the
   process ends.  Like disco_set_images, the FP16 scale search synchronises the stream. */
int disco_set_images_noalloc(disco_ctx *ctx, const float *R, const float *T, disco_stream stream);

/* Replace the moving image T of eq. 1 (device float32 [Nz][Ny][Nx]) and rebuild only its
   gradient volume; grad R is kept.  For callers that evaluate one fixed image against
   many moving images (the loss form).  DISCO_ERR_STATE if no images were set; on a
   device error the context has no images until the next disco_set_images.
   Invalidates the linearisation. */
int disco_set_moving(disco_ctx *ctx, const float *T, disco_stream stream);

/* Set n keypoints x_i and targets y_KP(x_i) of eq. 10 (HOST float32 [n][3], mm).  Every
   x_i must lie in the closed box [0, N_a h_a] (else DISCO_ERR_SHAPE).  n = 0 clears
   them.  Copies and bins them by control-grid cell; the host arrays may be reused on
   return. */
int disco_set_keypoints(disco_ctx *ctx, int32_t n, const float *x_mm, const float *t_mm, disco_stream stream);

/* Set the prior displacement uhat of eq. 5 (device node field), or NULL for uhat = 0. */
int disco_set_reference(disco_ctx *ctx, const float *u_ref, disco_stream stream);

/* NGF distance of eq. 1 at displacement u: *D_dev = h_x h_y h_z sum_v (1 - r_v^2). */
int ngf_eval(disco_ctx *ctx, double eta, const float *u, double *D_dev, disco_stream stream);

/* NGF distance of eq. 1 and its gradient g = dD/du (node field) by the matrix-free
   derivative rules of Sec. II-D3: g = -2 h^3 sum_v phi_v r_v s_v with
   s_v = J_G(y_v)^T dr/da the chain rule through the trilinear sample of grad T.  diag
   (nullable) receives the diagonal of the Gauss-Newton matrix 2 h^3 J^T J.  Also records
   u as the linearisation point and stores s_v per voxel for ngf_hessvec. */
int ngf_grad(disco_ctx *ctx, double eta, const float *u, double *D_dev, float *g, float *diag,
             disco_stream stream);

/* Gauss-Newton product of the NGF term of eq. 1 (Sec. II-D3, matrix-free):
   Hv = 2 h^3 J^T (J v) = 2 h^3 sum_v phi_v s_v (s_v . (P v)(x_v)) with the s_v of the last
   linearisation (ngf_grad or gn_pcg_step); DISCO_ERR_STATE if there is none.  v and Hv
   are device node fields [3][nz][ny][nx]. */
int ngf_hessvec(disco_ctx *ctx, const float *v, float *Hv, disco_stream stream);

/* Set the binary lung masks b_F of R and b_M of T (device uint8 [Nz][Ny][Nx], values 0
   or 1) of the lung-boundary term of eq. 6, copied into the context; both NULL clears
   them.  With masks set and params->beta != 0, the objective, gradient and GN products
   of gn_pcg_step, gn_hessvec, lbfgs_step and objective_linearise include
   beta B = beta/2 h^3 sum_v (b_M(y(x_v)) - b_F(x_v))^2, b_M sampled trilinearly at the
   warped voxel (zero outside the volume), with the exact-form Gauss-Newton matrix
   beta h^3 sum_v P_v^T grad b_M grad b_M^T P_v.  Allocates 14 bytes per voxel on the
   first call (masks and the per-voxel GN vectors of the term). */
int disco_set_masks(disco_ctx *ctx, const uint8_t *bF, const uint8_t *bM, disco_stream stream);

/* Linearise the joint objective of eq. 11 at u: terms_dev (nullable, device doubles [8])
   receives J, D, S, V (+inf on a fold), K, B, the fold count and |grad J|; g and diag
   (nullable) receive grad J and the diagonal of the GN matrix.  Sets the linearisation
   used by gn_hessvec. */
int objective_linearise(disco_ctx *ctx, const disco_params *p, const float *u, double *terms_dev, float *g,
                        float *diag, disco_stream stream);

/* The joint objective of eq. 11 at u without derivatives (one pass over the voxels, as a
   line-search trial): terms_dev (device doubles [8], 8-byte aligned, required) receives J,
   D, S, V (+inf on a fold), K, B, the fold count and NaN in the |grad J| slot.  Only the
   weights and eta of p are used.  Leaves the linearisation and the s vectors unchanged. */
int objective_eval(disco_ctx *ctx, const disco_params *p, const float *u, double *terms_dev, disco_stream stream);

/* Derivative of the NGF distance of eq. 1 with respect to the moving image values at
   displacement u: dT (device float32 [Nz][Ny][Nx]) = scale * dD/dT, through the
   trilinear sampling of grad T and its central-difference stencil.  scale_dev (nullable:
   1) is one device double read by the kernels, so that a caller's upstream gradient
   needs no host round trip and no extra pass.  The scatter to warped positions adds to
   the field with float atomics, so the last bits of dT may differ between runs.  Needs
   images set; allocates a [N][3] float32 work volume on the first call. */
int ngf_grad_T(disco_ctx *ctx, double eta, const float *u, const double *scale_dev, float *dT,
               disco_stream stream);

/* Curvature term of eq. 5 with weight alpha: w = u - u_ref (u_ref nullable: 0),
   *S_dev = alpha S(u) (nullable), out = alpha C_H L^T L w (the gradient; nullable),
   diag = alpha C_H diag(L^T L) (nullable).  Called with u = v and u_ref = NULL, out is
   the (exact) Hessian product.  L is the node-grid Laplacian with vanishing second
   differences at border nodes, C_H = 64 h_x h_y h_z. */
int curvature_apply(disco_ctx *ctx, double alpha, const float *u, const float *u_ref, double *S_dev, float *out,
                    float *diag, disco_stream stream);

/* Volume-change control of eq. 7-9 with weight gamma at displacement u:
   *V_dev = gamma Vhat(u) (+inf on a fold), g = gamma grad Vhat (nullable),
   diag = gamma diag of the GN matrix C sum psi''(d) grad d grad d^T (nullable),
   Hv = gamma GN matrix times v (v and Hv both NULL or both set),
   *nfold_dev = number of coefficients d <= 0 (nullable). */
int volchange_eval(disco_ctx *ctx, double gamma, const float *u, double *V_dev, float *g, float *diag, const float *v,
                   float *Hv, int32_t *nfold_dev, disco_stream stream);

/* Keypoint penalty of eq. 10 with weight delta: *K_dev = delta K(u) (nullable),
   g = 2 delta P^T res (nullable), diag = 2 delta diag(P^T P) (nullable),
   Hv = 2 delta P^T P v (v and Hv both NULL or both set). */
int keypoint_penalty(disco_ctx *ctx, double delta, const float *u, double *K_dev, float *g, float *diag,
                     const float *v, float *Hv, disco_stream stream);

/* Full Gauss-Newton product of eq. 11 at the last linearisation:
   Hv = H_D v + alpha C_H L^T L v + beta H_B v + gamma H_V v + delta 2 P^T P v + tau v
   (H_B only with masks set; then the linearisation must have had beta != 0 too, else
   DISCO_ERR_STATE). */
int gn_hessvec(disco_ctx *ctx, const disco_params *p, const float *v, float *Hv, disco_stream stream);

/* One Gauss-Newton step of eq. 11 from u (updated in place on success):
   linearise at u; solve (H + tau I) p = -grad J by Jacobi-PCG (x0 = 0, preconditioner
   diag H + tau + 1e-12 max diag H, pcg_iters iterations or |r| <= pcg_tol |g|, stop on
   p^T H p <= 0); Armijo backtracking t = 1, 1/2, ... (at most ls_max trials) accepting
   the first t with J(u + t p) finite and <= J(u) + c1 t g^T p.  report_dev (nullable)
   receives DISCO_REP_SIZE doubles; status_dev (nullable) the DISCO_STATUS_* bits.
   Without DISCO_FLAG_LS_DEVICE the host waits, once per line-search trial, for the
   acceptance flag of the previous trial while the GPU runs the next one (one trial past
   the accepted one is enqueued and does nothing); with it the call never synchronises and
   can be graph captured. */
int gn_pcg_step(disco_ctx *ctx, const disco_params *p, float *u_inout, double *report_dev, int32_t *status_dev,
                disco_stream stream);

/* One L-BFGS iteration on J of eq. 11 from u (updated in place), Sec. II-D3: J and
   grad J at u; if the previous call of this context made a step, the pair
   s = u - u_old, y = grad J(u) - grad J(u_old) joins a history of the last lb->m pairs
   (a pair failing s^T y > curv_eps |s||y| is kept with rho = 0, i.e. it changes nothing);
   the two-loop recursion gives p = -H g, with the initial inverse H0^{-1} applied by
   Jacobi-PCG on H0 = alpha C_H L^T L + tau I (x0 = 0, h0_iters iterations or
   |r| <= h0_tol |q|); then the Armijo line search of gn_pcg_step along p.  The report
   has the layout of gn_pcg_step's, with the H0 solve in the CG slots.  Only the
   weights, eta, armijo_c1, ls_max and flags of p are used.  The history buffers
   (2 m vectors of 3 (Nx/4+1)(Ny/4+1)(Nz/4+1) floats) are allocated on the first call and
   when m changes (which also clears the history; the call then synchronises the
   stream).  u must be the field returned by the previous call for the history to
   describe the iteration; lbfgs_reset starts a new one.  The history position is host
   state, so a graph-captured call would replay one fixed position: capture is not
   supported. */
int lbfgs_step(disco_ctx *ctx, const disco_params *p, const disco_lbfgs *lb, float *u_inout, double *report_dev,
               int32_t *status_dev, disco_stream stream);

/* Forget the L-BFGS history of the context (the next lbfgs_step starts from H0). */
int lbfgs_reset(disco_ctx *ctx);

/* ---- multilevel scheme (Sec. II-D3) ------------------------------------------------- */

#define DISCO_MAX_LEVELS 8
#define DISCO_OPT_GN 0    /* gn_pcg_step per iteration */
#define DISCO_OPT_LBFGS 1 /* lbfgs_step per iteration (fresh history on every level) */

/* The pyramid of a volume of n voxels at spacing h (host only, no device call): level 0
   is the input; each coarser level halves the axes of the valid non-empty subset (sizes
   divisible by 8, coarse size >= 8) whose coarse spacing is most nearly isotropic
   (smallest max h / min h; ties: more axes, then x before y before z), so the voxels
   approach isotropy as the paper asks.  Stops early when no subset is valid.  Writes
   *levels_out <= levels, and per level (finest first) n_out[3 l + a], h_out[3 l + a] and
   halve_out[3 l + a] (1 if axis a was halved from level l - 1; 0 on level 0).  The
   control grid follows the voxels (4 voxels per cell), so it halves with them.
   Arrays hold 3 * levels entries; levels in 1..DISCO_MAX_LEVELS; n multiples of 4. */
int pyramid_plan(const int32_t n[3], const double h[3], int32_t levels, int32_t *levels_out, int32_t *n_out,
                 double *h_out, int32_t *halve_out);

/* One pyramid step of a volume (device float32 [Nz][Ny][Nx], n = {Nx, Ny, Nz}): along
   each halved axis Gaussian smoothing (sigma = 1 voxel of the finer level, taps -3..3
   renormalised, border replicated), then each coarse voxel is the mean of the two finer
   voxels it covers (the smoothed value at the coarse voxel centre).  dst has the halved
   size.  Halved sizes must be even.  With two or more halved axes, work (device) holds
   N/2 + N/4 floats, N = Nx Ny Nz (NULL otherwise); axes are processed x, y, z. */
int pyramid_downsample(const float *src, const int32_t n[3], const int32_t halve[3], float *dst, float *work,
                       disco_stream stream);

/* Prolongation of a node field (device float32 [3][nz][ny][nx], nodes = {nx, ny, nz}) to
   the next finer level: along a halved axis the fine grid has 2 (n - 1) + 1 nodes, even
   ones copy a coarse node and odd ones average the two beside it, which is the coarse
   trilinear displacement evaluated at the fine nodes (the coarse field is represented
   exactly).  Values are displacements in mm and are not rescaled. */
int pyramid_prolong(const float *uc, const int32_t nodes[3], const int32_t halve[3], float *uf, disco_stream stream);

typedef struct {
    disco_params params;    /* weights, eta, line search, CG (GN); delta is ignored with adaptive_delta */
    disco_lbfgs lbfgs;      /* L-BFGS settings (optimizer DISCO_OPT_LBFGS) */
    int32_t levels;         /* requested levels, 1..DISCO_MAX_LEVELS (fewer if the pyramid stops) */
    int32_t optimizer;      /* DISCO_OPT_GN or DISCO_OPT_LBFGS */
    int32_t adaptive_delta; /* 1: delta with D = delta K at u = 0 on the coarsest level (Sec. II-D2) */
    int32_t storage;        /* DISCO_STORAGE_* of every level */
    int32_t iters[DISCO_MAX_LEVELS]; /* iterations per level, coarsest built level first */
} disco_multilevel;

/* Coarse-to-fine registration (Sec. II-D3) of R and T (device float32 [Nz][Ny][Nx] of
   geometry geom) with nkp keypoints (HOST float32 [nkp][3], mm): builds the pyramid
   (pyramid_plan, pyramid_downsample), starts from u = 0 on the coarsest level, runs
   iters[k] iterations of the optimiser on each level (a level ends early when a line
   search accepts no step) and prolongs u to the next level (pyramid_prolong).  u_out
   (device node field of the finest level) receives the result.  report_dev (nullable,
   device doubles [sum of iters over the built levels][DISCO_REP_SIZE]) receives one
   report per iteration in execution order; rows of iterations not run are NaN.
   *levels_out and *delta_out (host, nullable) receive the number of levels and the
   keypoint weight used.  Allocates every level's context and images for the duration of
   the call and synchronises the stream after each iteration (to stop a level early). */
int multilevel_register(const disco_geom *geom, const float *R, const float *T, int32_t nkp, const float *kp_x,
                        const float *kp_t, const disco_multilevel *cfg, float *u_out, double *report_dev,
                        int32_t *levels_out, double *delta_out, disco_stream stream);

/* ---- keypoint stage (Sec. II-C2, II-C3) ---------------------------------------------- */

typedef struct disco_kp disco_kp;

/* A keypoint-matching context for images of n = {Nx, Ny, Nz} voxels at spacing h (mm; the
   paper resamples both scans to 1 mm isotropic for this stage, so that displacements in
   voxels are displacements in mm), on the current device.  Allocates 2 x 16 bytes per
   voxel. */
int disco_kp_create(const int32_t n[3], const double h[3], disco_kp **out);
void disco_kp_destroy(disco_kp *kp);

/* Fixed image F and moving image M (device float32 [Nz][Ny][Nx]): central-difference
   gradients (replicated border, HU/mm) normalised with eta as in eq. 1, stored as the
   4-vectors (eta, grad I) / |(eta, grad I)|; outside the volume the gradient is zero. */
int disco_kp_set_images(disco_kp *kp, const float *F, const float *M, double eta, disco_stream stream);

/* The matching cost of eq. 2 for nkp keypoints (device int32 [nkp][3], voxel indices
   x, y, z): cost (device float32 [nkp][(2R+1)^3], labels [iz][iy][ix]) receives
   D_KP(k, d) = 1/64 sum_{p in P_k} (1 - r(p, p + d)^2) with P_k = k + {-3,-1,1,3}^3 (a
   7^3 patch of stride 2), d = 2 (i - R) voxels per axis (step 2, the paper's
   {0, +-2, ..., +-32} mm for R = 16), r the eta-normalised gradient cosine of eq. 1.
   1 <= R <= 16. */
int disco_kp_cost(disco_kp *kp, int32_t nkp, const int32_t *kp_vox, int32_t R, float *cost, disco_stream stream);

/* Regularised correspondences (Sec. II-C3): minimum spanning tree over all keypoint pairs
   with edge cost w_kq = |x_k - x_q| + |I_k - I_q| / sigma_I (Boruvka rounds: the cheapest
   edge of every keypoint found on the device, components merged on the host, edges
   ordered by (w, lower index, higher index); returned rooted at keypoint 0), then
   two-pass min-sum belief propagation on the tree with the data cost `cost` (as written by
   disco_kp_cost) and the regulariser of eq. 3, alpha_kp |d_k - d_q|^2 / w_kq (|.| in mm),
   each message a min-convolution done as three exact 1-D minimisations (x, y, z), one tree
   level per launch pair.  The messages are scheduled from the tree's centre (the middle
   of a longest path), which brings the levels down to the tree's radius; min-marginals do
   not depend on the root.  x_mm (HOST float32 [nkp][3]) and inten (HOST float32 [nkp], F
   at the keypoint) define w; the keypoints must be distinct (w > 0).  Writes the
   min-marginal energies to marg (device float32 [nkp][(2R+1)^3], nullable), the label of
   the smallest one per keypoint (lowest index on ties) to labels (device int32 [nkp]) and
   the tree to parent_out (HOST int32 [nkp], nullable; -1 at the root).  Work memory of
   3 x nkp x (2R+1)^3 floats (4 x when marg is null) and about 100 bytes per keypoint of
   tree set-up buffers (pinned host and device) are kept in the handle, grown when a call
   needs more and freed by disco_kp_destroy; the call waits for the stream before
   returning, and calls on one handle must not overlap. */
int disco_kp_regularise(disco_kp *kp, int32_t nkp, const float *x_mm, const float *inten, int32_t R,
                        const float *cost, double alpha_kp, double sigma_I, float *marg, int32_t *labels,
                        int32_t *parent_out, disco_stream stream);

/* Copy a derived buffer (DISCO_BUF_*) to dst, converted to float32 [Nz][Ny][Nx][3]. */
int disco_copy_buffer(disco_ctx *ctx, int32_t which, float *dst, disco_stream stream);

/* Per-kernel timing with HIP events recorded on the launch stream.  enable = 1 starts
   recording (clears counters), 0 stops.  disco_profile_read waits for the recorded
   events and returns the number of launches and total milliseconds of one kernel
   class: 0 = Gauss-Newton product pass over the voxels, 1 = gradient pass,
   2 = objective-only pass, 3 = image gradients, 4 = derivative with respect to T
   (ngf_grad_T: clear, scatter and stencil passes together). */
int disco_profile(disco_ctx *ctx, int32_t enable);
int disco_profile_read(disco_ctx *ctx, int32_t kernel, int64_t *launches, double *ms_total);

/* Human-readable text of a return code. */
const char *disco_status_string(int code);

/* ---- Batched Gauss-Newton steps over many pairs (uneven sizes) ----------------------
   A batch groups existing contexts (same device and storage, images and keypoints set)
   and runs one Gauss-Newton step of eq. 11 for every pair with ONE kernel launch per
   phase of the step: each launch walks the (pair, block) work items of all pairs, the
   largest pair first.  Each pair gets the arithmetic of gn_pcg_step with
   DISCO_FLAG_LS_DEVICE (equal up to the rounding of fused multiply-adds).  The step has no
   host synchronisation, so it can be captured in a graph (disco_batch_graph_capture) and
   replayed; replays are bitwise reproducible. */
typedef struct disco_batch disco_batch;

/* Group npairs contexts (not copied: they must outlive the batch; no context twice). */
int disco_batch_create(int32_t npairs, disco_ctx *const *ctxs, disco_batch **out);
void disco_batch_destroy(disco_batch *batch);

/* Fix what the next steps work on: params[i] (HOST array of npairs, each with
   DISCO_FLAG_LS_DEVICE; the terms present, pcg_iters and ls_max equal for all pairs) and
   u[i] (HOST array of npairs DEVICE node fields, updated in place by every step).
   report_dev (device, npairs x DISCO_REP_SIZE doubles, nullable) and status_dev (device,
   npairs int32, nullable) receive each pair's report and status.  Copies a descriptor
   table to the device (synchronous); invalidates a captured graph. */
int disco_batch_prepare(disco_batch *batch, const disco_params *params, float *const *u, double *report_dev,
                        int32_t *status_dev);

/* One GN step of every pair on `stream`. */
int disco_batch_gn_step(disco_batch *batch, disco_stream stream);

/* Launch shape of the batched passes: workgroups per compute unit of a persistent grid
   for the brick passes (pass 0), the node passes (1) and the vector passes (2), capped at
   each kernel's residency; 0 launches one workgroup per work item instead.  Invalidates a
   captured graph. */
int disco_batch_set_launch(disco_batch *batch, int32_t pass, int32_t wg_per_cu);

/* Brick tile of the batched passes: bricks of 16 x 4 x cells_z cells, cells_z = 4 (the
   single-pair tile, default) or 2 (twice the bricks, half the depth: more work items for
   batches of small pairs).  The tile changes the order in which brick contributions are
   summed, so steps on the two tiles agree to rounding.  Invalidates a captured graph and
   the prepared descriptors: call disco_batch_prepare again before the next step. */
int disco_batch_set_tile(disco_batch *batch, int32_t cells_z);

/* Capture nsteps GN steps into a graph owned by the batch (library stream; no host
   synchronisation inside), and replay it on `stream`.  A replay works on the arrays
   given to disco_batch_prepare. */
int disco_batch_graph_capture(disco_batch *batch, int32_t nsteps);
int disco_batch_graph_launch(disco_batch *batch, disco_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* DISCO_H */
