/*
 * wbsph.h -- C ABI of the MI355X (gfx950) well-balanced WCSPH hot path.
 *
 * Method: Zhang, Zhao, Gan, Xu, "A well-balanced weakly compressible SPH
 * formulation for free-surface flows and its GPU implementation".  The library
 * advances the semi-discrete system of Eq. (sph) (Sec. 2.3) with SSP-RK2
 * (Sec. 2.3), neighbours from the hashed background grid of Sec. 3
 * (Eqs. hashid/ixyz, Algorithm 1), walls by the dummy mirror of Sec. 2.4.
 *
 * Conventions for every entry point
 *   - Plain pointers and sizes only.  "Device" pointers are HIP device (or
 *     managed) addresses on the current device; "host" pointers are ordinary
 *     process memory.  Arrays of vectors are row-major, n rows of `dim`
 *     doubles (x0 y0 [z0] x1 y1 ...).
 *   - The caller owns every buffer it passes.  The workspace handed to
 *     sph_init (and sph_mlp_create) must stay allocated and untouched until
 *     the matching destroy call; the library allocates no device memory (the
 *     one fixed array it holds, for sph_mlp_forward_noalloc, is part of the
 *     loaded code object).
 *   - All device work is enqueued on the caller's hipStream_t (passed as
 *     void*; NULL = the null stream).  Calls return before the GPU finishes
 *     unless they write host memory, which synchronises the stream.
 *   - Errors: every call returns an sph_status.  Device-side faults (particle
 *     outside the hashed domain, non-finite state, a neighbour list beyond
 *     its capacity) are recorded on the device and reported by the next call
 *     that synchronises (sph_sync, sph_fields into host memory, sph_neighbors);
 *     after such an error only sph_fields (which still fills its output and
 *     returns the error), sph_last_error and sph_destroy are accepted
 *     (SPH_ESTATE otherwise).
 *   - A context is not thread-safe; several contexts may coexist.
 */
#ifndef WBSPH_H
#define WBSPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sph_status;
#define SPH_OK 0
#define SPH_EINVAL (-1)      /* bad argument or parameter                       */
#define SPH_EWORKSPACE (-2)  /* workspace missing, misaligned or too small       */
#define SPH_EHIP (-3)        /* a HIP runtime call failed                        */
#define SPH_EDOMAIN (-4)     /* a particle left the hashed domain                */
#define SPH_ENONFINITE (-5)  /* NaN / Inf in the state, or coincident particles  */
#define SPH_ESTATE (-6)      /* call not allowed in the context's state          */
#define SPH_EUNSUPPORTED (-7)
#define SPH_ECAPACITY (-8)   /* a per-particle neighbour list overflowed         */

/* precision */
#define SPH_FP64 0  /* FP64 storage and arithmetic throughout                     */
#define SPH_MIXED 1 /* int cell + FP32 offset positions, FP32 pair evaluation,
                       FP64 accumulation of L and of the potential-gradient sums */
#define SPH_FP32 2  /* the paper's single-precision design (Sec. 3): the
                       mixed path's storage (which keeps what Kahan-compensated
                       FP32 attributes keep), but every pair term in FP32 from
                       the absolute FP32 positions and FP32 potentials (sums
                       per list fill in FP32, totals and epilogue in FP64);
                       for comparison with the other two forms              */

/* free-surface detection */
#define SPH_FS_NONE 0
#define SPH_FS_EXACT 1   /* lambda_min thresholds + scan-region pass (Sec. 2.3) */
#define SPH_FS_LEARNED 2 /* MLP on 16 features, exact fallback at low margin    */

/* flags */
#define SPH_F_DELTA 1u       /* delta-SPH diffusion in the potential equation   */
#define SPH_F_PST 2u         /* particle shifting                               */
#define SPH_F_TIC 4u         /* conservative gradient where lambda_min < tic    */
#define SPH_F_FS_PROJECT 8u  /* shifting keeps only its tangential part at FS   */
#define SPH_F_CONT_UNCORR 16u /* uncorrected continuity where TIC is active     */
#define SPH_F_FEATURES 32u   /* keep the 16 classifier features of every fluid  */
                             /* particle (without it, the learned mode computes */
                             /* them for free-surface candidates only)          */
#define SPH_F_KEEP_LISTS 64u /* the first stage of a step keeps its candidate   */
                             /* lists (radius 2h + s, s the cells' room         */
                             /* ceil(2h/R) R - 2h) and the second stage runs    */
                             /* from them, without a sort or a search, when     */
                             /* twice the bound on any particle's move since    */
                             /* (1.5 dt U_max per first stage, 0.75 dt (U_max0  */
                             /* + U_max1) per second) plus a rounding pad fits  */
                             /* s; otherwise, or after a list overflow (more    */
                             /* than 256 candidates for a particle), it sorts   */
                             /* and searches.  Needs cells with room (R a       */
                             /* little above 2h / ceil(2h/R)).  Neighbour sets, */
                             /* and so results, are the same; about 1 KiB of    */
                             /* workspace per fluid particle.                   */
#define SPH_F_KEEP_ACROSS_STEPS 128u /* with SPH_F_KEEP_LISTS: the lists    */
                             /* also serve later steps under the same bound     */
                             /* (a step then sorts only when they run out; a    */
                             /* particle that leaves the domain is reported at  */
                             /* the next sort)                                  */
#define SPH_F_GRAPH 256u     /* sph_step runs pairs of steps as one HIP graph   */
                             /* captured at its first use (the same kernels in  */
                             /* the same order as without; recaptured after any */
                             /* call that changes what a step launches: a right-*/
                             /* hand side outside sph_step, a new classifier or */
                             /* dt_override).  Excludes SPH_F_KEEP_LISTS, whose */
                             /* reuse test reads the device between stages.     */

typedef struct sph_params {
    int32_t dim;        /* 2 or 3; gravity usually along the last axis          */
    int32_t precision;  /* SPH_FP64 | SPH_MIXED | SPH_FP32                      */
    int32_t fs_mode;    /* SPH_FS_*                                             */
    uint32_t flags;     /* SPH_F_*                                              */
    double dx;          /* initial particle spacing                             */
    double h;           /* smoothing length (Wendland C2, support 2h)           */
    double c0;          /* artificial sound speed                               */
    double rho0;        /* reference density                                    */
    double nu;          /* kinematic viscosity: enters the time-step rule only  */
    double delta;       /* delta-SPH coefficient                                */
    double cfl;         /* CFL number                                           */
    double pst_R, pst_n; /* shifting weight 1 + R (W/W(dx))^n                    */
    double lambda_tic;      /* TIC threshold (strict <)                         */
    double lambda_fs_lo;    /* lambda <= lo: free surface                       */
    double lambda_fs_hi;    /* lambda >  hi: interior; between: scan region     */
    double lambda_singular; /* lambda <= this: L treated as singular            */
    double gravity[3];      /* body force G0                                    */
    double forcing_amp[3];  /* G(t) = G0 + amp w^2 sin(w t) (tank-frame forcing) */
    double forcing_omega;
    double domain_lo[3], domain_hi[3]; /* hashed box; particles must stay inside */
    double cell_size;       /* background cell R (0 -> 2h); >= 2h/3: the search
                               spans ceil(2h/R) cells on each side                */
    /* Prescribed motion of a body made of wall dummies of kind 2 (the
     * aircraft-ditching case of Sec. 4 prescribes the body's velocity as a
     * piecewise function of time).  Velocity U(t) = body_a[k] + body_b[k] t
     * on piece k, body_t[k] <= t <= body_t[k+1] (the lower piece at a shared
     * breakpoint), zero before body_t[0] and after body_t[body_pieces].  The
     * body translates rigidly: a kind-2 dummy given at x sits at x + D(t),
     * D(t) the integral of U from body_t[0] to t, at every right-hand side;
     * its mirrored velocity keeps the wall's normal velocity, U_d = U_f -
     * ((U_f - U(t)).n_d) n_d.  body_pieces = 0: no motion (kind-2 dummies act
     * as fixed walls).  With a moving body the dummies are re-sorted at every
     * right-hand side and SPH_F_KEEP_LISTS has no effect.                    */
    int32_t body_pieces;    /* 0..4                                               */
    int32_t body_pad_;
    double body_t[5];       /* breakpoints, strictly increasing                   */
    double body_a[4][3];
    double body_b[4][3];
    /* A free rigid body made of the kind-2 dummies (the cylinder water entry
     * of Sec. 4: the body falls under G(t) and the water's force), used when
     * body_free != 0 (body_pieces must then be 0; every precision: the force
     * is summed in FP64 from the records of the path).
     * The kind-2 rows are given in a reference pose whose centre is body_c0;
     * a body state of centre c and unit quaternion q = (w, x, y, z) puts a
     * dummy given at x_ref, n_ref at c + R(q)(x_ref - body_c0) with normal
     * R(q) n_ref, and its wall velocity is v + omega x R(q)(x_ref - body_c0).
     * Force on the body: each of its dummies with a mirror source takes the
     * conservative-form acceleration of Eq. (sph) (the branch of Sec. 2.3)
     * from its fluid neighbours, a_d = -sum_i (phi_i + phi_d) grad_d W_di
     * V_i, with its mirrored potential; F = sum m_d a_d, torque about c =
     * sum (x_d - c) x m_d a_d.  The state advances with the fluid's SSP-RK2
     * stages: dc/dt = v, dv/dt = F/M + G(t), dq/dt = (0, omega) q / 2,
     * domega/dt = I_w^-1 (T - omega x I_w omega), I_w = R I_body R^T; the
     * quaternion is renormalised after each stage.  In 2D the body moves in
     * the plane and turns about z: q = (cos, 0, 0, sin), omega = (0, 0, wz).
     * The dummies are re-sorted at every right-hand side and
     * SPH_F_KEEP_LISTS has no effect.                                        */
    int32_t body_free;
    int32_t body_pad2_;
    double body_mass;        /* > 0                                                */
    double body_inertia[6];  /* about the centre, body frame: xx yy zz xy xz yz;
                                positive definite (2D: zz > 0)                    */
    double body_c0[3];       /* centre of the reference pose                      */
    double body_state0[13];  /* initial c[3], q[4] (unit), v[3], omega[3] (world) */
} sph_params;

typedef struct sph_ctx sph_ctx;

/* ---------------------------------------------------------------- host only */

/* Checks a parameter block; no GPU is touched.  SPH_OK or SPH_EINVAL. */
sph_status sph_validate(const sph_params *p);

/* Workspace bytes a context needs for n_fluid fluid and n_dummy wall
 * particles (0 if the parameters are invalid).  No GPU is touched. */
size_t sph_workspace_bytes(const sph_params *p, int64_t n_fluid, int64_t n_dummy);

const char *sph_status_string(sph_status s);

/* ------------------------------------------------------------------ lifetime */

/* Creates a context holding n particles in the caller's ("original") order.
 * x, u: n*dim doubles; phi: n doubles; mass: n doubles or NULL, in which case
 * m = rho0 exp(phi/C0^2) dx^dim (Sec. 2.2.1); kind: n bytes, 0 fluid, 1 fixed
 * dummy wall particle (Sec. 2.4), 2 dummy of the moving body (its position
 * of time body_t[0], or of the free body's reference pose); normal: n*dim
 * doubles, the unit wall normal of each dummy (fluid rows ignored).  inputs_on_device selects whether the
 * six arrays are device (1) or host (0) pointers; they are copied and may be
 * released after the call.  workspace: a device buffer of ws_bytes >=
 * sph_workspace_bytes(), 256-byte aligned.  hip_stream: the stream all work
 * goes to.  Validation (parameters, finiteness, positions inside the domain,
 * unit normals) happens on the host before any launch when inputs are host
 * pointers; for device inputs domain/finiteness errors surface at sph_sync. */
sph_status sph_init(const sph_params *p, int64_t n, const double *x, const double *u,
                    const double *phi, const double *mass, const uint8_t *kind,
                    const double *normal, int32_t inputs_on_device, void *workspace,
                    size_t ws_bytes, void *hip_stream, sph_ctx **out);

void sph_destroy(sph_ctx *ctx);

/* Last error text of the context (owned by the context). */
const char *sph_last_error(const sph_ctx *ctx);

/* ------------------------------------------------------------------ hot path */

/* Background grid and fluid ordering at the current positions: cell index
 * (Eq. ixyz, with N_a = floor((hi-lo)/R) + 1), HashID (Eq. hashid), a sort of
 * the fluid by (HashID, original index), reordering of the particle arrays
 * and the begin/end index of every cell (Sec. 3).  sph_step rebuilds before
 * every right-hand side; this entry exists for inspection and parity. */
sph_status sph_build_cells(sph_ctx *ctx);

/* Advances nsteps SSP-RK2 steps (Sec. 2.3).  dt_override > 0 fixes the step;
 * otherwise dt = CFL min(dx/(C0+|U|max), dx^2/(2 nu), sqrt(2 dx/|G|max)) from
 * the state at the start of each step, computed on the device.  Each stage:
 * rebuild cells, mirror dummies (Eq. phiBn, slip), fused pair pass and
 * epilogue (Eqs. renorm, parGrad, lfsover, sph; delta-SPH, shifting, TIC),
 * free-surface detection, stage update.  Asynchronous, except that with
 * SPH_F_KEEP_LISTS each stage first waits for the previous one (to choose
 * between the kept lists and a rebuild). */
sph_status sph_step(sph_ctx *ctx, int32_t nsteps, double dt_override);

/* One right-hand side at the current state and time (no integration):
 * rebuild, mirror, pair pass, detection.  Results readable by sph_fields. */
sph_status sph_eval_rates(sph_ctx *ctx);

/* Sets the simulation time of the state (e.g. when resuming from fields
 * saved at time t; the forcing G(t) depends on it).  Stream ordered. */
sph_status sph_set_time(sph_ctx *ctx, double t);

/* Waits for the stream and reports deferred device errors. */
sph_status sph_sync(sph_ctx *ctx);

/* field selectors for sph_fields: all per-particle fields are returned for the
 * n particles in ORIGINAL order.  Rows of dummies hold their mirrored phi / U
 * and zero rates; rows of the moving body hold its positions of the last
 * right-hand side (of sph_init before any). */
#define SPH_FIELD_X 0          /* n*dim double                                   */
#define SPH_FIELD_U 1          /* n*dim double                                   */
#define SPH_FIELD_PHI 2        /* n double                                       */
#define SPH_FIELD_RHO 3        /* n double: rho0 exp(phi/C0^2)                   */
#define SPH_FIELD_P 4          /* n double: C0^2 (rho - rho0)  (Eq. eos-water)   */
#define SPH_FIELD_DUDT 5       /* n*dim double (last right-hand side)            */
#define SPH_FIELD_DPHIDT 6     /* n double                                       */
#define SPH_FIELD_DELTA_U 7    /* n*dim double: shifting velocity                */
#define SPH_FIELD_LAMBDA 8     /* n*3 double: eigenvalues of L, ascending        */
#define SPH_FIELD_NORMAL 9     /* n*dim double                                   */
#define SPH_FIELD_FS 10        /* n int32: 1 = free surface                      */
#define SPH_FIELD_TIC 11       /* n int32: 1 = conservative branch used          */
#define SPH_FIELD_NNB 12       /* n int32: neighbour count                       */
#define SPH_FIELD_CELL 13      /* n*3 int32: cell coordinates (Eq. ixyz)         */
#define SPH_FIELD_FEATURES 14  /* n*16 float (SPH_F_FEATURES)                    */
#define SPH_FIELD_MASS 15      /* n double                                       */
#define SPH_FIELD_MIRROR_SRC 16 /* n int32: dummies' source fluid (orig) or -1   */
#define SPH_FIELD_LOGIT 17     /* n float: classifier logit (learned mode)       */
#define SPH_FIELD_FS_PATH 18   /* n int32: 0 by lambda, 1 by scan, 2 by MLP      */

/* Copies one field into out (host if out_on_device == 0, else device).  Host
 * output synchronises the stream and returns deferred device errors. */
sph_status sph_fields(sph_ctx *ctx, int32_t field, void *out, int32_t out_on_device);

/* Scalars: out[0] time, [1] last dt, [2] steps taken, [3] U_max of the last
 * right-hand side, [4] fluid count, [5] dummy count, [6] free-surface count,
 * [7] TIC-branch count, [8] scan-pass candidates, [9] MLP-decided count,
 * [10] singular-L count, [11] sum of fluid neighbour counts of the last
 * right-hand side (ordered pairs), [12] free-surface candidates of the last
 * right-hand side, [13] candidate pairs the last pair pass tested (distance
 * computations), [14] right-hand sides of sph_step run from kept candidate
 * lists (SPH_F_KEEP_LISTS), [15] right-hand sides of sph_step that sorted
 * (and, with the flag, built new lists), [16] and [17] the values of [11] and
 * [13] for the last right-hand side that searched, [18] and [19] for the last
 * one that ran from kept lists (tests: kept candidates).  Synchronises. */
sph_status sph_stats(sph_ctx *ctx, double out[20]);

/* State of the free body (body_free) after the last right-hand side or step:
 * out[0..2] centre c, [3..6] unit quaternion (w, x, y, z), [7..9] velocity,
 * [10..12] angular velocity (world frame), [13..15] force and [16..18]
 * torque about the centre of the water on the body at the last right-hand
 * side (zero before any).  Host output; synchronises.  SPH_ESTATE without a
 * free body. */
sph_status sph_body_state(sph_ctx *ctx, double out[19]);

/* Per-kernel timing with HIP events recorded on the context's stream around
 * each launch group while enabled: [0] pair pass with its own search, [1]
 * wall mirror, [2] grid rebuild (hash, sort, reorder; or the record refresh of
 * a right-hand side from kept lists), [3] free-surface detection, [4] stage
 * updates and reductions, [5] pair pass from kept lists.  sph_profile_read
 * synchronises and writes
 * out[2k] = total milliseconds and out[2k+1] = launch count of group k, then
 * clears the totals. */
sph_status sph_profile(sph_ctx *ctx, int32_t enable);
sph_status sph_profile_read(sph_ctx *ctx, double out[16]);

/* Neighbour lists N(i) = {j != i : |x_j - x_i| <= 2h} (Algorithm 1) of every
 * particle at the current positions, as CSR over ORIGINAL indices: offsets
 * (n+1 int64, host), ids (int32, host, ascending within a row).  Fluid rows
 * list fluid and dummy neighbours; dummy rows are empty.  If cap is smaller
 * than the total, ids is not written, *needed receives the total and
 * SPH_ECAPACITY is returned.  Synchronises. */
sph_status sph_neighbors(sph_ctx *ctx, int64_t *offsets, int32_t *ids, int64_t cap,
                         int64_t *needed);

/* ------------------------------------------------------- learned detection */

/* Classifier used in SPH_FS_LEARNED mode: 16 standardised features -> 64
 * (GELU) -> 64 (GELU) -> 1 logit.  params: 5,313 floats in the flat layout
 * W1[16x64] b1[64] W2[64x64] b2[64] W3[64] b3[1]; mean, std: 16 floats each
 * (z = (f - mean)/std); margin: |logit| < margin falls back to the exact
 * scan-region test.  Host pointers; copied into the context. */
sph_status sph_set_classifier(sph_ctx *ctx, const float *params, int64_t nparams,
                              const float *mean, const float *std, float margin);

typedef struct sph_mlp sph_mlp;

/* Workspace bytes for an MLP trainer with minibatches of up to max_batch
 * rows.  No GPU is touched. */
size_t sph_mlp_workspace_bytes(int64_t max_batch);

/* Creates a trainer (FP32 master weights, Adam moments, activations) in the
 * caller's device workspace; params0 (host, 5,313 floats) is the starting
 * point; mean/std (host, 16 floats) standardise the inputs. */
sph_status sph_mlp_create(int64_t max_batch, const float *params0, const float *mean,
                          const float *std, void *workspace, size_t ws_bytes, void *hip_stream,
                          sph_mlp **out);

void sph_mlp_destroy(sph_mlp *m);

/* FP32 forward pass: logits[b] for rows X[b*16..] (device pointers, B <= max_batch). */
sph_status sph_mlp_forward(sph_mlp *m, const float *X, int64_t B, float *logits);

/* Weighted mean binary cross-entropy on the logits (labels y in {0,1}, weights
 * w; device pointers) and its gradient into the trainer's gradient buffer.
 * loss (device, 1 float) and grad (device, 5,313 floats) may be NULL. */
sph_status sph_mlp_loss_grad(sph_mlp *m, const float *X, const float *y, const float *w,
                             int64_t B, float *loss, float *grad);

/* One Adam update from the current gradient (bias-corrected, step count kept
 * by the trainer). */
sph_status sph_mlp_adam(sph_mlp *m, float lr, float beta1, float beta2, float eps);

/* One epoch: minibatches of `batch` rows taken in the order perm[0..n) (device
 * int32) from X (n*16), y, w (device); loss_grad + adam per batch; the mean
 * batch loss goes to *mean_loss (host; synchronises). */
sph_status sph_mlp_train_epoch(sph_mlp *m, const float *X, const float *y, const float *w,
                               const int32_t *perm, int64_t n, int64_t batch, float lr,
                               float *mean_loss);

/* Current weights (host or device out, 5,313 floats). */
sph_status sph_mlp_get_params(sph_mlp *m, float *out, int32_t out_on_device);

/* Inference with BF16 MFMA tiles accumulated in FP32: logits for n rows of X
 * (device, n*16 floats) with the weights in `params` (device, 5,313 floats),
 * standardised by mean/std (device, 16 floats each).  Stateless; works in
 * stream order. */
sph_status sph_mlp_infer_bf16(const float *params, const float *mean, const float *std,
                              const float *X, int64_t n, float *logits, void *hip_stream);

/* ------------------------------------------------ allocation-free variant */

/* Largest batch of sph_mlp_forward_noalloc. */
#define SPH_MLP_NOALLOC_MAX_ROWS 8192

/* For callers that cannot allocate device memory or hand over a workspace
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the FP32 forward pass of sph_mlp_forward without a trainer.
 * Same kernel and same logits bit for bit; the weights come from `params`
 * (device, 5,313 floats, the layout of sph_set_classifier), the
 * standardisation from mean/std (device, 16 floats each), rows from X
 * (device, B*16 floats), logits[b] to `logits` (device, B floats).  The
 * activations the kernel stores go to a fixed scratch array inside the
 * library (B <= SPH_MLP_NOALLOC_MAX_ROWS, about 6.8 MB per device, held
 * until the process ends); no device memory is allocated, neither here nor
 * on the first call of a device (which only looks the array up).
 * B > SPH_MLP_NOALLOC_MAX_ROWS or B < 0 -> SPH_EINVAL before any launch; B
 * = 0 -> SPH_OK.  Asynchronous on hip_stream.  Every call on one device
 * shares that device's scratch array: calls that overlap in time on one
 * device (other streams, other threads) race on it and must be ordered by
 * the caller. */
sph_status sph_mlp_forward_noalloc(const float *params, const float *mean, const float *std,
                                   const float *X, int64_t B, float *logits, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* WBSPH_H */
