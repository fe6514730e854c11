/*
 * msbfm.h -- C ABI of the MI355X (gfx950) library for the matrix-structure-based
 * fast method (MSBFM) of linear bond-based peridynamics:
 *   C. Liu, H. Tian, W. S. Don, H. Wang, "A fast computational framework for the
 *   linear bond-based peridynamic model" (arXiv 2301.11828).
 *
 * The library applies the stiffness matrix A of the meshfree discretisation
 * (Sec. 2.3, eq. (mat:f1), entries eq. (matrix) in 2D and eq. (mae:e1) in 3D) on a
 * uniform grid as A = A_hat + D^e + D^f (Sec. 3.3-3.6, eq. (dec:e1)):
 *   - A_hat, the multilevel Toeplitz part, by zero-padded embedding, forward FFT,
 *     a pointwise d x d block product with the generating-array spectra and an
 *     inverse FFT (Alg. 3 in 2D, Alg. 4 in 3D);
 *   - D^e, the incomplete-horizon diagonal (eq. (mat:se), (tea:sc));
 *   - D^f, the broken-bond correction (eq. (df), (tea:fr));
 *   - rows of constrained DOFs (Omega_c, Sec. 3.4, Remark 2) masked per DOF.
 * On top of that product it runs the static model (eq. (mat:e2)) by conjugate
 * gradients in FP64 or FP32 inside FP64 iterative refinement, the dynamic model
 * (eq. (mat:e1)) by velocity Verlet (Alg. 2), and the adjoint gradient of a static
 * solve with respect to the influence-function coefficients.
 *
 * Conventions (all entry points):
 *   - Layout: batch-major structure of arrays, [B][d][Nz][Ny][Nx], x fastest
 *     (node order of Sec. 3 and Sec. 4), B = batch cases sharing one plan.
 *   - Arrays marked "device" are HIP device pointers (for example a torch CUDA
 *     tensor's data_ptr()); arrays marked "host" are ordinary host memory.  The
 *     caller owns every array it passes; the library owns only what a plan
 *     allocates.
 *   - stream: a hipStream_t passed as void* (NULL = the default stream).  Work is
 *     enqueued on it; calls that return host results synchronise it.
 *   - Every call returns an msb_status; nothing throws across the ABI.  On a
 *     non-OK status msb_last_error() gives a message (thread-local).
 *   - A plan is not thread-safe; distinct plans are independent.
 */
#ifndef MSBFM_H
#define MSBFM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct msb_plan_s *msb_plan;

typedef enum {
    MSB_OK = 0,
    MSB_EINVAL = -1,        /* invalid argument (sizes, pointers, non-finite input, bad bond list) */
    MSB_ENOMEM = -2,        /* device or host allocation failed */
    MSB_EDEVICE = -3,       /* a HIP runtime call failed */
    MSB_ENOCONV = -4,       /* iteration limit reached or refinement stagnated */
    MSB_ENOTSPD = -5,       /* CG breakdown: p.Kp <= 0 or non-finite (singular/unconstrained problem) */
    MSB_EUNSUPPORTED = -6   /* valid request the library does not support */
} msb_status;

typedef enum {
    MSB_FP64 = 0,           /* all arithmetic in FP64 */
    MSB_FP32 = 1,           /* FFT product and vectors in FP32 */
    MSB_FP32_REFINED = 2    /* FP32 inner CG inside an FP64 iterative-refinement loop (solve only) */
} msb_precision;

/*
 * Problem description: grid (Sec. 3: x_i = x_l + (i - 1/2) h, 1-based; here
 * node (i,j,k), 0-based, sits at ((i+1/2)h, (j+1/2)h, (k+1/2)h)), horizon
 * delta = M h (Sec. 3.2, M = delta/h), micromodulus scale alpha (Sec. 2.1:
 * 9E/(pi delta^3 t) in 2D, 12E/(pi delta^4) in 3D, computed by the caller),
 * optional radial influence omega(r) = sum_k infl[k] (r/delta)^k multiplying
 * C of eq. (ker:e1) (n_infl = 0 means omega = 1, the paper's kernel), density rho
 * (eq. (mat:e1)) and the number B of load cases sharing the plan.
 */
typedef struct {
    int dim;                /* 2 or 3 */
    int64_t n[3];           /* Nx, Ny, Nz (Nz ignored in 2D); each >= 1 */
    double h;               /* grid spacing, > 0; node volume V = h^dim */
    int M;                  /* horizon in cells, 1 <= M <= 32 */
    double alpha;           /* micromodulus scale, finite */
    int n_infl;             /* 0..8 */
    const double *infl;     /* host, [n_infl], copied at plan creation */
    double rho;             /* density > 0 (dynamic model only) */
    int batch;              /* B >= 1 */
} msb_problem_desc;

/*
 * Create a plan: stencil weights of eq. (frb:e1) (lambda of eq. (fac:e1)), the
 * real spectra of the generating arrays G (Sec. 3.3, Alg. 3; Sec. 4, Alg. 4)
 * on padded lengths L >= N + M per axis, the D^e table (eq. (mat:se)), FFT
 * schedules and device workspace.  Allocates device memory on the current
 * device.  *out is NULL on failure.
 */
msb_status msb_plan_create(const msb_problem_desc *desc, msb_plan *out);
void msb_plan_destroy(msb_plan plan);

/*
 * Volume constraints, per DOF (Sec. 3.4, eq. (up); Remark 2 allows one direction
 * of a node to be constrained and another free).  fixed: host, [d][N] bytes,
 * nonzero = constrained; NULL clears all constraints.  Constrained DOFs are
 * shared by every case of the batch.
 */
msb_status msb_plan_set_constraints(msb_plan plan, const uint8_t *fixed);

/*
 * Broken bonds (bond status mu = 0, eq. (mu); correction D^f of eq. (df)).
 * pairs: host, [nb][2] node ids (p, q) with p != q, each pair once (either order),
 * both nodes in the grid and within each other's horizon.  nb = 0 clears the
 * list.  Returns MSB_EINVAL (list unchanged) on an out-of-range id, a pair
 * outside the horizon, or a duplicate.
 */
msb_status msb_plan_set_bonds(msb_plan plan, const int64_t *pairs, int64_t nb);

/*
 * Pre-crack to broken bonds for 2D problems (Sec. 3.6, Sec. 5.2): the bond {p,q}
 * is broken iff the segment [x_p, x_q] properly crosses a crack segment (both
 * orientation tests strictly of opposite sign, in FP64; touching or collinear
 * does not count).  seg: host, [ns][4] = (x0, y0, x1, y1) in the coordinates of
 * msb_problem_desc.  pairs_out: host, capacity cap pairs (p < q, sorted); *nb_out
 * receives the number found (MSB_EINVAL with *nb_out set if it exceeds cap).
 */
msb_status msb_crack_to_bonds(const msb_problem_desc *desc, const double *seg, int64_t ns,
                              int64_t *pairs_out, int64_t cap, int64_t *nb_out);

/*
 * Replace the influence coefficients (rebuilds the spectra, D^e table and bond
 * weights; same n_infl as at creation, or any count <= 8 when the plan was
 * created with n_infl > 0).  infl: host.  With per_case != 0, infl holds
 * [B][n_infl] coefficients and every case of the batch gets its own operator.
 */
msb_status msb_plan_set_infl(msb_plan plan, const double *infl, int n_infl, int per_case);

/*
 * f = A u (eq. (mat:f1)) on free DOFs, 0 on constrained DOFs (Remark 1 leaves
 * those rows arbitrary).  u, f: device, [B][d][N], double (MSB_FP64) or float
 * (MSB_FP32); u and f must not overlap.
 */
msb_status msb_apply(msb_plan plan, msb_precision prec, const void *u, void *f, void *stream);

/*
 * Same product with the operator built for omega = (r/delta)^k (the derivative of
 * A with respect to the influence coefficient a_k), FP64.  Used by the adjoint.
 */
msb_status msb_apply_dinfl(msb_plan plan, int k, const double *u, double *f, void *stream);

/*
 * The preconditioner of the preconditioned solver (msb_solve_opts.precond), applied
 * on its own: z = Pi_F E^T C^{-1} E r, where E zero-pads [d][N] to the plan's padded
 * lengths L (msb_plan_info), C = Khat + s I is the L-periodic operator with the
 * stiffness generating array (diagonal in Fourier space: per frequency the d x d block
 * Khat(k) = -Ghat(k) of the Toeplitz part of Sec. 3.2 / 4), s = 1e-3 x max over k of
 * the largest row sum of |Khat(k)|, and Pi_F zeroes constrained DOFs of the output.
 * r is read as given on constrained DOFs (the solver passes residuals that are 0
 * there).  r, z: device [B][d][N], double (MSB_FP64) or float (MSB_FP32), no overlap.
 * Cases with per-case influence coefficients use their own C.  Builds C on first use.
 */
msb_status msb_apply_precond(msb_plan plan, msb_precision prec, const void *r, void *z, void *stream);

typedef struct {
    double tol;             /* stop when ||b' - K u||_2 <= tol ||b'||_2 on free DOFs (FP64 apply) */
    int maxit;              /* cap on CG iterations (inner iterations for FP32_REFINED), > 0 */
    double inner_tol;       /* FP32_REFINED: relative residual reduction per inner solve
                               (0 = auto: 1e-4 restarted, 0.1 with reliable updates) */
    int graph_block;        /* CG iterations per hipGraph launch (0 = no graph, plain launches) */
    int reliable_update;    /* FP32_REFINED: 0 = restart CG after each FP64 residual update
                               (iterative refinement); 1 = keep the search direction and
                               replace the residual by the FP64 one (reliable updates): the
                               first beta after a replacement is the new r.r (r.z with
                               precond) over that of the step that formed the direction */
    int precond;            /* 0 = plain CG; 1 = CG preconditioned by the circulant inverse
                               of the periodic operator on the padded grid (prior fast
                               methods cited in the introduction): per frequency the d x d
                               block (Khat(k) + s I)^{-1}, Khat = -Ghat, s = 1e-3 x a bound on
                               the largest block eigenvalue; applied by the same FFT chain
                               without the D^e / D^f corrections and masked to the free DOFs.
                               Built on first use (host work like the operator's spectra),
                               freed when the influence coefficients change.  Two product
                               chains per iteration (for a plan group, two group launches:
                               every member's preconditioner chain, then every member's
                               stiffness chain). */
} msb_solve_opts;

typedef struct {
    int status;             /* msb_status of this case */
    int outer_iters;        /* refinement steps (1 for FP64) */
    int inner_iters;        /* total CG iterations */
    double rel_residual;    /* ||b' - K u|| / ||b'||, FP64 apply, free DOFs */
    double seconds;         /* wall time of the call (whole batch) */
} msb_solve_info;

/*
 * Static model, eq. (mat:e2): K = -A; solve K_FF u_F = b_F - K_FC g_C and set
 * u_C = g_C (Sec. 3.4, eq. (up)).  b: device [B][d][N] double; g: device
 * [B][d][N] double with values read on constrained DOFs only, or NULL for g = 0;
 * u: device [B][d][N] double output.  info: host [B].  Synchronises the stream.
 * MSB_ENOCONV if any case misses tol within maxit; MSB_ENOTSPD on CG breakdown.
 */
msb_status msb_solve_static(msb_plan plan, msb_precision prec, const double *b, const double *g,
                            double *u, const msb_solve_opts *opts, msb_solve_info *info,
                            void *stream);

/*
 * Dynamic model, eq. (mat:e1), by velocity Verlet (Alg. 2) with a = (A u + b)/rho:
 *   u <- u + dt v + dt^2 a / 2;  u_C <- g_C (eq. (up));  a' = (A u + b)/rho (0 on
 *   constrained DOFs);  v <- v + dt (a + a')/2 (0 on constrained DOFs);  a <- a'.
 * u, v, a: device [B][d][N] (double for MSB_FP64, float for MSB_FP32), updated in
 * place; on entry a must hold the acceleration of the entry state (msb_vv_init).
 * b: device, same type, constant in time.  g: device, same type, or NULL (= 0).
 * energy: host [nsteps/every] doubles or NULL; entry s receives, after step
 * (s+1)*every, H = rho V/2 sum v^2 - V/2 sum u (A u) - V sum b u over free DOFs,
 * accumulated in FP64 (whole batch).  Synchronises the stream when energy != NULL.
 */
msb_status msb_vv_init(msb_plan plan, msb_precision prec, const void *u, const void *b, void *a,
                       void *stream);
msb_status msb_vv_run(msb_plan plan, msb_precision prec, double dt, int64_t nsteps, void *u,
                      void *v, void *a, const void *b, const void *g, double *energy, int every,
                      void *stream);

/*
 * Quasi-static model by adaptive dynamic relaxation (Sec. 2.2, eq. (ADR:e1), Alg. 1 CDEI,
 * time step 1):
 *   v^{1/2} = D^{-1} F^0 / 2,  v^{n+1/2} = ((2 - c^n) v^{n-1/2} + 2 D^{-1} F^n) / (2 + c^n),
 *   u^{n+1} = u^n + v^{n+1/2},  F = A u + b on free DOFs (0 on constrained ones, u_C = g).
 * The fictitious density D and the damping c^n are those of the ADR method the paper
 * cites: D_ii = 1/4 sum_j |K_ij| (a Gershgorin bound of K = -A as the product applies it,
 * broken bonds and surface factors included), c^n = 2 sqrt(u^T K1 u / u^T u) over the free
 * DOFs with K1_ii = -(F^n_i - F^{n-1}_i) / (D_ii v^{n-1/2}_i) (0 where v = 0), c^n = 0 when
 * the quotient is not positive.  The fixed point is the static solution of eq. (mat:e2).
 * restart != 0: start from u (u_C set to g), build D, evaluate F^0 and take nsteps
 * updates.  restart = 0: continue from (u, v, F) with the damping sums the previous call
 * on this plan left in its workspace (same precision and launch configuration;
 * MSB_EINVAL otherwise); if the operator changed in between (coefficients, broken bonds
 * -- crack updates included --, surface factors, constraints) D is rebuilt for it; the
 * next update still uses the F given and the damping sums formed with it (the force and
 * the density before the change).
 * u, v (= v^{n-1/2}), F (= F(u^n) on return): device [B][d][N] in/out; b: device, constant;
 * g: device or NULL (= 0); all double (MSB_FP64) or float (MSB_FP32).  res: host [B] or
 * NULL: ||F||_2 of the final state per case (synchronises the stream).
 */
msb_status msb_adr_run(msb_plan plan, msb_precision prec, int64_t nsteps, int restart, void *u, void *v,
                       void *F, const void *b, const void *g, double *res, void *stream);

/*
 * Adjoint gradient of a loss of a static solution u (Sec. 2.1 kernel with
 * omega = sum_k a_k (r/delta)^k): K symmetric, so with w = K_FF^{-1} dL/du_F
 * (w from msb_solve_static on dL/du) the gradient is dL/db_F = w and
 * dL/da_k = w . (A_k u)_F, A_k the operator for omega = (r/delta)^k.
 * u, w: device [B][d][N] double; dL_da: host [B][n_infl].  Synchronises.
 */
msb_status msb_grad_infl(msb_plan plan, const double *u, const double *w, double *dL_da,
                         void *stream);

/*
 * msb_grad_infl for callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same dL/da_k =
 * w . (A_k u)_F, with the epilogue partial sums and per-case sums kept in a fixed 8 MiB
 * device array that the library holds on every GPU it runs on until the process ends,
 * instead of the plan's solver workspace.  Calls no hipMalloc or hipFree.
 *   u, w: device [B][d][N] double; dL_da: host [B][n_infl] (written on return).
 *   Needs 3 B P + n_infl B doubles of the array (P: epilogue partials per case of the
 *   plan's launch configuration); larger plans get MSB_EINVAL with the sizes in the
 *   message.  The derivative operators A_k must already exist on the plan (built by one
 *   msb_grad_infl or msb_apply_dinfl call per k), else MSB_EINVAL.  Synchronises.
 *   All calls on one GPU share the array: calls that overlap on one GPU (other host
 *   threads, other streams) race and must be serialised by the caller.
 */
msb_status msb_grad_infl_noalloc(msb_plan plan, const double *u, const double *w, double *dL_da,
                                 void *stream);

/*
 * Measurement helper: launches every kernel of the product chain nrep times back to
 * back on `stream`, with HIP events recorded between the kernels, and returns in ms[i]
 * the mean duration in milliseconds of one launch of kernel i: 2D x-forward, y line
 * product, x-inverse (*npass = 3); 3D x-forward, y-forward, z line product, y-inverse,
 * x-inverse (*npass = 5).  Then computes f = A u once (as msb_apply), so f holds the
 * product on return.  ms: host, capacity >= 5.  Synchronises the stream.
 */
msb_status msb_profile_apply(msb_plan plan, msb_precision prec, const void *u, void *f, int nrep,
                             double *ms, int *npass, void *stream);

/* Plan geometry queries (host): padded FFT lengths L[3] and the number of
 * nodes N per case. */
msb_status msb_plan_info(msb_plan plan, int64_t *L, int64_t *N, int64_t *n_bonds);

/*
 * Launch configuration of the product's kernels, one per arithmetic precision
 * (MSB_FP64 or MSB_FP32; the refined solve uses both).  It changes how the
 * work is cut into workgroups and which Stockham radices are used, never the
 * result beyond rounding order.  A plan starts with a size-based default.
 *
 *   x passes (forward and inverse transforms along x, with the prologue and
 *   the D^e / D^f / epilogue work):
 *     rows_per_wg   grid rows per workgroup, 1..16
 *     team_x        0: the whole workgroup works on each Stockham stage
 *                   (workgroup barriers); 1: every wavefront owns its own
 *                   signals (no workgroup barrier inside the transform)
 *     slots_fwd     team_x = 1: complex signals (two real rows each) per
 *     slots_inv     wavefront in the forward / inverse x pass, 1..8
 *     threads_x     team_x = 0: threads per workgroup, multiple of 64, 64..512
 *   line passes (2D: the y column transform with the block spectral product;
 *   3D: the y transforms and the z transform with the block product):
 *     lines_per_wg  lines per workgroup, 1..16
 *     team_line     as team_x
 *     lines_per_wave  team_line = 1: lines per wavefront, 1..8
 *     threads_line  team_line = 0: threads per workgroup, multiple of 64, 64..512
 *   max_radix       largest Stockham radix of the schedules: 4 (radices 2, 3,
 *                   4; with 5 where the length needs it), 8 (adds 8; 5 always) or
 *                   16 (adds 6, 9, 10, 12, 15, 16)
 *   tile            2D only.  0: the global chain above (x-forward, line product,
 *                   x-inverse).  > 0: the tiled single-pass product with frame
 *                   length tile (5-smooth, 8..64 in FP64, 8..96 in FP32; tile - 2M
 *                   >= 4).  The Toeplitz part is a correlation with a kernel of
 *                   support +-M, so the output on a block of T = tile - 2M nodes per
 *                   axis needs u only on that block grown by M (zero outside the
 *                   grid, the embedding of Sec. 3.3): one workgroup loads that
 *                   tile x tile patch, transforms it in LDS (rows, then columns),
 *                   multiplies by the spectra of the generating array wrapped to
 *                   tile x tile (Alg. 3 on the patch; both displacement components in
 *                   one complex transform), transforms back and keeps the inner
 *                   T x T block, whose D^e / D^f corrections, mask and epilogue it
 *                   applies before the one store.  One read of u, one write of f,
 *                   one launch.  A fused solver update runs first as its own
 *                   elementwise pass (the patches overlap).  The preconditioner of
 *                   the solvers always uses the global chain; plan groups run one
 *                   launch over the blocks of all members (tile_run must be 1).
 *   threads_tile    threads per workgroup of the tiled product, multiple of 64,
 *                   64..512
 *   tile_regs       0: the tiled product's frame transforms run as LDS Stockham
 *                   stages (any tile above); 1: tile 16, 32 or 64 only, each thread
 *                   keeps R points of a line in registers (tile = R S: 4 x 4, 8 x 4,
 *                   8 x 8) and a 1D transform is a radix-R butterfly, one LDS exchange
 *                   and R / S radix-S butterflies; the workgroup has S tile threads
 *                   (threads_tile is not used)
 *   tile_run        tile_regs = 1: consecutive blocks per workgroup, 1..64; a
 *                   workgroup issues the loads of its next block before it
 *                   transforms the current one (the blocks of a workgroup run one
 *                   after another, their memory and arithmetic overlapped)
 *   lds_inplace     bit 0: x passes, bit 1: line passes; a set bit runs every
 *                   Stockham stage in place (each thread reads its butterflies
 *                   into registers, a barrier, then it writes them back into the
 *                   same buffer): half the signal LDS per workgroup, one more
 *                   barrier per stage.  Valid with max_radix 16 when a schedule
 *                   uses a composite radix (6, 9, 10, 12, 15 or 16), and while no
 *                   thread owns more than max(1, 16 / R) butterflies of a
 *                   radix-R stage.
 *
 * msb_plan_set_config validates (LDS per workgroup <= 160 KiB, threads <=
 * 512) and returns MSB_EINVAL without changing the plan otherwise.
 */
typedef struct {
    int rows_per_wg, team_x, slots_fwd, slots_inv, threads_x;
    int lines_per_wg, team_line, lines_per_wave, threads_line;
    int max_radix;
    int lds_inplace;
    int tile, threads_tile;
    int tile_regs, tile_run;
} msb_launch_config;

msb_status msb_plan_get_config(msb_plan plan, msb_precision prec, msb_launch_config *cfg);
msb_status msb_plan_set_config(msb_plan plan, msb_precision prec, const msb_launch_config *cfg);

/*
 * Change the zero-padded transform lengths.  The generating array G of Sec. 3.3
 * (Alg. 3) and Sec. 4 (Alg. 4) is nonzero only for offsets |o_a| <= M, so any
 * L_a >= N_a + M, not only the paper's 2 N_a, gives the exact product.  L: host [3]; L[a]
 * for a >= dim is ignored; each must be >= N_a + M, <= 65535 and have no prime
 * factor other than 2, 3, 5.  Rebuilds the spectra and the transform
 * workspace; the launch configurations return to their defaults.  Synchronises
 * the device.
 */
msb_status msb_plan_set_lengths(msb_plan plan, const int64_t *L);

/*
 * Autotuner: times candidate launch configurations of the product f = A u for
 * `prec` (MSB_FP32_REFINED tunes both precisions) on `stream`, with every
 * kernel of the chain timed by HIP events, and keeps the fastest in the plan.
 * The search is coordinate-wise: x-pass settings (per kernel where the two x
 * kernels can differ), then line-pass settings, then max_radix (4, 8, 16), then
 * (effort 1) the x-pass and line-pass settings again with in-place stages
 * (lds_inplace), kept where they are faster.  With
 * lengths != 0 it also tries padded lengths up to 12.5% longer than the
 * default, keeping the fastest (msb_plan_set_lengths).  effort: 0 = a small
 * candidate set, 1 = full.  best: host, receives the chosen configuration of
 * `prec` (of MSB_FP32 for the refined case) or may be null; best_ms: its
 * product time in ms, or null.  Allocates two temporary product buffers on the
 * device; synchronises the stream.
 */
msb_status msb_plan_autotune(msb_plan plan, msb_precision prec, int effort, int lengths,
                             msb_launch_config *best, double *best_ms, void *stream);

/*
 * Plan groups: several plans of the same dimension (grids of different sizes, each
 * with its own batch of cases, constraints, bonds and operator) whose products run
 * as one launch per pass (2D with tile > 0: one launch of the tiled product over the
 * blocks of all members, after a transform-free pass for a fused solver update).
 * Every kernel's grid covers the tiles of all members; each workgroup finds its
 * member in a table of tile offsets and reads that member's arguments from device
 * memory.  The group's CG advances every case of every member
 * in the same launches, with per-case stop flags, and hipGraph capture of blocks of
 * iterations (graph_block) as for one plan.  For many small grids this replaces one
 * latency-bound launch chain per grid by one chain for all of them.
 *
 * msb_group_create: plans: host [nplans] (1..4096), distinct, same dimension, same
 *   device.  The group refers to the plans, which must outlive it and may still be
 *   used on their own (not concurrently with group calls on the same stream).  The
 *   common launch configuration is the largest member's when every member accepts
 *   it (its tile_run set to 1), else one row / one line per workgroup and no tiles
 *   (msb_group_set_config changes it: every member must accept the configuration,
 *   tile_run > 1 with tile > 0 is MSB_EINVAL).  A tiled configuration builds each
 *   member's frame spectra for that length.
 * msb_group_apply: f_i = A_i u_i for every member i; u, f: host arrays [nplans] of
 *   device pointers laid out as for msb_apply.  Synchronises `stream` first (the
 *   group's argument arrays are rewritten).
 * msb_group_solve_static: the static solve of msb_solve_static for every member at
 *   once: b, u: host arrays [nplans] of device pointers; g: null or such an array
 *   (entries may be null); info: host [total cases], member-major.  MSB_FP64,
 *   MSB_FP32 or MSB_FP32_REFINED (restarts, or reliable_update keeping each member's
 *   search direction, as for one plan).
 *   opts->precond = 1 preconditions every member by its own circulant inverse (each
 *   built on first use, as for one plan; the host work of the missing ones runs on
 *   parallel host threads).
 * msb_group_set_infl: msb_plan_set_infl for every member i: infl[i] holds n_infl
 *   values, or B_i x n_infl when per_case (host [nplans], or null: all shared) has
 *   per_case[i] != 0.  The members' host work (bond weights, spectra, D^e tables)
 *   runs on parallel host threads, the uploads follow in member order.  Validates
 *   every member before changing any; synchronises the device.
 * msb_group_autotune: the coordinate search of msb_plan_autotune (x passes and line
 *   passes, each with two-buffer and in-place stages, then max_radix, then in 2D the
 *   tiled product's frame lengths at one block per workgroup) over
 *   configurations every member accepts, each timed as whole group products of all
 *   members; keeps the fastest in the group (both precisions for
 *   MSB_FP32_REFINED).  best / best_ms as for msb_plan_autotune.  Allocates one input
 *   and one output vector per member for the timing; synchronises the device.  A member with the surface correction set
 *   is rejected (MSB_EUNSUPPORTED: that operator is not symmetric).
 */
typedef struct msb_group_s *msb_group;
msb_status msb_group_create(const msb_plan *plans, int nplans, msb_group *out);
void msb_group_destroy(msb_group group);
msb_status msb_group_get_config(msb_group group, msb_precision prec, msb_launch_config *cfg);
msb_status msb_group_set_config(msb_group group, msb_precision prec, const msb_launch_config *cfg);
msb_status msb_group_apply(msb_group group, msb_precision prec, const void *const *u, void *const *f,
                           void *stream);
msb_status msb_group_set_infl(msb_group group, const double *const *infl, int n_infl, const int *per_case);
msb_status msb_group_autotune(msb_group group, msb_precision prec, int effort, msb_launch_config *best,
                              double *best_ms);
msb_status msb_group_solve_static(msb_group group, msb_precision prec, const double *const *b,
                                  const double *const *g, double *const *u, const msb_solve_opts *opts,
                                  msb_solve_info *info, void *stream);

/*
 * Surface correction (Remark 3, eq. (scr)): on the rows of nodes p whose horizon leaves
 * the grid (Omega_e: within M of a face) every bond {p, q} is scaled by
 * v_pq = (nu_p + nu_q) / 2, so f_p = sum_q mu_pq v_pq A_pq (u_q - u_p) there; other rows
 * are unchanged.  The paper leaves v_pq to the cited surface-correction method; per-node
 * factors averaged over the bond are the form taken here.  nu: host [N] factors (finite,
 * > 0, shared by the cases), copied; NULL switches the correction off.  Applied as a
 * banded O(|Omega_e| (2M+1)^d) term in the product's last pass, so msb_apply, the Verlet
 * run, plan groups' products and the derivative operators of msb_apply_dinfl include
 * it.  The corrected A is not symmetric: msb_solve_static and msb_group_solve_static
 * return MSB_EUNSUPPORTED while it is on.
 */
msb_status msb_plan_set_surface(msb_plan plan, const double *nu);

/*
 * Volume factors for msb_plan_set_surface: nu_p = sum over the full discrete horizon of
 * lambda(o) / the same sum over the neighbours inside the grid, lambda the partial-volume
 * factor of eq. (fac:e1); 1 on nodes with a complete horizon.  nu: host [N] output.
 */
msb_status msb_surface_volume_factors(msb_plan plan, double *nu);

/*
 * Crack propagation, the history-dependent factor mu of eq. (mu): every bond {p, q} not
 * yet broken whose stretch s = (|x_q + u_q - x_p - u_p| - |x_q - x_p|) / |x_q - x_p|
 * (eq. (fra:s1), FP64 from u) satisfies s >= s0 breaks and joins the plan's broken set,
 * whose stiffness the D^f correction (eq. (df)) removes from every later product (the
 * paper's Phase III, Sec. 5.2).  Bonds never heal.  u: device [1][d][N], double
 * (MSB_FP64) or float (MSB_FP32).  s0 > 0 (e.g. sqrt(4 pi G0 / (9 E delta)), plane
 * stress, eq. (fra:s1)).  *n_new: bonds broken by this call.  Single-case plans only
 * (MSB_EUNSUPPORTED for batch > 1: the broken set is shared by the cases).
 * Synchronises the stream.
 */
msb_status msb_crack_update(msb_plan plan, msb_precision prec, const void *u, double s0, int64_t *n_new,
                            void *stream);

/*
 * The broken set: *count = number of broken bonds; the first min(cap, count) pairs
 * (p < q, sorted by p then q) go to pairs [cap][2] (host; may be NULL when cap = 0).
 */
msb_status msb_plan_get_bonds(msb_plan plan, int64_t *pairs, int64_t cap, int64_t *count);

/* Message for the last non-OK status on this thread ("" if none). */
const char *msb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MSBFM_H */
