/*
 * vh.h -- C ABI of the MI355X (gfx950) Vanka-smoothed shifted-Laplacian Helmholtz solver.
 *
 * Method: Yovel, He, Treister, "Vanka-smoothed Shifted Laplacian multigrid
 * preconditioners for the Helmholtz equations" (2025).  The library solves the
 * finite-difference acoustic Helmholtz equation of Sec. 1 eq. (acousitcHelm),
 *     -Lap u - omega^2 kappa^2 (1 - i gamma/omega) u = q,
 * discretised by the 2nd-order 5-point (2D) / 7-point (3D) stencil of Sec. 2.1 on a
 * nodal grid, with an absorbing layer and a first-order absorbing closure, by
 * right-preconditioned flexible GMRES(m) (Sec. 2.3).  The preconditioner is one
 * V(nu1,nu2) cycle (Sec. 2.2) on the shifted operator H_s = H + i alpha omega^2 M
 * (eq. (shift)) with Galerkin coarse operators (Sec. 3.1), the additive Vanka
 * smoother of eq. (smoother) with boundary patches and weights (Sec. 3.2, 3.3), and
 * a direct solve on the coarsest grid.
 *
 * Conventions shared by every call
 *   - Grid: n[d] nodes per dimension (n[d] - 1 cells), all nodes unknown; spacing h.
 *     Node (x, y[, z]) has linear index x + n[0]*(y + n[1]*z) (x fastest).
 *   - Complex numbers are interleaved (re, im) pairs: "c128" = two doubles,
 *     "c64" = two floats.
 *   - Every array argument is a DEVICE pointer (memory of the GPU that is current
 *     when vh_setup runs) unless the argument says "host".  The library never takes
 *     ownership of caller memory; it copies what it keeps.
 *   - Work is enqueued on the stream given in vh_options.stream (NULL = the null
 *     stream).  vh_setup and vh_solve return after their work has completed on that
 *     stream.
 *   - Every call returns a vh_status; no C++ exception crosses the ABI.  On error,
 *     vh_last_error() returns a thread-local message.
 *   - A handle is used by one host thread at a time; distinct handles may be used
 *     concurrently from different threads.
 */
#ifndef VH_H
#define VH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int vh_status;
#define VH_OK 0
#define VH_EINVAL (-1)      /* invalid argument (dims, levels, kappa <= 0, non-finite input) */
#define VH_ENOMEM (-2)      /* device allocation failed or footprint above the budget      */
#define VH_ENOCONV (-3)     /* maxit reached before tol; the last iterate is returned      */
#define VH_EBREAKDOWN (-4)  /* NaN/Inf in the Krylov recurrences                           */
#define VH_EDEVICE (-5)     /* a HIP runtime call failed                                    */
#define VH_EUNSUPPORTED (-6)/* combination of options with no kernel (see vh_setup)         */

/* Precision of the preconditioner (V-cycle).  FGMRES, the unshifted operator,
 * the true residual and the coarsest factorisation are always FP64. */
#define VH_PREC_FP64 0      /* whole V-cycle in complex128                               */
#define VH_PREC_C64 1       /* V-cycle vectors, coefficients, patch inverses in complex64 */

/* Intergrid schemes, Sec. 3.1. */
#define VH_IG_LEVDEP 0      /* eq. (level1Intergrid)/(levelDepIntergrid): cubic R,P from the finest level, then linear R / cubic P */
#define VH_IG_MIXED 1       /* linear R / cubic P on every level                      */
#define VH_IG_LINEAR 2      /* (bi/tri)linear R and P on every level (3D default)      */
#define VH_IG_CUBIC 3       /* eq. (bicubicIntergrid): cubic R and P on every level (2D) */

/* Vanka patches, Sec. 3.2 list of patches. */
#define VH_PATCH_FULL 0     /* 3x3 (2D) / 3x3x3 (3D) box around every node, truncated at the boundary */
#define VH_PATCH_POINT 1    /* 1x1 patch = damped point Jacobi (Sec. 4.1)              */
/* Sec. 3.2 patches; member order as the Fourier matrices of Sec. 4.1 (3^d box order,
 * x fastest, restricted to the members); truncated at the boundary (Sec. 3.3) except
 * ELEMENT, which is anchored at the lowest corner of every cell and has no boundary
 * patches.  Value 2 is not a patch. */
#define VH_PATCH_PLUS 3     /* node and its 2d axis neighbours (5 / 7 members)          */
#define VH_PATCH_RB 4       /* 3^d box members of the centre's red-black colour (5 / 13) */
#define VH_PATCH_ELEMENT 5  /* the 2^d corners of a cell (4 / 8)                        */

/* Boundary treatment of the finest operator. */
#define VH_BC_ABC 0         /* absorbing layer + first-order absorbing closure (default) */
#define VH_BC_DIRICHLET 1   /* no layer, missing neighbours are zero (test mode)         */

/* Smoother storage. */
#define VH_SMOOTHER_PATCH 0     /* per-patch inverses, [Np*Np][node]; block multiply + weighted overlap-add */
#define VH_SMOOTHER_ASSEMBLED 1 /* the same operator summed into a 5^d-point stencil at setup */
#define VH_SMOOTHER_SYMMETRIC 2 /* the assembled stencil stored as one half where H_s^l is
                                   complex symmetric (Sec. 3.2, 3.3: every A_c and its inverse
                                   are then symmetric): 63 (3D) / 13 (2D) entries per node, so
                                   each sweep reads about half the bytes.  H_s is symmetric
                                   for VH_STENCIL_FD2; a level keeps it while every transfer
                                   above it has R and P of one family, and the levels below
                                   a mixed transfer (VH_IG_MIXED, VH_IG_LEVDEP past the first)
                                   keep the full stencil.  Needs the Full patch on every
                                   level, VH_STENCIL_FD2, batch = 0 and the VALU contraction
                                   (VH_EUNSUPPORTED otherwise) and damping > 0; exported and
                                   sampled as the full 5^d stencil */

/* Fine-grid stencil (vh_options.stencil).
 *   FD2      : 2nd-order 5-point (2D) / 7-point (3D) stencil (Sec. 2.1); with VH_BC_ABC the
 *              absorbing layer plus a first-order absorbing closure of the boundary rows.
 *   COMPACT4 : compact 4th-order 9-point (2D) / 19-point (3D) stencil, eq. (disc4thCompact)
 *              and (disc4thCompact3D), H = L - M diag(beta) (the mass stencil acting on
 *              beta u), shift i alpha omega^2 M; stencil truncated at the boundary, with
 *              VH_BC_ABC the absorbing layer only. */
#define VH_CYCLE_V 0
#define VH_CYCLE_W 1
#define VH_STENCIL_FD2 0
#define VH_STENCIL_COMPACT4 1

/* Batched smoother contraction (vh_options.contraction).  The per-patch product
 * E_c = A_c^{-1} [r_c^(1..S)] of eq. (smoother) for S >= 16 sources sharing a sweep:
 *   VALU        complex64 FMAs on the vector ALUs (every configuration)
 *   MFMA_F32    real-embedded [S x 18] . [18 x 18] products on the matrix cores, FP32
 *   MFMA_BF16X3 the same in split BF16 (hi*hi + hi*lo + lo*hi), FP32 accumulation;
 *               about 2^-16 relative error per product on top of complex64 rounding. */
#define VH_CONTRACT_VALU 0
#define VH_CONTRACT_MFMA_F32 1
#define VH_CONTRACT_MFMA_BF16X3 2

typedef struct vh_options {
    int precision;          /* VH_PREC_*; default VH_PREC_FP64                         */
    int restart;            /* FGMRES restart length m; default 20                     */
    int maxit;              /* total preconditioner applications; default 1000         */
    int nu1, nu2;           /* pre/post smoothing steps; default 1, 1                  */
    int intergrid;          /* VH_IG_*; default VH_IG_LEVDEP (2D), VH_IG_LINEAR (3D) when -1 */
    int bc;                 /* VH_BC_*; default VH_BC_ABC                              */
    int sponge_width;       /* absorbing-layer width in cells; default 20              */
    double sponge_amp;      /* layer attenuation at the face, in units of omega; default 1 */
    int smoother;           /* VH_SMOOTHER_*; default VH_SMOOTHER_PATCH                */
    int ndamping;           /* number of valid entries in damping[]; 0 = defaults      */
    double damping[16];     /* w_l for level l = 0 (finest) ...; the last one repeats   */
    void *stream;           /* hipStream_t; NULL = null stream                         */
    int timing;             /* 1: vh_solve brackets every V-cycle and every finest-level
                               smoothing launch with HIP events on `stream` and reports the
                               summed durations in vh_solve_stats; default 0              */
    int batch;              /* 0: vh_solve handles the sources one after another (default);
                               1: in groups of up to 64 sources that share every V-cycle
                               sweep (each coefficient and patch-inverse entry is read once
                               per group), each source with its own FP64 FGMRES state    */
    int stencil;            /* VH_STENCIL_*; default VH_STENCIL_FD2                     */
    int fine_patch;         /* VH_PATCH_* of the finest level's smoother, or -1 (default)
                               for the patch of vh_setup on every level.  Sec. 5.5, Sec. 6:
                               damped Jacobi (VH_PATCH_POINT) on the fine level with
                               Element-patch Vanka below                                  */
    int cycle;              /* VH_CYCLE_V (default) or VH_CYCLE_W (Sec. 2.2: the coarse
                               correction visits each coarser level twice, except the
                               coarsest, solved directly)                                */
    int contraction;        /* VH_CONTRACT_*: how a batch of >= 16 sources applies the
                               per-patch smoother (2D, Full patch, VH_SMOOTHER_PATCH,
                               VH_PREC_C64 only; VH_EUNSUPPORTED otherwise); default VALU */
    int sweep_tile;         /* variant of the 64-source 2D sweep of the assembled smoother
                               and of the 64-source stencil (batch = 1, VALU contraction):
                               0 (default) = the fastest of the 10 variants, timed on each
                               level's grid at the first 64-source solve and kept for the
                               process; 1..10 forces one.  The variants give identical
                               results */
    int split_residual;     /* where the residual q - A u is formed: inside the kernel
                               that consumes it (the 2D smoothing sweep, Sec. 3.2 eq.
                               (smoother); the restriction of the two-grid cycle, Sec. 2.2,
                               2D and 3D-trilinear), so that it is never stored, or by a
                               separate residual launch.  0 (default): per level, timed at
                               setup on the level's own grid (the one-launch form when it
                               is at least 5 % faster) and kept for the process; 1: always
                               separate; 2: inside wherever such a kernel exists.  Results
                               are identical bit for bit */
    int sym_planes;         /* 3D symmetric-half sweep (VH_SMOOTHER_SYMMETRIC): how many
                               z-planes one workgroup walks, reading the entries of each
                               plane once for its own terms and, from the caches, for the
                               mirrored terms of the planes above.  0 (default): 6 where
                               the level still gets >= 1024 workgroups, else one plane per
                               workgroup; -1: one plane per workgroup; 2..64 forced (a
                               walked level keeps a small carry buffer: two planes per
                               chunk boundary).  The forms agree to rounding (they sum
                               in different orders)                                      */
    int setup_pivot;        /* patch inversion (Sec. 3.2): 0 (default) eliminates in the
                               natural order without pivoting where the patch matrices are
                               complex symmetric with a positive definite imaginary part
                               (5/7-point operator, transfers with R = c P^T, shift > 0, Full
                               patch), else with partial pivoting; 1: partial pivoting on
                               every level.  The two agree to rounding                   */
} vh_options;

typedef struct vh_solve_stats {
    int iterations;         /* preconditioner applications (summed over restarts)      */
    int restarts;
    int converged;          /* 1 when the true relative residual <= tol                */
    double relres;          /* true ||q - H u|| / ||q||, FP64                          */
    double relres_est;      /* Arnoldi estimate at exit                                */
    double solve_ms;        /* wall time of the solve on the stream (HIP events)       */
    /* filled when vh_options.timing = 1 (zero otherwise):                              */
    int vcycles;            /* V-cycle applications                                     */
    double vcycle_ms;       /* their summed duration                                    */
    int smooth0_launches;   /* finest-level smoothing launches from u = 0 (u = B q)     */
    double smooth0_ms;
    int smooth1_launches;   /* finest-level smoothing launches u += B r                 */
    double smooth1_ms;
    /* always filled:                                                                   */
    double setup_ms;        /* wall time of the vh_setup that built the handle          */
    double bytes_moved;     /* algorithmic device bytes of the solve's kernels: every
                               array a kernel reads or writes counted once per launch
                               (the 5/7-point finest operator as its centre entries);
                               sources solved together in one batch (opt.batch = 1)
                               report the batch's total                                 */
    double c_f;             /* convergence factor of eq. (cf) (Sec. 5.1) on the residual
                               estimates: (r_k / r_5)^(1/(k-5)) after k iterations, the
                               first 5 as warm-up; NaN when k <= 5                        */
} vh_solve_stats;

typedef struct vh_level_info {
    int n[3];               /* nodes per dimension (n[2] = 1 in 2D)                    */
    int stencil_points;     /* K: coefficients per node of the level operator          */
    int smoother_entries;   /* Np*Np (patch form) or 5^d (assembled) per node          */
    int offsets[125][3];    /* stencil offsets, K used entries                          */
    size_t bytes;           /* device bytes owned by this level                        */
    int mfma_sources;       /* batch width the matrix-core sweep was tuned for (0: none) */
    int mfma_tile;          /* patches per strip row chosen by the tuner (16 or 32)      */
    int mfma_rows;          /* rows per block chosen by the tuner                        */
    int sweep_tile;         /* variant of the 64-source 2D sweep in use (0: none chosen)  */
    int fused_sweep;        /* 1: the level's smoothing steps form the residual in the sweep */
    int fused_restrict;     /* 1: the restriction to the next level forms the residual    */
    int sym_planes;         /* 3D symmetric half: z-planes one workgroup of the level's
                               sweep walks (0: not symmetric, or one plane per workgroup) */
    int setup_pivot;        /* 1: the level's patch inverses used partial pivoting       */
} vh_level_info;

typedef struct vh_handle vh_handle;

/* Fills *opt with the defaults listed above. */
void vh_options_default(vh_options *opt);

const char *vh_status_string(vh_status s);
const char *vh_last_error(void);

/* vh_setup -- build the whole preconditioner on the device (Sec. 2.3, 3.1, 3.2, 3.3).
 *   out     : host pointer receiving the new handle.
 *   dim     : 2 or 3.
 *   n       : host array of dim node counts, each >= 3; (n[d]-1) must be divisible by
 *             2^(levels-1) and every level must keep >= 3 nodes per dimension.
 *   h       : grid spacing (> 0).   omega : angular frequency (>= 0).
 *   kappa   : device, float64[N], slowness > 0 (N = prod n).
 *   gamma   : device, float64[N], physical attenuation >= 0, or NULL for zero.
 *   shift   : alpha of eq. (shift) (>= 0).
 *   levels  : number of multigrid levels (>= 1; 1 = direct solve only).
 *   patch   : VH_PATCH_*.
 *   opt     : host, or NULL for defaults.
 * Builds: finest H (FP64) and H_s; Galerkin H_s^l = R H_s^{l-1} P; every patch inverse
 * of every non-coarsest level (batched FP64 Gauss-Jordan, stored at the preconditioner
 * precision with the weights w_l / cnt folded in); the FP64 inverse of the coarsest
 * H_s^L.  Returns VH_EINVAL for bad arguments (checked before any allocation),
 * VH_EUNSUPPORTED for an intergrid/dimension pair without kernels, VH_ENOMEM if an
 * allocation fails (nothing is leaked). */
vh_status vh_setup(vh_handle **out, int dim, const int *n, double h, double omega,
                   const double *kappa, const double *gamma, double shift, int levels,
                   int patch, const vh_options *opt);

/* vh_solve -- FGMRES(m) (Sec. 2.3) preconditioned by one V-cycle, from u = 0.
 *   q     : device, c128[nsrc][N], right-hand sides (source-major).
 *   nsrc  : number of right-hand sides (>= 1), solved one after another.
 *   tol   : relative residual target (> 0), checked on the true FP64 residual.
 *   u     : device, c128[nsrc][N], output (may not alias q).
 *   stats : host array of nsrc entries, or NULL.
 * Returns VH_ENOCONV if some source did not reach tol within maxit (u holds the last
 * iterate), VH_EBREAKDOWN on NaN/Inf. */
vh_status vh_solve(vh_handle *hd, const void *q, int nsrc, double tol, void *u,
                   vh_solve_stats *stats);

/* vh_destroy -- frees every device allocation of the handle.  NULL is allowed. */
vh_status vh_destroy(vh_handle *hd);

/* ---- inspection hooks (used by the parity tests) ----------------------------- */

int vh_num_levels(const vh_handle *hd);

/* Device bytes the handle holds now (*in_use) and the most it has held at any time
 * since vh_setup began (*peak), both HOST outputs (either may be NULL).  vh_footprint_bytes
 * with the handle's arguments is an upper bound of *peak. */
vh_status vh_get_memory(const vh_handle *hd, size_t *in_use, size_t *peak);
vh_status vh_get_level_info(const vh_handle *hd, int level, vh_level_info *info);

/* y = A x on level `level` (0 = finest): which = 0 -> unshifted H (finest only, FP64),
 * which = 1 -> H_s^level at the preconditioner precision.  x, y: device c128[N_level]. */
vh_status vh_apply_operator(vh_handle *hd, int level, int which, const void *x, void *y);

/* z = M^{-1} v: one V-cycle from zero, v and z device c128[N]. */
vh_status vh_apply_vcycle(vh_handle *hd, const void *v, void *z);

/* u <- u + B_l (q - A_l u) on level l (one damped smoothing step, eq. (smoother));
 * q, u device c128[N_l]. */
vh_status vh_apply_smoother(vh_handle *hd, int level, const void *q, void *u);

/* The multi-source forms of the two hooks above, through the batched kernels that
 * vh_solve uses with vh_options.batch = 1 (and vh_options.contraction):
 *   q, u, v, z : device c128[nsrc][N_l] (source-major, as in vh_solve), 1 <= nsrc <= 64.
 * vh_apply_smoother_batch: u_s <- u_s + B_l (q_s - A_l u_s) for every source s;
 * vh_apply_vcycle_batch:   z_s = M^{-1} v_s (one V-cycle from zero) for every source. */
vh_status vh_apply_smoother_batch(vh_handle *hd, int level, int nsrc, const void *q, void *u);
vh_status vh_apply_vcycle_batch(vh_handle *hd, int nsrc, const void *v, void *z);

/* Copies level data to HOST buffers (each may be NULL):
 *   coef : c128[K][N]  operator coefficients (H_s^level)
 *   smoother : c128[E][N] smoother entries (E = smoother_entries), weights folded in
 *   coarse_inv : c128[N][N] inverse of the coarsest operator (coarsest level only). */
vh_status vh_export_level(const vh_handle *hd, int level, void *coef, void *smoother,
                          void *coarse_inv);

/* Copies the entries of sampled nodes of level `level` to a HOST buffer:
 *   which = 0 -> operator coefficients (K per node, order of vh_level_info.offsets),
 *   which = 1 -> smoother entries (E per node, weights folded in);
 *   nodes : HOST int64[count], linear node indices (< N_level);
 *   out   : HOST c128[count][K or E].  VH_EINVAL for out-of-range nodes. */
vh_status vh_sample_level(const vh_handle *hd, int level, int which, int count,
                          const int64_t *nodes, void *out);

/* Device bytes a handle holds after vh_setup plus the workspace vh_solve adds for
 * nsrc sources (the multi-source workspace when opt->batch = 1), excluding the
 * caller's arrays; 0 for invalid grids.  Pure function of its arguments (no device
 * call), used for admission by footprint. */
size_t vh_footprint_bytes(int dim, const int *n, int levels, int patch, int nsrc,
                          const vh_options *opt);

/* ---- parameter selection: local Fourier analysis, convergence factor, tuners ------ */

/* Local Fourier analysis of one smoother on an infinite grid with constant coefficients
 * (Sec. 2.4, Sec. 4).  The interior stencil A of the operator is the 5/7-point stencil
 * (VH_STENCIL_FD2) or the compact one (VH_STENCIL_COMPACT4) for sigma = omega^2 kappa^2
 * (no attenuation), plus i*shift times the mass stencil.  For a patch with members o_k
 * (vh.h patch order) the smoother symbol is eq. (smoother_symbol),
 *     S(theta) = 1 - w * (phi^H A_i^{-1} phi / Np) * A(theta),  phi_k = exp(i theta.o_k),
 * with A_i the patch matrix of the stencil.  theta runs over npts^dim samples
 * theta_k = -pi/2 + 2 pi k / npts of [-pi/2, 3pi/2)^dim.
 *   mu(w)  = max |S(theta)| over the high frequencies (Definition "def_mu_loc");
 *   rho(w) = max spectral radius of the two-grid symbol of eq. (symbolTG),
 *            S^nu2 (I - P H_c^{-1} R A) S^nu1 on the 2^dim harmonics of every low
 *            frequency theta != 0, with H_c = sum_h R(theta_h) A(theta_h) P(theta_h)
 *            (Galerkin) and the restriction / prolongation symbols of the 1D
 *            families (Definition "def_rho_loc", Sec. 4.2).
 * All of it runs on the device in FP64. */
typedef struct vh_lfa_problem {
    int dim;                 /* 2 or 3                                                   */
    int stencil;             /* VH_STENCIL_FD2 or VH_STENCIL_COMPACT4                     */
    int patch;               /* VH_PATCH_*                                               */
    double h;                /* grid spacing (> 0)                                       */
    double sigma;            /* omega^2 kappa^2 (>= 0)                                   */
    double shift;            /* imaginary shift alpha omega^2 of the mass term (>= 0)    */
    int rfam, pfam;          /* VH_IG_LINEAR or VH_IG_CUBIC: 1D restriction / prolongation
                                weights (1/4)[1 2 1] or (1/16)[1 4 6 4 1]; default cubic  */
    int npts;                /* samples per dimension: even, <= 512 (2D) / <= 128 (3D);
                                default 256 (2D), 64 (3D)                                 */
    int nu1, nu2;            /* smoothing steps of the two-grid cycle; default 1, 1       */
    void *stream;            /* hipStream_t, NULL = the null stream                       */
} vh_lfa_problem;

void vh_lfa_problem_default(vh_lfa_problem *p);

/* mu[j] = mu(w[j]), rho[j] = rho(w[j]) for the nw damping values w (HOST arrays; mu or
 * rho may be NULL to skip that factor).  VH_EINVAL for bad fields or nw < 1. */
vh_status vh_lfa_factors(const vh_lfa_problem *p, int nw, const double *w, double *mu,
                         double *rho);

/* vh_lfa_factors_noalloc -- the same factors as vh_lfa_factors, computed by the same
 * kernels, for callers that cannot allocate device memory: code under HIP graph capture,
 * serving loops that must not call hipMalloc/hipFree, harnesses that forbid allocation.
 * It calls no hipMalloc, hipFree, hipHostMalloc or other allocating routine.  Its work
 * arrays (per-sample symbols, damping values, block maxima, factors) live in one
 * statically allocated 16 MiB device array per GPU, held until the process ends; the
 * limit admits npts^dim <= 2^18 samples (every 2D npts, 3D npts <= 64) with nw <= 1024,
 * and a problem that needs more returns VH_EINVAL before any device work.  Arguments,
 * layout (mu, rho, w are HOST arrays of nw) and other errors as vh_lfa_factors; p->stream
 * must belong to the current device.  Every call on one GPU shares that GPU's array
 * (nothing in it needs to start at zero; each call writes what it reads): calls that
 * overlap on one GPU, from different threads or on different streams, race. */
vh_status vh_lfa_factors_noalloc(const vh_lfa_problem *p, int nw, const double *w, double *mu,
                                 double *rho);

/* LFA damping tuner (Sec. 5.2: the fine-level damping is the minimiser of the LFA
 * factor): evaluates objective 0 = mu, 1 = rho on the nw candidates w (HOST) and
 * returns the first minimiser in *w_best and its factor in *f_best (HOST). */
vh_status vh_lfa_tune(const vh_lfa_problem *p, int objective, int nw, const double *w,
                      double *w_best, double *f_best);

/* The cycle as a stationary solver (Sec. 5.1, eq. (cf)): from x = 0,
 *     x <- x + M^{-1} (q - A x)
 * with A = H (which = 0, FP64) or A = H_s (which = 1; handles built with VH_PREC_FP64
 * only, else VH_EUNSUPPORTED), until ||q - A x|| <= tol ||q|| or maxit cycles, or
 * until the residual exceeds 1e12 ||q|| (divergence).
 *   q, x : device c128[N] (x receives the last iterate; may not alias q).
 *   hist : HOST double[maxit + 1] or NULL, ||r^(k)|| / ||q|| for k = 0..iterations.
 * The convergence factor is c_f = (||r^(k)|| / ||r^(warmup)||)^(1/(k - warmup)) at the
 * last k (NaN when k <= warmup). */
typedef struct vh_cf_stats {
    int iterations;          /* cycles applied                                           */
    int converged;           /* 1 when tol was reached                                   */
    double relres;           /* ||q - A x|| / ||q|| at exit                              */
    double cf;               /* c_f of eq. (cf)                                          */
} vh_cf_stats;

vh_status vh_mg_iterate(vh_handle *hd, int which, const void *q, void *x, int warmup,
                        int maxit, double tol, double *hist, vh_cf_stats *stats);

/* Per-level damping by exhaustive search (Sec. 5.2): for l = 0 .. levels-2 in turn,
 * each candidate w[j] (HOST, nw values) is tried as w_l with w_0..w_{l-1} fixed at the
 * values already chosen and the deeper levels at opt's values (or the defaults); a
 * handle is built with vh_setup's arguments (shift, levels, patch, opt) and scored by
 *   objective 0: FGMRES iterations to tol (vh_solve; maxit + 1 if not converged),
 *   objective 1: c_f of vh_mg_iterate(which = 1, warmup, maxit, tol) (inf if the cycle
 *                does not run warmup + 1 steps).
 * The first minimiser is kept.  q: device c128[N], the source.  damping: HOST
 * double[levels-1] receives the chosen w_l; scores: HOST double[(levels-1)*nw] or NULL,
 * score of candidate j on level l at scores[l*nw + j].  opt->precision is forced to
 * VH_PREC_FP64 when objective = 1. */
vh_status vh_tune_damping(int dim, const int *n, double h, double omega, const double *kappa,
                          const double *gamma, double shift, int levels, int patch,
                          const vh_options *opt, const void *q, int objective, int warmup,
                          int maxit, double tol, int nw, const double *w, double *damping,
                          double *scores);

/* Shift selection (Sec. 5.2, 5.5): the smallest alpha among the na candidates alphas
 * (HOST, increasing) for which the cycle on H_s converges as a stationary solver
 * (c_f of vh_mg_iterate(which = 1, warmup, maxit, tol) below 1, or tol reached), on the
 * problem given by vh_setup's arguments.  *alpha (HOST) receives it; cfs: HOST
 * double[na] or NULL receives every candidate's c_f (tried in order, NaN after the
 * chosen one).  VH_ENOCONV if no candidate converges. */
vh_status vh_tune_shift(int dim, const int *n, double h, double omega, const double *kappa,
                        const double *gamma, int levels, int patch, const vh_options *opt,
                        const void *q, int na, const double *alphas, int warmup, int maxit,
                        double tol, double *alpha, double *cfs);

/* ---- serving: persistent request loop with admission by HBM footprint ----------
 * Requests are copied at submission and queued.  vh_server_create allocates one device
 * arena of hbm_budget bytes; a request runs in a contiguous region of it that holds its
 * kappa, gamma, q and u arrays and its whole handle at its peak (vh_footprint_bytes plus
 * alignment), so no request allocates or frees device memory while others run.  Up to
 * max_slots requests run at once, each on its own worker thread and HIP stream (default
 * priority); a queued request is admitted as soon as a slot and a free region of its
 * size are available (first fit).  Later requests may overtake a queued head that does
 * not fit at most a bounded number of times.  Each request runs vh_setup + vh_solve on a
 * handle of its own, so its result does not depend on the other requests in flight.
 * Results are held until fetched with vh_server_result.  The server uses the device that
 * is current when it is created. */
typedef struct vh_server vh_server;

typedef struct vh_request {
    int dim;                 /* 2 or 3                                                   */
    int n[3];                /* nodes per dimension                                      */
    double h, omega;         /* grid spacing, angular frequency                          */
    const double *kappa;     /* HOST, float64[N], copied at submission                   */
    const double *gamma;     /* HOST, float64[N] or NULL, copied                          */
    double shift;            /* alpha of eq. (shift)                                     */
    int levels, patch;       /* as in vh_setup                                           */
    const void *q;           /* HOST, c128[nsrc][N], copied                              */
    int nsrc;                /* sources (>= 1)                                           */
    double tol;              /* relative residual target                                 */
    const vh_options *opt;   /* NULL = defaults; the stream field is ignored             */
} vh_request;

typedef struct vh_server_info {
    size_t budget, in_use, peak_in_use;  /* bytes                                        */
    int running, peak_running, queued;
    uint64_t completed;
} vh_server_info;

/* VH_ENOMEM if the arena of hbm_budget bytes cannot be allocated; max_slots in [1, 64]. */
vh_status vh_server_create(vh_server **out, size_t hbm_budget, int max_slots);
/* VH_ENOMEM if the request alone exceeds the budget, VH_EINVAL for bad requests. */
vh_status vh_server_submit(vh_server *srv, const vh_request *req, uint64_t *ticket);
vh_status vh_server_poll(vh_server *srv, uint64_t ticket, int *done);
vh_status vh_server_wait(vh_server *srv, uint64_t ticket);
/* Waits for the request, copies its solution to u (HOST c128[nsrc][N], may be NULL)
 * and its stats (array of nsrc, may be NULL), reports latency (submission ->
 * completion) and queueing time in ms, releases the ticket, and returns the
 * request's own vh_solve status. */
vh_status vh_server_result(vh_server *srv, uint64_t ticket, void *u, vh_solve_stats *stats,
                           double *latency_ms, double *queue_ms);
vh_status vh_server_get_info(vh_server *srv, vh_server_info *info);
/* Finishes every submitted request, then stops the workers and frees the server
 * (unfetched results are discarded). */
vh_status vh_server_destroy(vh_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* VH_H */
