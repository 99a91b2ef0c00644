/*
 * admm.h -- C ABI of the MI355X (gfx950) ADMM micromechanics library.
 *
 * The library runs the operator-splitting method of Zhou & Bhattacharya,
 * "Accelerated computational micromechanics" (arXiv 2010.06697), on periodic
 * voxel grids: the incremental variational problem written with an augmented
 * Lagrangian (Sec. 2.1) and solved by ADMM, one iteration being
 *   Step 1  local problem      F <- argmin W(F) + rho/2 |F - grad u - Lambda/rho|^2
 *   Step 2  Helmholtz projection of F - Lambda/rho onto gradients, by FFT with
 *           central-difference symbols (Sec. 2.3)
 *   Step 3  multiplier update  Lambda <- Lambda + rho (grad u - F)
 *   Step 4  primal / dual residuals r_p, r_d and the convergence test,
 *           then the adaptive penalty rule (Sec. 2.1, "Penalty parameter").
 * Every step runs in the library's HIP kernels; the host only launches them.
 *
 * Conventions
 *   - Grid n1 x n2 x n3 (each even, 4..256, of the form 2^a 3^b; n3 = 1 is
 *     also allowed: plane strain, every field independent of x3), spacing 1.
 *     Voxel (k1,k2,k3) has linear index (k3*n2 + k2)*n1 + k1 (x1 fastest);
 *     V = n1*n2*n3.
 *   - Fields are structure-of-arrays, component-major: a 3-vector field is
 *     3*V scalars, component i at [i*V + idx]; a 3x3 tensor field is 9*V
 *     scalars, component (i,J) at [(3*i+J)*V + idx] (row-major F_iJ).
 *   - Scalar type: double in ADMM_FP64, float in ADMM_FP32_FP64RED, except
 *     the displacement fluctuation u (and u_prev), which is double in both.
 *   - u is the periodic displacement fluctuation (grad u = Fbar + D_h u).
 *   - The deformation-gradient field stores E = F - I (both precisions).
 *   - All field pointers are DEVICE pointers owned by the caller; the library
 *     never frees them. The context owns only its own metadata and the small
 *     device tables it allocates in admm_init.
 *   - Functions never throw; they return an admm_status code. On an error
 *     return (< 0) the state is left as it was, except ADMM_EDOMAIN and
 *     ADMM_EDIVERGED, which leave the last iterate and mark the offending
 *     cell.
 *   - A context is bound to one HIP stream and is not thread safe. Work is
 *     enqueued on that stream; calls returning host scalars synchronise it.
 */
#ifndef ADMM_H
#define ADMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ADMM_OK = 0,
  ADMM_NOT_CONVERGED = 1, /* result valid; iteration cap reached */
  ADMM_EINVAL = -1,       /* invalid argument */
  ADMM_EUNSUPPORTED = -2, /* grid size or model not supported */
  ADMM_EHIP = -3,         /* HIP runtime error */
  ADMM_ENOMEM = -4,       /* workspace too small / allocation failed */
  ADMM_EDOMAIN = -5,      /* det F <= 0 or NaN met in a cell */
  ADMM_EDIVERGED = -6,    /* residuals grew or stagnated (admm_solve's
                             divergence watch); the last iterate is kept */
  ADMM_ENOGPU = -7        /* no HIP device */
} admm_status;

typedef enum {
  ADMM_FP64 = 0,         /* everything in double precision */
  ADMM_FP32_FP64RED = 1  /* float F, Lambda, FFT and Newton; double u, det F /
                            ln J, residual norms, averages and convergence
                            test. Step 2 solves for the correction
                            u_{i+1} - u_i (its right-hand side, the defect
                            D_h^T(F - Lambda/rho - D_h u_i), formed in double)
                            so that the float transforms' rounding scales
                            with the correction and not with u */
} admm_precision;

typedef enum {
  ADMM_NEOHOOKE = 0, /* W = mu/2 (|F|^2 - 3) - mu ln J + lambda/2 (ln J)^2 */
  ADMM_LCE = 1       /* W = mu/2 [a^(1/3)(|F|^2 + (1/a - 1)|F^T n|^2) - 3]
                            + kappa/2 (J - 1)^2, director n per voxel
                        (neo-classical energy of Sec. 5.1 with step-length
                        tensor a^(-1/3)(I + (a-1) n n), a >= 1, and a
                        volumetric penalty). The local problem minimises over
                        F and the unit director jointly: the director is
                        eliminated (top eigenvector of F F^T, double precision,
                        unit length) and Newton's method runs on the relaxed
                        energy, with a multiple of the identity added to its
                        Hessian where that is not positive definite, down to
                        a stationary point of the joint problem. */
} admm_model;

/* One phase of the material table. */
typedef struct {
  int32_t model; /* admm_model */
  int32_t reserved;
  double mu, lambda; /* neo-Hookean moduli */
  double a, kappa;   /* LCE: step-length ratio (>= 1), volumetric penalty */
  /* The rest of Sec. 5.1's LCE model (0 = off; each needs a > 1):
   *   alpha: non-ideality mu alpha/2 tr((I - n0 n0) F^T (n n) F) with the
   *          voxel's cross-link director n0 (admm_rve.director0);
   *   frank: Frank constant kappa_F of kappa_F/2 |grad(n (x) n)|^2 with
   *          forward differences between neighbouring LCE voxels (lengths
   *          in voxels), the neighbours' directors taken from the previous
   *          iteration;
   *   nu_n:  director dissipation nu_n/(2 dt)(1 - (n . n^n)^2), n^n the
   *          director at the start of the load step.
   * nu_F (any model): dissipation nu_F/(2 dt)|F - F^n|^2, F^n the field at
   * the start of the load step. The library keeps the start-of-step copies
   * (and the previous iteration's directors for the Frank term) in device
   * memory it allocates at admm_init. */
  double alpha, frank, nu_F, nu_n;
} admm_material;

/* One periodic cell (representative volume element). Pointers: device. */
typedef struct {
  int32_t n[3];          /* n1, n2, n3 */
  int32_t reserved;
  const uint8_t *phase;  /* V bytes, index into the material table */
  void *u;               /* 3V doubles: displacement fluctuation (in/out) */
  void *u_prev;          /* 3V doubles: second buffer the library iterates into */
  void *F;               /* 9V: F - I (in/out) */
  void *Lambda;          /* 9V: multiplier (in/out) */
  void *director;        /* 3V unit director (in/out; required when a phase
                            is ADMM_LCE, else may be NULL) */
  const void *director0; /* 3V unit cross-link director n0 of the
                            non-ideality (read only; required when a phase
                            has alpha > 0, else may be NULL) */
  double Fbar[9];        /* macroscopic gradient <F>, row-major, det > 0 */
} admm_rve;

/* Iteration parameters (Sec. 2.1; defaults in parentheses). */
typedef struct {
  double rho0;          /* initial penalty (10) */
  double rho_min;       /* lower clamp of the adaptive rule (1) */
  double rho_max;       /* upper clamp (50) */
  double kappa_rho;     /* adaptive factor kappa (1.3) */
  double tau;           /* adaptive ratio threshold tau (10) */
  double tol_p, tol_d;  /* primal / dual tolerances */
  double mu_ref;        /* representative modulus in r_d */
  double newton_gtol;   /* local Newton: stop when |grad| <= gtol * (mu + lambda
                           + rho)(1 + |F| + |A|) (1e-14 FP64, 1e-10 FP32) */
  double newton_step_tol; /* local Newton: stop after a full Newton step
                           |dF| <= step_tol * max(1, |F|) (1e-10 FP64, 2e-6 FP32) */
  int32_t adapt_rho;    /* 1: adaptive penalty after each test */
  int32_t max_iter;     /* iteration cap of admm_solve */
  int32_t check_every;  /* admm_solve: iterations between host checks; also
                           the length of the captured graph (10) */
  int32_t newton_max;   /* local Newton iteration cap (100). In
                           ADMM_FP32_FP64RED without an inexact strategy the
                           neo-Hookean local problem is solved in closed form
                           up to one scalar (the minimiser is coaxial with the
                           data; Sec. 2.1, Step 1), whose Newton iteration this
                           also caps; newton_gtol and newton_step_tol apply
                           where that form does not (det of the data <= 0),
                           to the LCE and to the double precision mode. */
  int32_t use_graph;    /* 1: admm_step / admm_solve replay check_every
                           iterations as one captured hipGraph (built on
                           first use, kept by the context); 0: launch every
                           kernel. Profiling (admm_profile_enable) launches
                           every kernel. (1) */
  int32_t reserved;
  /* Inexact local step (Sec. 2.1, local residual r_l; Sec. 4, the two
   * strategies compared there). Step 1 runs in passes of at most local_chunk
   * Newton iterations per voxel, each pass continuing from the previous
   * iterate (F and, for the LCE, the director), until the pass's test holds
   * or local_passes passes ran. r_l is reduced inside the local kernel (one
   * partial sum per workgroup) and tested on the device; the host is not
   * involved. At most one of local_ratio and local_fraction is nonzero; both
   * zero: every local problem solved to the Newton tolerances. The ideal
   * LCE's local problem (three unknowns in the singular basis of A) is solved
   * in full in every pass, at most max(local_chunk, newton_max, 100)
   * iterations: it costs less than the passes a truncated solve would need
   * (each rebuilds the singular basis). With either
   * strategy, admm_solve counts a cell as converged only when r_l <= tol_d
   * as well (equilibrium needs the local residual small too). */
  double local_ratio;   /* > 0: from the second iteration of a load step,
                           stop once r_l = |P(F) - Lambda - rho (grad u - F)|
                           / mu_ref (RMS over the cell) <= local_ratio * r_d
                           of the previous iteration (0) */
  int32_t local_chunk;  /* Newton iterations per voxel and pass (1) */
  int32_t local_passes; /* passes per iteration at most (8) */
  double local_fraction; /* in (0, 1]: every iteration, stop once the local
                           Newton solves (their own stopping rule) have
                           converged at >= local_fraction of the voxels (0) */
  double dt;            /* time step of a load step, for the dissipation
                           terms (admm_material nu_F, nu_n) (1) */
  /* Divergence watch of admm_solve (Sec. 4 reports that too small a penalty
   * diverges; the method itself has no test for it). After each iteration's
   * convergence test, with merit = max(r_p / tol_p, r_d / tol_d), a cell
   * stops with ADMM_EDIVERGED when the merit exceeds div_growth times the
   * smallest merit of its load step, or when the merit has not halved for
   * stall_iters iterations. 0 switches either rule off. admm_step (a fixed
   * count) does not watch. */
  double div_growth;    /* (1e3) */
  int32_t stall_iters;  /* (500) */
  int32_t reserved2;
} admm_params;

typedef struct admm_ctx admm_ctx;

/* Validates one grid (host only, no GPU needed): ADMM_OK, ADMM_EINVAL
 * (non-positive) or ADMM_EUNSUPPORTED (odd, outside 4..256, not 2^a 3^b;
 * n3 = 1, plane strain, is supported, n1 = 1 or n2 = 1 is not). */
int admm_check_grid(int32_t n1, int32_t n2, int32_t n3);

/* Device workspace the library needs for these cells and precision (bytes):
 * the half-spectrum buffers of Step 2, three components of n3 * n2 rows per
 * cell, each row n1/2 + 1 complex values padded to 32 bytes (2 complex128 or
 * 4 complex64), 256-byte aligned per cell; in ADMM_FP32_FP64RED also the
 * correction of Step 2 (3V floats, 256-byte aligned) after each cell's
 * spectra. The context owns the buffer for its lifetime. Host only. Returns
 * 0 on invalid input. */
size_t admm_workspace_bytes(const admm_rve *rves, int32_t n_rve, int32_t precision);

/* Creates a context for n_rve cells sharing one material table.
 *   rves, mats, params: host arrays, copied (the field pointers inside rves
 *   are kept and must stay valid for the context's life).
 *   workspace: device buffer of at least admm_workspace_bytes(), or NULL to
 *   let the library allocate (and free) its own.
 *   hip_stream: hipStream_t to enqueue on (NULL = default stream).
 * The penalty of every cell starts at params->rho0, the iteration count at 0.
 * The fields are used as given (the caller zeroes u, F - I and Lambda for a
 * fresh start). In ADMM_FP32_FP64RED without nu_F or the full LCE model's
 * terms the context also allocates 36 bytes per voxel for F - A as the
 * local step leaves it for Step 2, and without LCE materials 40 more for
 * the local step's data as the multiplier update forms it (reused within
 * one call; every call reads the fields afresh, so the caller may write
 * them between calls). Errors: EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ENOGPU. */
int admm_init(admm_ctx **out, const admm_rve *rves, int32_t n_rve,
              const admm_material *mats, int32_t n_mat, const admm_params *params,
              int32_t precision, void *workspace, size_t workspace_bytes,
              void *hip_stream);

/* Starts a new load step of cell `rve` (Algorithm 1, outer loop): sets its
 * macroscopic gradient, resets its iteration count and convergence flag and
 * keeps u, F, Lambda and rho as warm start. Errors: EINVAL (det Fbar <= 0). */
int admm_set_load(admm_ctx *ctx, int32_t rve, const double Fbar[9]);

/* Mixed boundary conditions (Sec. 2.3: components of <F> prescribed and the
 * complementary components of the average stress zero, as in the uniaxial
 * stress and plane stress protocols of Sec. 5). Bit k (k = 3i + j, row-major)
 * of free_mask leaves <F>_ij of cell `rve` free: Step 2 minimises over it as
 * well as over u, which sets it to the average of F - Lambda/rho, and the
 * multiplier update then keeps the average of Lambda_ij at zero, so that
 * <P>_ij = 0 at convergence. Free components start from their current value
 * (the load given to admm_init or admm_set_load, or the last iterate);
 * admm_set_load afterwards changes only the prescribed components. 0 (the
 * default): <F> prescribed. Errors: EINVAL (mask >= 512). */
int admm_set_free(admm_ctx *ctx, int32_t rve, uint32_t free_mask);

/* The current <F> of cell `rve` (row-major): the prescribed load and the free
 * components' iterate. Synchronises the stream. */
int admm_get_fbar(admm_ctx *ctx, int32_t rve, double Fbar_out[9]);

/* Stability modulus over Bloch waves (Sec. 2.5, Steps 1'-4'): for cell
 * `rve` of a double-precision context,
 *   beta = min over periodic p with <p, p> = 1 of <D_w p, L D_w p>,
 * L(x) = d2W/dF2 at the cell's current F (and director: the LCE with the
 * director eliminated; the ideal LCE model only), D_w the central
 * difference of the Bloch wave p exp(i omega . x), omega in radians per voxel
 * (2 pi / (k n_j) for a k-cell super-lattice along x_j); beta < 0 means the
 * periodic state is unstable against that wave. ADMM with penalty rho (L +
 * rho I must be positive definite at every voxel); Step 2' minimises over
 * the unit sphere exactly (Fourier space and a scalar secular equation), so
 * the fixed point is the smallest eigenvalue's mode. Runs until the RMS
 * residuals r_p, r_d <= tol or max_iter iterations.
 *   p: device buffer of 3V complex doubles (interleaved re, im; [c][x3][x2][x1]):
 *      start in, unit mode out.
 *   beta_out: <D_w p, L D_w p> of the mode; sigma_rho_out (may be NULL):
 *      rho sigma of the last Step 2' (equals beta at the fixed point);
 *   iters_out, status_out (may be NULL): iterations, ADMM_OK or
 *      ADMM_NOT_CONVERGED.
 * Allocates its work buffers (about 960 bytes per voxel) for the call.
 * Errors: EINVAL, EUNSUPPORTED (float context, full LCE model terms),
 * EDOMAIN (L + rho I not positive definite), ENOMEM, EHIP. */
int admm_bloch(admm_ctx *ctx, int32_t rve, const double omega[3], double rho, double tol,
               int32_t max_iter, void *p, double *beta_out, double *sigma_rho_out,
               int32_t *iters_out, int32_t *status_out);

/* admm_bloch without any device allocation, for callers that cannot
 * allocate (harnesses that forbid hipMalloc, loops that must not touch the
 * allocator). Same arguments, results and errors as admm_bloch, computed by
 * the same kernels in the same order (the results are identical). The work
 * buffers live in a fixed array of admm_bloch_static_max_bytes() bytes
 * (128 MiB) in the library's device code, one per GPU, held until the
 * process ends; a cell needs about 960 bytes per voxel (at most about
 * 139,000 voxels, e.g. 48^3). Larger cells: ADMM_ENOMEM, nothing run. The
 * array keeps the last call's contents (every call clears what it needs at
 * zero); calls on one GPU share it, so calls that overlap on one GPU (other
 * threads, other streams) race and must be serialised by the caller. */
int admm_bloch_static(admm_ctx *ctx, int32_t rve, const double omega[3], double rho,
                      double tol, int32_t max_iter, void *p, double *beta_out,
                      double *sigma_rho_out, int32_t *iters_out, int32_t *status_out);
size_t admm_bloch_static_max_bytes(void);

/* Orientation tensor of the LCE voxels of cell `rve` (the order parameter of
 * Sec. 5's polydomain studies): S = 3/2 (<n (x) n> - I/3), row-major.
 * Synchronises the stream. Errors: EINVAL (no LCE voxel). */
int admm_orientation(admm_ctx *ctx, int32_t rve, double S_out[9]);

/* Sets the penalty of one cell (rve >= 0) or of all cells (rve < 0). */
int admm_set_rho(admm_ctx *ctx, int32_t rve, double rho);

/* Runs exactly n_iter ADMM iterations (Steps 1-4 and the penalty rule) on
 * every cell, ignoring the tolerances. Host arrays of n_rve doubles receive
 * the last r_p, r_d and the penalty for the next iteration (each may be
 * NULL). Synchronises the stream. Errors: EINVAL, EDOMAIN, EHIP. */
int admm_step(admm_ctx *ctx, int32_t n_iter, double *r_p, double *r_d, double *rho);

/* Iterates every cell until r_p <= tol_p and r_d <= tol_d or max_iter
 * iterations of the current load step; converged cells are skipped on the
 * device. iters_out / status_out (n_rve entries each, may be NULL) receive the
 * iteration count and ADMM_OK / ADMM_NOT_CONVERGED / ADMM_EDOMAIN per cell.
 * Returns ADMM_OK if all converged, ADMM_NOT_CONVERGED if some did not, or an
 * error. Synchronises the stream. */
int admm_solve(admm_ctx *ctx, int32_t *iters_out, int32_t *status_out);

/* The three parts of one iteration, for testing each on its own:
 *   admm_local_step    Step 1 on every cell (F from u, Lambda, rho);
 *   admm_project_step  Step 2 on every cell (the new fluctuation, from
 *                      F - Lambda/rho, is written to u_prev; u keeps u_i);
 *   admm_update_step   Step 3 and Step 4 (Lambda, r_p, r_d, the penalty
 *                      rule) from u_i and u_{i+1}; u_{i+1} then is in u.
 * admm_step(ctx, 1, ...) equals the three in this order. */
int admm_local_step(admm_ctx *ctx);
int admm_project_step(admm_ctx *ctx);
int admm_update_step(admm_ctx *ctx);

/* Homogenised stress <P> = (1/V) sum_x W_F(F(x)) and <Lambda> of one cell
 * (Sec. 2.3; Lambda converges to the stress, Sec. 2.1), accumulated in
 * double precision on the device. Host outputs of 9 doubles (Lambda_out may
 * be NULL). Synchronises the stream. */
int admm_homogenized_stress(admm_ctx *ctx, int32_t rve, double P_out[9],
                            double Lambda_out[9]);

/* Residual history of the current load step of one cell: up to max_n entries
 * of r_p, r_d and the penalty used (host arrays, each may be NULL); n_out
 * receives the number of iterations recorded. */
int admm_history(admm_ctx *ctx, int32_t rve, int32_t max_n, double *r_p,
                 double *r_d, double *rho, int32_t *n_out);

/* Iteration count of the current load step, status (as admm_solve reports
 * it), the number of local solves that hit the Newton cap, and the Newton
 * iterations summed over voxels since the load step began (for cost
 * accounting) of one cell. Outputs may be NULL. */
int admm_cell_info(admm_ctx *ctx, int32_t rve, int32_t *iters, int32_t *status,
                   int32_t *newton_fail, int64_t *newton_iters);

/* Kernels timed by the profiling interface, in launch order. */
typedef enum {
  ADMM_KERNEL_LOCAL = 0,     /* Step 1: local Newton solve per voxel */
  ADMM_KERNEL_DIV_FWDX = 1,  /* b = D_h^T (F - Lambda/rho), forward FFT along x1 */
  ADMM_KERNEL_FFT_Y_FWD = 2, /* forward FFT along x2 */
  ADMM_KERNEL_POISSON_Z = 3, /* FFT along x3, Fourier-space solve, inverse along x3 */
  ADMM_KERNEL_FFT_Y_INV = 4, /* inverse FFT along x2 */
  ADMM_KERNEL_INV_X = 5,     /* inverse FFT along x1 into u */
  ADMM_KERNEL_UPDATE = 6,    /* Step 3 + residual partial sums */
  ADMM_KERNEL_FINALIZE = 7,  /* Step 4 reductions, test, penalty rule */
  ADMM_KERNEL_MEAN = 8,      /* homogenised stress reductions */
  ADMM_KERNEL_COUNT = 9
} admm_kernel;

/* Profiling (for measurement, not part of the method): when on, every kernel
 * launch of the context is bracketed by a pair of hipEvents on the context's
 * stream. Enabling clears the accumulated totals. */
int admm_profile_enable(admm_ctx *ctx, int32_t on);

/* Sum of the measured durations (ms) and number of launches of one kernel
 * since profiling was enabled. Synchronises the stream. */
int admm_profile_read(admm_ctx *ctx, int32_t kernel, double *total_ms, int32_t *launches);

/* Launch configuration of Step 2 (Sec. 3 runs the Fourier-space solve with
 * a vendor FFT; here the transforms are the library's own, and these are
 * their free parameters). */
typedef struct {
  int32_t tile_y, tile_z;   /* columns per workgroup of the x2 / x3 passes,
                               or ADMM_TILE_REG16 (below) */
  int32_t n_len;            /* distinct edge lengths of the context's cells */
  int32_t x_points;         /* points per workgroup of the x1 transforms
                               (256, 512 or 1024; lines = points / n1) */
  int32_t len[24];          /* those lengths, ascending */
  int32_t radix[24][8];     /* radix sequence of each length (2, 3, 4, 8),
                               0-terminated */
  double ms_default;        /* Step 2 over all cells, ms per call, before */
  double ms_tuned;          /* and after tuning */
} admm_tuning;

/* Tile width of the register-resident x2 / x3 pass, open to an axis where
 * every cell's length along it is 32, 48, 64, 96, 128 or 256 (float with
 * double reductions) or 256 (double). A length N = T P (T dividing P: 2 x 16,
 * 4 x 12, 4 x 16, 4 x 24, 8 x 16, 16 x 16) is taken by T threads per column,
 * P points each, 256 / T columns per workgroup: a length-P DFT in
 * registers, a twiddle, one exchange through LDS and P / T length-T DFTs
 * (Cooley-Tukey); each thread ends with the points it loaded. */
#define ADMM_TILE_REG16 (-16)

/* Autotuner (a performance control with no counterpart in the method): times
 * Step 2 over all cells on the context's stream, `reps` calls per candidate
 * (best of three), and keeps the fastest number of points per workgroup of
 * the x1 transforms, then the fastest tile width of the x2 pass, then of
 * the x3 pass (a quarter, half, default or double width, LDS <= 64 KiB, or
 * ADMM_TILE_REG16 where every cell's length along that axis is supported), then the
 * fastest radix sequence of each transform length in turn (every order of
 * the radix-8/4/2/3 splits, at most 24 per length). Results change only by
 * rounding (the transforms' operation order). Step 2 writes each cell's
 * second displacement buffer (u_prev) and the workspace; u, F, Lambda, the
 * director and the iteration state are unchanged. reps = 0 only reports the
 * current configuration. The choice stays with the context; captured graphs
 * are rebuilt. Not thread-safe with other calls on the same context. */
int admm_autotune(admm_ctx *ctx, int32_t reps, admm_tuning *out);

/* Persisted tuning: when the environment variable ADMM_AUTOTUNE_CACHE names
 * a file, admm_autotune (reps > 0) first looks there for the configuration
 * of this precision and these grids and applies it without timing; after
 * tuning it appends its result. (The file is plain text, one line per
 * configuration.) */

/* Applies a Step 2 launch configuration (a tuning admm_autotune reported,
 * or any other): tile widths of the x2 / x3 passes (compiled widths, LDS
 * <= 64 KiB, or ADMM_TILE_REG16 where every cell's length along that axis
 * is supported), points per workgroup of the x1 transforms (256, 512, 1024)
 * and, for each of the n_len lengths listed, its radix sequence (2, 3, 4,
 * 8, product equal to the length; lengths the context does not have are
 * refused). ms_default / ms_tuned are ignored. ADMM_EINVAL, with nothing
 * changed, on an invalid configuration. Results change only by rounding.
 * Captured graphs are rebuilt. */
int admm_set_tuning(admm_ctx *ctx, const admm_tuning *t);

/* Replays admm_solve's divergence watch (admm_params div_growth,
 * stall_iters, tol_p, tol_d) on a recorded residual history of one load
 * step (host arrays of n entries): *at receives the index of the iteration
 * at which the watch stops the cell, or -1 if it never does (a converged
 * iteration ends the replay with -1). Host only, no GPU needed. */
int admm_divergence_check(const admm_params *params, const double *r_p, const double *r_d,
                          int32_t n, int32_t *at);

/* Checkpoint and resume (Algorithm 1 carries u, F, Lambda, the director and
 * the penalty from one iteration and one load step to the next). The state
 * is everything the iteration reads: per cell u, F - I, Lambda, the
 * director, the library's start-of-step copies and lagged directors of the
 * full LCE model, the penalty, <F> and its prescribed load, the iteration
 * count, status and residual history of the current load step, the Newton
 * counters; and the Step 2 launch configuration (tiles, x1 points, radix
 * plans), on which the rounding of the transforms depends. A context
 * created with the same cells (grid sizes, phase maps), materials and
 * parameters, given this state with admm_set_state, continues bit for bit
 * as the original would have.
 *   admm_get_state: blob == NULL (or *bytes too small: ADMM_ENOMEM) only
 *     sets *bytes to the size needed; else writes the state to the host
 *     buffer blob and sets *bytes. Synchronises the stream.
 *   admm_set_state: reads a blob written by admm_get_state; ADMM_EINVAL
 *     (nothing changed) when it does not match this context (format, cell
 *     count, grid sizes, precision, which optional fields exist) or bytes
 *     is not its size. Synchronises the stream. */
int admm_get_state(admm_ctx *ctx, void *blob, size_t *bytes);
int admm_set_state(admm_ctx *ctx, const void *blob, size_t bytes);

/* Static description of an error code. */
const char *admm_strerror(int code);

/* Releases the context (not the caller's buffers). NULL is a no-op. */
void admm_destroy(admm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* ADMM_H */
