/*
 * lsh.h -- C ABI of the MI355X Lippmann--Schwinger homogenisation solver.
 *
 * The library solves the discrete Lippmann--Schwinger system of the periodic
 * corrector problem (Brisard & Legoll, "Periodic homogenization using the
 * Lippmann--Schwinger formalism", eq. (13)):
 *
 *   (A_beta - A0)^{-1} tau_beta + DFT^{-1}_beta[ Gamma_hat_k DFT_k[tau] ] = p,  beta in I0,
 *   tau_beta = 0 outside I0,
 *
 * matrix-free on one GPU, and returns the polarisation tau, the strain
 * estimate p - Gamma tau and the homogenised matrix A*_h p = A0 p + <tau>
 * (Theorem 4).  Physics: scalar conduction in 2D/3D (c = d components per
 * voxel) and 3D linear elasticity (c = 6 Mandel components
 * (e11, e22, e33, sqrt2 e23, sqrt2 e13, sqrt2 e12)).
 *
 * Conventions for every entry point:
 *  - Fields are stored [load][component][z][y][x] with x fastest (2D: nz = 1).
 *  - Matrices (moduli, A0, effective tensors) are row-major FP64.
 *  - "Host" pointers are read during the call and may be reused at once.
 *    "Device" pointers must stay valid until the work queued on the
 *    context's stream has finished; the library never frees them.
 *  - The library never allocates device memory: the caller binds one
 *    workspace buffer (lsh_workspace_bytes / lsh_bind_workspace).
 *  - Every entry point returns an lsh_status; nothing is thrown across the
 *    ABI.  Arguments are validated before any GPU work is queued; on an
 *    error the context keeps its previous state and lsh_last_error() holds
 *    a message.
 *  - A context is bound to one HIP stream and is not thread-safe.
 */
#ifndef LSH_H
#define LSH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lsh_ctx lsh_ctx;

typedef enum {
  LSH_OK = 0,
  LSH_MAXIT = 1,        /* warning: results valid but a load did not converge */
  LSH_EINVAL = -1,      /* invalid argument */
  LSH_ENOMEM = -2,      /* workspace missing or too small */
  LSH_EHIP = -3,        /* HIP runtime error */
  LSH_EHYP2 = -4,       /* A_phase - A0 neither zero nor definite (hypothesis (2)) */
  LSH_EBREAKDOWN = -5,  /* CG breakdown: |p.Lp| at rounding level (see lsh_solve) */
  LSH_ENUMERIC = -6,    /* NaN or Inf met during the solve */
  LSH_ESTATE = -7       /* call out of order (e.g. solve before phases are set) */
} lsh_status;

enum { LSH_SCALAR = 0, LSH_ELASTIC = 1 };            /* physics */
enum { LSH_FP64 = 0, LSH_MIXED = 1 };                /* precision */
enum { LSH_GREEN_TRUNCATED = 0, LSH_GREEN_FILTERED = 1, LSH_GREEN_CONSISTENT = 2, LSH_GREEN_FD = 3 };
enum {
  LSH_SOLVER_BASIC = 0,
  LSH_SOLVER_CG = 1,
  LSH_SOLVER_MINRES = 2,
  LSH_SOLVER_EYRE_MILTON = 3,
  LSH_SOLVER_SYMMLQ = 4
};
enum { LSH_HOST = 0, LSH_DEVICE = 1 };               /* memory space of a pointer */
enum { LSH_F64 = 0, LSH_F32 = 1 };                   /* element type of a field buffer */
enum { LSH_FIELD_TAU = 0, LSH_FIELD_STRAIN = 1 };

/* Per-load outcome of lsh_solve. */
typedef struct {
  int32_t iterations;     /* operator applications spent on this load (inner + outer) */
  int32_t status;         /* lsh_status of this load */
  double rel_residual;    /* ||b - L tau||_2 / ||b||_2, recomputed in FP64 after the solve */
} lsh_load_report;

/* Whole-solve outcome of lsh_solve. */
typedef struct {
  int64_t applications_fp64;   /* FP64 operator applications (all loads, each counted once per load) */
  int64_t applications_fp32;   /* FP32 operator applications (mixed precision inner solves) */
  int32_t outer_iterations;    /* iterative-refinement steps (mixed precision), else 0 */
  int32_t pad;
  double seconds;              /* wall time of the solve on the host clock (stream synchronised) */
} lsh_solve_report;

/*
 * Create a context for a grid of n[0] x n[1] (x n[2]) voxels along x, y (, z)
 * (the unit cell (0,1)^dim with h_a = 1/n[a], Section 3.1).
 *   dim        2 or 3 (elasticity needs 3).
 *   n          voxels per axis; each a power of two (n[0] >= 4, n[1], n[2] >= 2, all
 *              <= 1024) or one of 48, 96, 192 (3 * 2^m) and 80, 160 (5 * 2^m).
 *   physics    LSH_SCALAR or LSH_ELASTIC.
 *   precision  LSH_FP64: FP64 fields, transforms and reductions.
 *              LSH_MIXED: FP32 fields and transforms with FP64 dot products,
 *              FP64 A*, and FP64 iterative refinement of the residual.
 *   max_loads  largest batch of macroscopic loads solved together (>= 1).
 *   stream     hipStream_t the context queues its work on (NULL: the null stream).
 * Does not touch the GPU.  *out receives the context.
 */
lsh_status lsh_create(lsh_ctx** out, int dim, const int64_t* n, int physics, int precision,
                      int max_loads, void* stream);

/* Release the context (host memory only; the bound workspace stays the caller's). */
lsh_status lsh_destroy(lsh_ctx* ctx);

/* Bytes of device workspace the context needs (256-byte aligned base expected). */
lsh_status lsh_workspace_bytes(const lsh_ctx* ctx, size_t* bytes);

/* Bind caller-owned device memory of at least lsh_workspace_bytes bytes.
 * The library carves every field, spectrum, table and reduction buffer out of it. */
lsh_status lsh_bind_workspace(lsh_ctx* ctx, void* dev_ptr, size_t bytes);

/*
 * Reference medium A0 (Section 2.2.2): a constant symmetric positive definite
 * c x c matrix.  Scalar: any SPD d x d matrix.  Elastic: an isotropic 6x6 Mandel
 * stiffness (lambda0 in the upper-left 3x3 off-diagonal, 2 mu0 + lambda0 on its
 * diagonal, 2 mu0 on the shear diagonal); other forms return LSH_EINVAL.
 */
lsh_status lsh_set_reference(lsh_ctx* ctx, const double* A0);

/*
 * Microstructure: one phase id per voxel (uint8, [z][y][x]) in host or device
 * memory, and nphase (1..32) c x c moduli (conductivity, or Mandel stiffness)
 * in host memory, phase-major.  A voxel whose phase modulus equals A0 exactly
 * is outside I0 (its polarisation vanishes).  Voxel moduli are the phase
 * values (no sub-voxel averaging of eq. def_ah).  Hypothesis (2) is checked
 * at lsh_solve/lsh_apply time against the current A0: every other phase needs
 * A_phase - A0 definite (either sign), else LSH_EHYP2.  Phase ids >= nphase are
 * LSH_EINVAL with the context unchanged: host maps are checked on the host,
 * device maps (which need a bound workspace) by a kernel during the call.
 */
lsh_status lsh_set_phases(lsh_ctx* ctx, const uint8_t* phase, int mem, int nphase,
                          const double* moduli);

/*
 * Microstructure given voxel by voxel (instead of lsh_set_phases), isotropic
 * at every voxel: m is [ncoef][z][y][x] in host or device memory, element type
 * dtype (LSH_F64 or LSH_F32):
 *   scalar      ncoef = 1: a_beta, A_beta = a_beta Id;
 *   elasticity  ncoef = 2: bulk and shear moduli (K_beta, mu_beta), Mandel
 *               stiffness K m m^T + 2 mu (Id - m m^T / 3), m = (1,1,1,0,0,0).
 * Needs the reference set first, isotropic (scalar A0 = a0 Id, else
 * LSH_EINVAL), and a bound workspace; the voxel data are converted during the
 * call into the short form of (A_beta - A0)^{-1} (Section 3.1, eq. 13), so
 * changing A0 afterwards asks for the moduli again (LSH_ESTATE at solve time).
 * Hypothesis (2) per voxel: A_beta = A0 exactly (outside I0), or
 * a_beta - a0 nonzero, or K_beta - K0 and mu_beta - mu0 nonzero and of one sign;
 * differences below 1e-12 of the moduli, and non-finite values, give
 * LSH_EHYP2 with the context unchanged.  Host data are checked on the host,
 * device data by a counting kernel before anything is written.
 */
lsh_status lsh_set_voxel_moduli(lsh_ctx* ctx, const void* m, int dtype, int mem, int ncoef);

/* Discrete Green operator: truncated (eqs. 14/15 with the Nyquist rule of
 * Section 3.2.1), filtered (Section 3.2.2), consistent (eq. 11, stored; needs a
 * bound table, see below) or finite-difference (Section 3.2.3, scalar physics
 * only; LSH_EINVAL for elasticity).  Default: filtered. */
lsh_status lsh_set_green(lsh_ctx* ctx, int variant);

/*
 * The consistent operator of eq. (11) is a slowly converging lattice series
 * that has to be stored (Section 3.2).  It is evaluated once on the GPU, in
 * FP64, into caller-owned device memory of lsh_green_table_bytes bytes bound
 * with lsh_bind_green_table, keeping the aliases whose reduced frequency
 * k_a/N_a + n_a lies in [-(nmax + 1/2), nmax + 1/2] on every axis
 * (lsh_set_green_series, default nmax = 8; 0 <= nmax <= 64).  The table holds
 * the upper triangle of the c x c matrix at every stored wave-vector.
 */
lsh_status lsh_green_table_bytes(const lsh_ctx* ctx, size_t* bytes);
lsh_status lsh_bind_green_table(lsh_ctx* ctx, void* dev_ptr, size_t bytes);
lsh_status lsh_set_green_series(lsh_ctx* ctx, int nmax);

/*
 * MINRES and SYMMLQ keep four FP64 fields per load (MINRES: two Lanczos
 * vectors, two search directions; SYMMLQ uses three: two Lanczos vectors and
 * the partially rotated direction wbar) in caller-owned device memory of
 * lsh_solver_buffer_bytes bytes (the same for both) bound with
 * lsh_bind_solver_buffer (256-byte aligned); the other solvers need none
 * (0 bytes).
 */
lsh_status lsh_solver_buffer_bytes(const lsh_ctx* ctx, int solver, size_t* bytes);
lsh_status lsh_bind_solver_buffer(lsh_ctx* ctx, void* dev_ptr, size_t bytes);

/*
 * Initial guess tau_0 for load slot `load` (0..max_loads-1) of the next
 * lsh_solve (warm start; the default is tau_0 = 0).  tau: c x grid field,
 * component-major with x fastest (the lsh_get_field layout), FP64 or FP32
 * (dtype), host or device memory (mem; device memory is read in stream order
 * and may be reused after the call returns).  It is copied into the FP64
 * solution slot of that load, so the fields of the previous solve are no
 * longer available (lsh_get_field returns LSH_ESTATE until the next solve).
 * Values outside I0 are ignored (tau vanishes there).  tau = NULL clears the
 * guess of that slot.  A guess applies to the next lsh_solve only.  The solve
 * then starts from r_0 = b - L tau_0 (one extra FP64 application) with the
 * same stopping rule ||b - L tau|| <= tol ||b||, so a guess that already meets
 * it takes no iteration; the fixed-point schemes start their iteration at
 * tau_0, and the mixed-precision solve begins with an FP64 refinement step.
 * Errors: LSH_EINVAL (slot, dtype, mem), LSH_ESTATE (no workspace bound).
 */
lsh_status lsh_set_initial_guess(lsh_ctx* ctx, int load, const void* tau, int dtype, int mem);

/*
 * Solve eq. (13) for nload (1..max_loads) macroscopic loads p_l (host,
 * nload x c row-major FP64; Mandel in elasticity), starting from tau = 0,
 * until ||b - L tau||_2 <= tol ||b||_2 with b = p on I0 (mixed precision: the
 * FP64 refined residual), or maxit operator applications per load, with
 *   LSH_SOLVER_BASIC        the fixed point tau = (A - A0)(p - Gamma tau);
 *   LSH_SOLVER_CG           conjugate gradients (Section 5);
 *   LSH_SOLVER_MINRES       MINRES (Paige and Saunders), for the symmetric
 *                           indefinite systems of an A0 between the phases;
 *                           needs the solver buffer; the stopping test uses
 *                           its recursive residual norm;
 *   LSH_SOLVER_EYRE_MILTON  the fixed point tau = (A - A0)(A + A0)^{-1}
 *                           (tau + 2 A0 (p - Gamma tau)) of the Eyre--Milton
 *                           scheme, contracting for any SPD A0 (factor
 *                           max |(a - a0)/(a + a0)| for scalar A0 = a0 Id);
 *   LSH_SOLVER_SYMMLQ       SYMMLQ (Paige and Saunders), named beside CG as
 *                           a solver of the discretised equation (Section 1),
 *                           for the symmetric indefinite system of an A0
 *                           between the phases: LQ iterates of
 *                           least error over L K_k(L, b); it stops on the
 *                           residual of the CG point and returns that point
 *                           (also after maxit steps, when it exists); needs
 *                           the solver buffer.
 * The basic, MINRES, SYMMLQ and Eyre--Milton iterations run in FP64 in either
 * precision; CG in a mixed context uses FP32 fields with FP64 refinement.
 *   reports   host array of nload lsh_load_report (may be NULL).
 *   summary   host lsh_solve_report (may be NULL).
 * Returns LSH_OK, LSH_MAXIT (results valid, some load unconverged), or an error.
 * The basic scheme converges only when A0 dominates (scalar isotropic:
 * max|a - a0| < a0).  CG is guaranteed to converge when the system is positive
 * definite (A0 softer than every phase, Section 5); with A0 between the phases
 * the system is symmetric indefinite and CG proceeds, reporting
 * LSH_EBREAKDOWN for a load whose |p.Lp| falls to g r.r or below, with
 * g = eps (max over the phases of ||(A - A0)^{-1}||_2 + ||A0^{-1}||_2) a bound
 * of ||L||_2 times eps = 1e-12 (FP64 fields) or 1e-6 (FP32 fields of the
 * mixed inner solve): as p.p >= r.r, the Rayleigh quotient of p is then below
 * eps ||L||, unresolved at the field precision (per-voxel media use
 * ||A0^{-1}|| alone).  In a mixed solve, a breakdown or NaN/Inf of the inner
 * FP32 solve ends that load with that status after its progress is refined
 * into the FP64 solution.  Loads converge independently: a converged load is
 * frozen while the others iterate.
 */
lsh_status lsh_solve(lsh_ctx* ctx, int solver, int nload, const double* loads, double tol,
                     int maxit, lsh_load_report* reports, lsh_solve_report* summary);

/*
 * Copy a field of the last solve for load `load` into dst
 * ([component][z][y][x], dtype LSH_F64 or LSH_F32, host or device memory):
 *   LSH_FIELD_TAU     the polarisation tau, the unknown of eq. (13);
 *   LSH_FIELD_STRAIN  p - Gamma tau on every voxel: the estimate of
 *                     p + grad w_p that the proof of the equivalence lemma of
 *                     Section 2.2.2 reads off the Lippmann--Schwinger equation
 *                     (equal to (A - A0)^{-1} tau on I0 at convergence); one
 *                     extra FP64 operator pass, computed during the call.
 * LSH_ESTATE without a solve (or after lsh_set_initial_guess overwrote the
 * load's solution slot); LSH_EINVAL for a load beyond the last solve's.
 */
lsh_status lsh_get_field(lsh_ctx* ctx, int load, int which, void* dst, int dtype, int mem);

/* Mean stress A0 p_l + <tau_l> of the last solve, host FP64 array nload x c:
 * the discrete homogenised matrix of Theorem 4, A*_h p = A0 p + <tau_h(p)>,
 * with the mean over the voxels reduced in FP64 in a fixed order.  With the
 * c unit loads, row l is column l of A*_h.  LSH_ESTATE without a solve. */
lsh_status lsh_get_effective(lsh_ctx* ctx, double* sigma_mean);

/*
 * Residual history of load `load` in the last solve: the relative residual
 * ||r_k|| / ||b|| after every iteration, in order, as the solver's own
 * recurrences give it (CG: the recursive residual of Section 5's CG setting;
 * the fixed-point schemes of Section 3: the residual of the iterate; MINRES:
 * |phi_k|; SYMMLQ: the residual of the CG point, +inf where it has none),
 * with a level per entry: 0 for an FP64 iteration (and the FP64 residual
 * b - L tau that a mixed solve refreshes after each inner solve), 1 for an
 * iteration of the FP32 inner CG of a mixed solve, relative to its own
 * right-hand side (the FP64 residual it started from).  The device keeps the
 * last 4096 entries per load.  Copies the last min(cap, total, 4096) entries
 * into rel and level (host arrays of cap entries; both may be NULL when cap
 * is 0) and the number of entries the solve made into *total (may be NULL).
 * Synchronises the context's stream.  LSH_EINVAL for a load beyond the last
 * solve's or cap < 0.
 */
lsh_status lsh_get_residual_history(lsh_ctx* ctx, int load, int cap, double* rel, int32_t* level, int64_t* total);

/*
 * Derivative of J = sum_lm W_lm p_l . A*_h p_m over the loads of the last solve
 * (W: host FP64 nload x nload, symmetrised as (W + W^T)/2) with respect to the
 * isotropic coefficients of every voxel.  The operator M of eq. (13) is
 * symmetric and only its local block (A_beta - A0)^{-1} depends on A_beta, so
 * with A*_h p = A0 p + <tau_p> (Theorem 4)
 *   dJ/dA_beta = (1/V) sum_lm W_lm sym(eps_l (x) eps_m),  eps = p - Gamma tau,
 * which costs one operator pass per load and no further solve.  Written to
 * grad (device, [ncoef][z][y][x], LSH_F64 or LSH_F32):
 *   scalar      dJ/da  = tr(dJ/dA_beta);
 *   elasticity  dJ/dK  = m^T (dJ/dA_beta) m,  dJ/dmu = 2 (tr - m^T (.) m / 3).
 * Valid for phase maps and per-voxel moduli alike (the derivative is then the
 * one of an isotropic perturbation of each voxel).  LSH_ESTATE without a solve.
 */
lsh_status lsh_gradient(lsh_ctx* ctx, const double* W, void* grad, int dtype);

/*
 * Matrix-free operator of eq. (13): out_l = 1_{I0} ((A - A0)^{-1} tau_l + Gamma tau_l)
 * for nload fields tau (device, [load][component][z][y][x], element type
 * dtype: LSH_F64 uses the FP64 kernels, LSH_F32 the FP32 ones, the latter in
 * a LSH_MIXED context only).  tau is meant to vanish outside I0 (Gamma acts
 * on tau as given).  out is a device buffer of the same shape and type; it
 * may not alias tau.
 */
lsh_status lsh_apply(lsh_ctx* ctx, int nload, const void* tau, void* out, int dtype);

/*
 * lsh_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same operator and kernels, with no scratch taken from the workspace.  The
 * main spectrum is formed in `out` itself (it has exactly the bytes of the
 * real output) and the Nyquist plane (kx = nx/2; nload * c * nz * ny complex
 * values of dtype) in a fixed per-GPU scratch array of 64 MiB, a device
 * global of the library that every GPU it runs on holds until the process
 * ends; larger planes return LSH_ENOMEM before any GPU work.  Material
 * tables are formed on first use after a change, as by lsh_apply; the
 * solution fields of the workspace are not touched, so the last solve's
 * results stay available.  `out` must be 256-byte aligned.  The call
 * makes no device allocation (no hipMalloc, no allocating library call); the
 * first call on a device looks up the scratch address once.  The scratch
 * holds the last call's plane and needs no clearing (every entry is written
 * before it is read); calls that overlap in time on one GPU (other streams or
 * threads) share it and race.  Blocks until the result is in `out`.
 */
lsh_status lsh_apply_noalloc(lsh_ctx* ctx, int nload, const void* tau, void* out, int dtype);

/*
 * Forward DFT of nload real fields (device, [load][component][z][y][x],
 * dtype LSH_F64/LSH_F32) into the library's packed half spectrum, copied to
 * `spec` (device): complex [load][component][nz][ny][nx/2] (interleaved
 * re,im; entry kx = 0 holds the kx = 0 column) followed by the Nyquist plane
 * complex [load][component][nz][ny] (kx = nx/2).  Unnormalised, sign -1
 * (Section 3.1).  Exposed to test and profile the transform passes.
 */
lsh_status lsh_forward_dft(lsh_ctx* ctx, int nload, const void* field, void* spec, int dtype);

/* Bytes of the packed spectrum of one field for dtype (see lsh_forward_dft). */
lsh_status lsh_spectrum_bytes(const lsh_ctx* ctx, int dtype, size_t* bytes);

/*
 * Kernel shapes.  The transform passes over 128- and 256-point axes are
 * compiled in four workgroup shapes each (pencils per workgroup and points
 * per thread); pass 0..3 = x forward, y, z with Green operator, x inverse, for
 * the FP32 (fp64 = 0) or FP64 (fp64 = 1) kernels.  The z pass has a fifth
 * shape (4): one workgroup per wave-vector tile handles every load, forming
 * the operator matrices once (FP32, truncated, filtered and consistent
 * operators; otherwise shape 0 runs).  Its sixth shape (5) runs 8-pencil
 * tiles on a component-paired copy of the spectrum that the y passes write
 * and read back (FP32 six-component fields of a mixed context with the stored
 * filtered operator, 128- or 256-point y and z axes; otherwise shape 0 runs;
 * the copy lives in the FP64 spectrum buffer of the workspace, so the
 * workspace size does not change).  Every shape computes the
 * same result up to rounding; only speed differs.  lsh_get_variants writes the 8 current
 * choices (FP32 passes, then FP64).  The environment variable LSH_TUNE (for
 * example "zg32=1,xinv64=2") sets them when the context is created.
 */
lsh_status lsh_set_variant(lsh_ctx* ctx, int pass, int fp64, int variant);
lsh_status lsh_get_variants(const lsh_ctx* ctx, int32_t* variants);

/*
 * Autotuner: times every shape of every pass that has several (the others
 * held at their current choice; the z pass before the y passes, whose layout
 * its shape 5 sets) with HIP events over operator applications
 * of nload loads on the context's own buffers, in the modes the solvers run
 * (the CG modes for FP32 fields of a mixed context and FP64 fields of an FP64
 * context, the refinement modes for the FP64 passes of a mixed context), and
 * keeps the fastest.
 * With cache_path (may be NULL) the choice is looked up first in, and
 * afterwards written to, a text file with one line per key: device, grid,
 * components, precision, nload, Green operator and material form.  A cache
 * hit runs nothing on the GPU (*from_cache = 1).  Needs a prepared context
 * (reference and material set); invalidates the last solution.  variants
 * (may be NULL) receives the 8 choices as lsh_get_variants.
 */
lsh_status lsh_autotune(lsh_ctx* ctx, int nload, const char* cache_path, int32_t* variants, int* from_cache);

/*
 * Ensembles (the stochastic-homogenisation use of Section 2.1: one
 * microstructure per member): solve n independent contexts (distinct, each on
 * its own HIP stream of default priority) as lsh_solve would, each, so that the
 * work of small grids overlaps on the GPU.  The solves run as cooperative
 * fibers on the calling thread: up to nthreads members are in flight (< 1:
 * 4); a member runs until it waits for the GPU (its solver states or results),
 * then the next one enqueues its work.  Every HIP call is made from the calling
 * thread, one member at a time (no concurrent graph captures), and each
 * member's sequence of launches is the one of its own lsh_solve, so results
 * equal those of solving the members one after another.  Per context i:
 * nloads[i], loads[i], reports[i] (array of nloads[i] lsh_load_report, or
 * reports NULL), summaries[i] and statuses[i] (each array may be NULL).
 * Returns the first error status, else LSH_MAXIT if any context stopped at
 * maxit, else LSH_OK.  Contexts sharing one stream are still correct but
 * serialise.  Not reentrant from within an ensemble solve.
 */
lsh_status lsh_solve_many(int n, lsh_ctx* const* ctxs, int solver, const int32_t* nloads,
                          const double* const* loads, double tol, int maxit,
                          lsh_load_report* const* reports, lsh_solve_report* summaries,
                          int32_t* statuses, int nthreads);

/*
 * Persistent launch (default on): for small grids (squares of 8..64 voxels in
 * 2D, cubes of 8 voxels, and cubes of 16 for scalar problems: at most 12288
 * unknowns per load, where it beats the multi-kernel loop on MI355X)
 * conjugate gradients run as one kernel launch per
 * solve, one workgroup per load performing every iteration (the same fused
 * step, its passes separated by workgroup barriers), which removes the
 * per-kernel latency that dominates such grids.  0 keeps the multi-kernel
 * loop.  The environment variable LSH_PERSISTENT=0 sets 0 at creation.
 */
lsh_status lsh_set_persistent(lsh_ctx* ctx, int enable);

/*
 * Iteration graphs (default on): the kernels of one solver iteration are
 * captured once into a HIP graph (on a private stream of default priority)
 * and the graph is replayed on the context's stream for every iteration.
 * Graphs are not used while kernel timing is enabled.  The captured graph
 * holds only kernel nodes.
 */
lsh_status lsh_set_graphs(lsh_ctx* ctx, int enable);

/*
 * Kernel timing: when enabled, every kernel launch is bracketed by HIP events
 * on the context's stream and accumulated per kernel class (transform and
 * update classes are split by element type, e.g. "zgamma_f32").
 * lsh_kernel_times fills up to cap entries of names (static strings), total
 * milliseconds, launch counts and algorithmic bytes (the HBM traffic each
 * pass must move: its inputs read once, its outputs written once, for the
 * loads still iterating) since the last reset; any output array may be NULL.
 * *count receives the number of classes.  Reading synchronises the stream.
 * Enabling or disabling resets the counters.
 */
lsh_status lsh_set_timing(lsh_ctx* ctx, int enable);
lsh_status lsh_kernel_times(lsh_ctx* ctx, const char** names, double* total_ms, int64_t* launches,
                            double* alg_bytes, int cap, int* count);

/* Message of the last error on this context ("" when none). */
const char* lsh_last_error(const lsh_ctx* ctx);

/* Library version string. */
const char* lsh_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LSH_H */
