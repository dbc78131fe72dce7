/*
 * xfft.h -- C ABI of the MI355X X-FFT solver for periodic 3-D linear-elastic
 * cell problems (Gehrig & Schneider, arXiv 2601.02172).
 *
 * The problem (Sec. 2): find the mean-free periodic displacement fluctuation u
 * in the scaled X-FEM space (eq. X-FEM scaled space) such that the weak
 * equilibrium (eq. discreteFormConti) holds for a prescribed macro strain.
 * Discretisation (Sec. 3): every voxel of a regular grid is split into six P1
 * tetrahedra; elements cut by the linearly interpolated nodal level set carry
 * modified-abs enriched shape functions (eqs. enrichedN, modified abs
 * enrichment) scaled by D0^-1/2 (eq. scaling factors); cut elements are
 * integrated exactly on the subdivision along the interface.  The system is
 * solved by the linear CG of Algorithm 1 with the block preconditioner
 * diag(A11^0, I) (eq. scaledPreconditioner) whose FE block is inverted by FFT
 * (eq. GreenHermitian), stopped by eq. stoppingCriterion.
 *
 * Conventions shared by every entry point:
 *  - Grid n[3] nodes per axis (periodic; node (i,j,k) at (i,j,k)*h), cubic
 *    voxels h = len[0]/n[0] = len[1]/n[1] = len[2]/n[2].  Each n[k] must be
 *    even, >= 4 and of the form 2^a 3^b (FFT radices 2, 3, 4), and its line
 *    FFT must fit one workgroup: at most 1024 (x, y) or 2048 (z, three lines)
 *    butterflies in its smallest-radix stage and 64 KiB of LDS.  Accepted:
 *    every such length up to 1296 on all axes, and on x and y also 1458 to
 *    2304, 2916 and 3072; other lengths give XFFT_EINVAL.
 *  - Nodal arrays have N = n0*n1*n2 entries at index i + n0*(j + n1*k).
 *  - Symmetric tensors are Voigt-Mandel 6-vectors (11, 22, 33, sqrt2*23,
 *    sqrt2*13, sqrt2*12); C_eff is the 6x6 Mandel matrix, row-major.
 *  - Vectors of unknowns (step-level entry points) are component-major: FE
 *    dof (node i, component c) at c*N + i, followed by the scaled enriched dof
 *    (enriched node j, component c) at 3N + c*nX + j.  Enriched nodes are
 *    numbered in increasing node index.  These vectors are in voxel units
 *    (h = 1); the solve entry points convert displacements to units of len.
 *  - Host pointers unless the name says _device.  The caller owns every array
 *    it passes; the library copies inputs during the call and owns all device
 *    memory of a problem until xfft_destroy.
 *  - A handle is not thread safe; distinct handles may be used concurrently.
 *  - The reductions of the solve (CG dot products, residual norms, average
 *    stress) are fixed-order trees over per-workgroup partial sums, so solves
 *    are bitwise reproducible for a given problem, option set and device;
 *    there is no nondeterministic mode to select.  The per-phase sums of
 *    xfft_grad_lame add into workgroup tables with LDS atomics (then reduce in
 *    a fixed order), so gradients may differ between runs in the last bits.
 *  - Return value: XFFT_OK (0), XFFT_NOT_CONVERGED (+1: outputs hold the last
 *    iterate), or a negative error code; xfft_strerror names it.
 */
#ifndef XFFT_H
#define XFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    XFFT_OK = 0,
    XFFT_NOT_CONVERGED = 1,
    XFFT_EINVAL = -1,      /* bad argument: sizes, NaN/Inf, phase out of range, non-PD moduli */
    XFFT_ENOMEM = -2,      /* device allocation failed */
    XFFT_EDEVICE = -3,     /* HIP runtime error or no usable gfx950 device */
    XFFT_EBREAKDOWN = -4   /* CG breakdown: d^T A d <= 0 or not finite */
};

enum { XFFT_FP64 = 0, XFFT_MIXED = 1, XFFT_FP32 = 2 /* step-level entry points only */ };

/* Solution schemes (Sec. 3, solvers).  All share the operator, the
 * preconditioner and the stopping criterion of Algorithm 1 and differ in the
 * step alpha and the direction weight beta of an iteration; s0 is the step
 * size of eq. stepsize, 2 / (C_- + C_+) over the stiffness eigenvalues
 * (3 lambda + 2 mu and 2 mu) of all phases.
 *   XFFT_LCG    linear CG (Algorithm 1): alpha = res^2 / <A d, d>, beta = res_new^2 / res^2
 *   XFFT_NLCG   nonlinear CG: fixed step alpha = s0, Fletcher-Reeves beta = res_new^2 / res^2
 *   XFFT_BB     Barzilai-Borwein: beta = 0, alpha = <s, P s> / <s, A s> of the previous update s
 *               (the previous iteration's res^2 / <A d, d>); the first step is s0
 *   XFFT_BASIC  basic scheme: beta = 0, alpha = s0 (Richardson iteration u += s0 P^-1 f) */
enum { XFFT_LCG = 0, XFFT_NLCG = 1, XFFT_BB = 2, XFFT_BASIC = 3 };

/* Discretisations (Sec. 4.1, Tab. discretizations).
 *   XFFT_XFEM  the X-FEM discretisation of the method (default)
 *   XFFT_P1    voxel-segmented P1 Galerkin FEM on the same six elements per voxel: no enrichment, one
 *              material per voxel.  The voxel's side is the sign of the level set at its centre (the
 *              mean of its eight corner values); it takes the label of its corner with the largest |L|
 *              on that side (L >= 0 for a centre value >= 0, else L < 0), ties to the corner with the
 *              smallest x + 2y + 4z offset. */
enum { XFFT_XFEM = 0, XFFT_P1 = 1 };

typedef struct xfft_problem xfft_problem;

typedef struct {
    double rtol;        /* tol of eq. stoppingCriterion (default 1e-10) */
    int32_t maxit;      /* max CG iterations per load; mixed: total inner iterations (default 20000) */
    int32_t precision;  /* XFFT_FP64 (plain CG in FP64) or XFFT_MIXED (FP32 CG inside FP64
                           iterative refinement); default XFFT_FP64 */
    double snap_eps;    /* |L|/h below this is set to 0 (Sec. 3 reads 1e-6; default 1e-6) */
    double d0_scale;    /* multiplies every D0_jj; the converged result is independent (default 1) */
    double inner_rtol;  /* mixed: residual reduction of each inner FP32 solve (default 1e-6); an inner solve also
                           ends once its residual meets half the outer tolerance rtol */
    int32_t batch;      /* 1: all loads of a call iterate together; 0: one load at a time (default 1) */
    int32_t device;     /* HIP device ordinal (default 0) */
    int32_t check_every;/* host polls convergence every this many iterations (default 8; rounded up to even) */
    int32_t use_graph;  /* 1: the check_every iterations between polls are captured once into a hipGraph and
                           replayed (default 1); 0: launched one by one */
    int32_t autotune;   /* 1: at the first solve, time the operator's tile depths and keep the fastest (default 1) */
    void *stream;       /* hipStream_t to run on, or NULL for a library-owned stream */
    int32_t scheme;     /* XFFT_LCG (default), XFFT_NLCG, XFFT_BB or XFFT_BASIC; schemes other than
                           XFFT_LCG need precision XFFT_FP64 */
    int32_t discretization; /* XFFT_XFEM (default) or XFFT_P1 */
    int32_t voxel_matrices; /* cached voxel matrices of the irregular voxels (Sec. 3, caching strategy): the
                               scaled 48 x 48 matrix of each irregular voxel (FP64, and FP32 rounded once) replaces
                               the moment form in the CG iterations (up to 6 loads per launch), read once for all
                               loads: -1 (default) the faster of the two, timed at the first solve per precision
                               (only when the tables fit in a quarter of the free device memory, else the moment
                               form); 0 never; 1 always (also for xfft_apply_operator).  Costs 11.8 KB (FP64) / 5.9 KB
                               (FP32) of device memory per irregular voxel; falls back to the moment form when the
                               allocation fails.  Rebuilt after xfft_set_lame. */
    int32_t warm_start;     /* 1: a solve of the six unit Mandel loads (xfft_solve, xfft_solve_device) starts the
                               CG of each load from that load's solution of the previous unit-load solve of this
                               problem (same geometry, possibly other moduli after xfft_set_lame) instead of
                               u = 0; other solves, the first one and xfft_batch_solve start from 0.  The converged result does not depend on the start; the stopping
                               test of eq. stoppingCriterion is the same.  Default 0. */
    int32_t fft_variant;    /* kernels of the Green operator (eq. GreenHermitian): -1 (default) timed at the first
                               solve of a precision, the fastest kept (with autotune on; else 0); or fixed: bit 0
                               set = separate x and y passes instead of the xy-plane kernels (grids with
                               n0 = n1 in {16, 32, 48, 64, 96, 128}), bit 1 set = the alternative z-pass tile
                               (twice the kx columns per workgroup at n2 = 256, half of them for the other
                               compile-time lengths 16 ... 128).  A bit a grid has no choice for is ignored.
                               Every variant computes the same transform. */
} xfft_options;

typedef struct {
    int32_t *iters;        /* NULL or [nload]: CG iterations (mixed: inner iterations summed) */
    int32_t *outer_iters;  /* NULL or [nload]: refinement steps (mixed only) */
    double *final_res;     /* NULL or [nload]: last res / ||<sigma>|| (FP64 criterion) */
    double seconds_setup;  /* wall time of xfft_setup */
    double seconds_solve;  /* wall time of the last xfft_solve */
    int64_t n_enriched;    /* |J| */
    int64_t n_irregular_voxels; /* voxels with a cut element or mixed element materials */
    int64_t n_cut_elements;
    int64_t n_multilabel;  /* cut elements whose vertices on one side carry different labels */
    int32_t voxel_matrices;/* 1 if the CG iterations of the last solve used the cached voxel matrices */
    int32_t fft_variant;   /* FFT variant (bits as option fft_variant) of the last solve's CG iterations */
} xfft_stats;

/* Fill *opt with the defaults listed above. */
void xfft_default_options(xfft_options *opt);

/* Build a problem (Sec. 2, Sec. 3): snap the level set, find cut elements and
 * the enriched node set J (eq. X-FEM space), number them, compute the scaling
 * factors D0 (eq. scaling factors) and the Green-operator tables (eq.
 * GreenHermitian).  levelset[N] is the nodal signed distance in units of len
 * (eq. levelset); phase[N] holds nodal labels in [0, nphase); lame[nphase][2]
 * = (lambda, mu) per phase, each with mu > 0 and 3 lambda + 2 mu > 0 (eq.
 * boundsStiffness).  Material of an element: uncut -> label of its vertex with
 * the largest |L|; cut -> side L > 0 takes the label of its vertex with the
 * largest L, side L < 0 that of its vertex with the largest |L| (ties: first
 * vertex along the Kuhn path).  On success *out owns device memory until
 * xfft_destroy.  Size limits (32-bit byte offsets inside one load's fields):
 * 24 N < 2^32 and 384 x (irregular voxels) < 2^32, else EINVAL.
 * Errors: EINVAL, ENOMEM, EDEVICE (nothing is allocated then). */
int xfft_setup(const int32_t n[3], const double len[3], const double *levelset,
               const int32_t *phase, int32_t nphase, const double *lame,
               const xfft_options *opt, xfft_problem **out);

/* Solve the cell problem for nload macro strains (Algorithm 1 with eqs.
 * stoppingCriterion and convergence; mixed precision refines an FP64
 * residual with FP32 CG corrections).  macro_strain[nload][6].  Outputs, each
 * optional (NULL):
 *   disp[nload][3][N]      nodal FE displacement fluctuation in units of len
 *                          (enriched functions vanish at the nodes);
 *   stress[nload][6][N]    voxel-average Mandel stress (eq. average stress per voxel);
 *   avg_stress[nload][6]   cell-average stress <sigma> (eq. average stress);
 *   c_eff[6][6]            requires nload == 6 with the unit Mandel basis as
 *                          macro strains (else EINVAL); column k = <sigma> of load k.
 * stats may be NULL.  Returns OK, NOT_CONVERGED, EBREAKDOWN, EINVAL, ENOMEM, EDEVICE. */
int xfft_solve(xfft_problem *p, int32_t nload, const double *macro_strain,
               double *disp, double *stress, double *avg_stress, double *c_eff,
               xfft_stats *stats);

/* Same as xfft_solve with caller-owned device buffers (e.g. torch tensors):
 * strain_dev[nload][6], disp_dev[nload][3][N] or NULL, avg_stress_dev[nload][6]
 * or NULL, all float64 on the problem's device; runs on `stream` (hipStream_t,
 * NULL = the problem's stream) and returns after it completes.  With the six
 * unit Mandel loads, avg_stress_dev holds C_eff: row k of avg_stress_dev is
 * column k of C_eff (C_eff is symmetric, so the [6][6] block is C_eff itself up
 * to the solver's tolerance); no separate C_eff output is needed. */
int xfft_solve_device(xfft_problem *p, int32_t nload, const double *strain_dev,
                      double *disp_dev, double *avg_stress_dev, void *stream,
                      xfft_stats *stats);

/* Replace the per-phase Lame pairs (same nphase) keeping the geometry, J and
 * D0 (they do not depend on the moduli).  EINVAL on non-PD moduli. */
int xfft_set_lame(xfft_problem *p, const double *lame);

/* Gradient of the energy form of C_eff with respect to the Lame pairs, using
 * the six unit-load solutions of the last xfft_solve (which must have been
 * called with nload == 6 and the unit Mandel basis): by Galerkin
 * orthogonality (App. A) dC_kl/dlambda_p = |Y|^-1 int_p tr eps_k tr eps_l and
 * dC_kl/dmu_p = 2 |Y|^-1 int_p eps_k . eps_l.  dL_dC[6][6] weights the 36
 * derivatives: grad[p][0] = sum_kl dL_dC[k][l] dC_kl/dlambda_p, grad[p][1]
 * likewise for mu.  dC_out (NULL or [nphase][2][6][6]) receives the raw
 * derivatives.  EINVAL if no suitable solve is stored. */
int xfft_grad_lame(xfft_problem *p, const double *dL_dC, double *grad, double *dC_out);

/* Solve several problems (uneven grids allowed, same precision option), each
 * for the six unit Mandel loads, returning c_eff[nprob][6][6]: the CG
 * iterations of all problems are captured once as parallel branches of one
 * hipGraph (fork/join over the problems' streams) and replayed until every load
 * of every problem has converged; mixed precision refines all problems in
 * lock step.  The unit-load solutions are kept for xfft_grad_lame.  stats may
 * be NULL or [nprob] (iters/outer_iters arrays of length 6 each). */
int xfft_batch_solve(xfft_problem *const *ps, int32_t nprob, double *c_eff, xfft_stats *stats);

/* Step-level entry points (host arrays, voxel units, layout above).
 * xfft_apply_operator: y = r(x) = A x + sum_e Lambda_e^T int B^T C eps_bar
 *   (eq. resVector with the macro strain; macro_strain NULL means zero, giving
 *   y = A x); avg_stress (NULL or [6]) = <sigma(eps_bar + grad^s x)>.
 * xfft_apply_precond: y = P^-1 f (eq. scaledPreconditioner: Green operator of
 *   eq. GreenHermitian on the FE block, identity on the enriched block);
 *   res2 (NULL or [1]) = f^T P^-1 f (eq. convergence before the square root).
 * precision: XFFT_FP64 or XFFT_FP32 (inputs rounded to float, outputs widened). */
int xfft_apply_operator(xfft_problem *p, int32_t precision, const double *x,
                        const double *macro_strain, double *y, double *avg_stress);
int xfft_apply_precond(xfft_problem *p, int32_t precision, const double *f,
                       double *y, double *res2);

/* Voxel-average stress of a state (eq. Sapp_q per element, summed over the six
 * elements of each voxel; voxel volume 1 in voxel units): stress[6][N] (Mandel,
 * voxel index fastest) = sum_e in voxel int_e C (eps_bar + grad^s x), FP64.
 * x[3N + 3nX] in the step-level layout, macro_strain NULL (zero) or [6].  The
 * same kernels produce the stress output of xfft_solve.
 * xfft_apply_operator runs the kernels without the stress integral when
 * avg_stress is NULL (the variant of the CG iterations), with it otherwise. */
int xfft_voxel_stress(xfft_problem *p, const double *x, const double *macro_strain, double *stress);

/* Allocation-free variant of xfft_apply_operator, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops).
 * FP64 only, device pointers: x_dev[3N + 3nX] (step-level layout, voxel
 * units), macro_strain_dev NULL (zero) or [6], y_dev[3N + 3nX] receives
 * r(x) (eq. resVector), avg_stress_dev NULL or [6] receives <sigma>.  Runs on
 * `stream` (hipStream_t; NULL = the problem's stream) without waiting for it;
 * the outputs are ready when the stream reaches this point.  The per-workgroup
 * partial sums and the corner-force buffer of the irregular voxels live in a
 * static 64 MiB device array per GPU (held until the process ends), so the call
 * makes no allocation; grids needing more (8 NPART nslots + 384 x irregular
 * voxels bytes, about 150 k irregular voxels) give XFFT_EINVAL, as does a call
 * between xfft_profile_begin and xfft_profile_end.  All calls on one GPU share
 * that array: calls that overlap in time on one GPU (other streams, other
 * threads, other problems) race and must be serialised by the caller.
 * Returns OK, EINVAL or EDEVICE (launch failure). */
int xfft_apply_operator_noalloc(xfft_problem *p, const double *x_dev, const double *macro_strain_dev,
                                double *y_dev, double *avg_stress_dev, void *stream);

/* Sizes and enriched-node data: info[0..5] = N, nX, irregular voxels, cut
 * elements, multi-label cut elements, nphase; jlist[nX] (NULL allowed) = node
 * index of each enriched node; d0[nX] (NULL allowed) = D0_jj. */
int xfft_get_layout(xfft_problem *p, int64_t *info, int64_t *jlist, double *d0);

/* Kernel timing of the CG iteration (Algorithm 1) in the launch configuration
 * of a solve with nrhs loads: runs nrep iterations on the problem's stream with
 * a HIP event after every kernel and returns, per kernel class, the average
 * time between the event before and the event after a launch (ms_out[11],
 * ms) and the number of launches timed (count_out[11]); either may be NULL.
 * Classes: 0 irregular-voxel operator, 1 regular-voxel operator, 2 enriched
 * gather, 3 FFT x forward (+ residual update), 4 FFT y forward, 5 FFT z +
 * Green multiply + inverse z, 6 FFT y inverse, 7 FFT x inverse (+ CG update),
 * 8 enriched residual, 9 enriched CG update, 10 scalar recurrences.  Work
 * that runs inside another class's launch is timed there and its own class
 * counts no launches: the enriched gather always (class 1), the enriched
 * residual with the compile-time z pass (class 5), the enriched CG update with
 * the xy-plane kernels (class 7).
 * precision: XFFT_FP64 or XFFT_FP32.  Overwrites the problem's work fields. */
int xfft_profile(xfft_problem *p, int32_t precision, int32_t nrhs, int32_t nrep, double *ms_out,
                 int32_t *count_out);

/* Timing of every kernel launched on the problem's stream between the two
 * calls (e.g. around xfft_solve): a HIP event is recorded before and after
 * each launch; xfft_profile_end returns per kernel class the average window
 * length in ms (ms_out[22]) and the number of launches (count_out[22]);
 * classes 0..10 as for xfft_profile in FP32, 11..21 the same in FP64 (the
 * scalar recurrences are FP64: class 21).  Adds a little host overhead. */
int xfft_profile_begin(xfft_problem *p);
int xfft_profile_end(xfft_problem *p, double *ms_out, int32_t *count_out);

void xfft_destroy(xfft_problem *p);
const char *xfft_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* XFFT_H */
