/*
 * vmfmm -- fast multipole evaluation of the Gaussian-regularised Biot-Savart
 * velocity and vortex-stretching term for N vortex particles on one AMD
 * Instinct MI355X (gfx950).
 *
 * Method (Yokota & Barba, "FMM-based vortex method for simulation of
 * isotropic turbulence on GPUs, compared with a spectral method"):
 *   - particles carry strength alpha_j (= gamma_j), Gaussian core sigma
 *     (Sec. 2.2, eqs. 3-4);
 *   - velocity u_i = 1/(4 pi) sum_j q(r) alpha_j x r, r = x_i - x_j,
 *     q = g(r/sigma)/r^3, g the cutoff of eq. 6 (eq. 5);
 *   - gradient J_i[a][b] = d u_b / d x_a; stretching (eq. 8)
 *     dalpha_i/dt = sum_a alpha_{i,a} J_i[a][:]  ("classic"), or the
 *     transpose J_i . alpha_i, which conserves sum_i alpha_i;
 *   - far field by multipole/local expansions of degree 0..p of the three
 *     Laplace potentials psi = G * omega (eqs. 10-15), u = curl psi, with the
 *     cutoff dropped there; near field (27 adjacent leaves) exact (Sec. 3.1);
 *   - periodic cube: the 26 neighbouring images through the tree, further
 *     images of the cubic block 3^K x 3^K x 3^K by a lattice operator on the
 *     root multipole (Sec. 3.1 last paragraph; Sec. 4.1 uses K = 3).
 *
 * Conventions for every entry point:
 *   - device pointers are HIP device addresses; particle arrays are SoA
 *     [3][n] (component-major) doubles, 8-byte aligned, owned by the caller;
 *   - work is enqueued on the context's stream and the call returns after
 *     enqueueing (no host synchronisation unless stated);
 *   - a context is used by one host thread at a time; calls on one context
 *     run in stream order;
 *   - argument errors return VM_EINVAL before anything is launched; HIP
 *     failures return VM_EDEVICE; allocation failures VM_ENOMEM; the text
 *     of the last error is kept in the context (vm_last_error);
 *   - graph capture: after one call with the same sizes and options (which
 *     grows the workspace and builds the operator caches), vm_fmm_eval,
 *     vm_fmm_eval_at, vm_rk2_step and vm_run without reinitialisation enqueue
 *     kernels only -- no allocation, copy, memset or host synchronisation --
 *     when check_domain is 0 and timing is off, so the caller may capture them
 *     into a HIP graph on the context's stream and replay it.  The solvers
 *     (vm_rbf_solve, vm_reinit) synchronise and cannot be captured.
 */
#ifndef VMFMM_H
#define VMFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vm_ctx vm_ctx;

typedef enum {
    VM_OK = 0,
    VM_EINVAL = -1,   /* invalid argument (nothing launched) */
    VM_ENOMEM = -2,   /* device or host allocation failed */
    VM_EDEVICE = -3,  /* HIP runtime / launch failure */
    VM_EDOMAIN = -4   /* check_domain: a position was non-finite or outside the box */
} vm_status;

typedef enum { VM_FP64 = 0, VM_MIXED = 1 } vm_precision;
typedef enum { VM_CLASSIC = 0, VM_TRANSPOSE = 1 } vm_scheme;
/* M2L truncation: VM_SQUARE keeps every target degree n <= p against every
 * source degree n' <= p (eqs. 12-13 as printed); VM_TRIANGULAR keeps n + n' <= p
 * only (the classical truncation: at p = 10 about a fifth of the products,
 * similar accuracy).  M2M, L2L and the lattice operator are exact either way. */
typedef enum { VM_SQUARE = 0, VM_TRIANGULAR = 1 } vm_truncation;

typedef struct {
    double box_lo[3];  /* lower corner of the root cube */
    double box_len;    /* edge of the root cube; the period when periodic > 0 */
    int periodic;      /* 0: free space; K in 1..4: images in the block 3^K per side */
    int precision;     /* vm_precision */
    int scheme;        /* vm_scheme (stretching form written to dalpha_dt) */
    int check_domain;  /* 1: flag non-finite / out-of-box positions (one 4-byte
                          device-to-host copy and a stream synchronisation) */
    int truncation;    /* vm_truncation of the M2L operators (0: square) */
} vm_opts;

/* Limits checked on every call. */
#define VM_MAX_P 18   /* the FP64 translation tile's LDS staging bounds the degree */
#define VM_MAX_LEVEL 10

/* Creates a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t, or NULL for the default stream).  The context owns its
 * workspace (grown on demand, reused across calls), its operator cache and
 * a second non-blocking stream (default priority) with two events, which
 * vm_fmm_eval forks from and joins back into the bound stream, so callers
 * still see every call ordered on their stream (graph capture included).
 * VM_EDEVICE when the device, the stream or the events cannot be set up. */
vm_status vm_create(vm_ctx **ctx, int device, void *hip_stream);
/* Waits for the context's work on its bound and second streams, then frees
 * its workspace, operator cache, second stream and events (NULL: no-op). */
void vm_destroy(vm_ctx *ctx);
/* Binds the context to another stream for the calls that follow.  Nothing is
 * enqueued: work a previous call left on the old stream is not waited for, and
 * since every call reuses the context's workspace, the caller orders the two
 * streams (an event or a synchronisation) before the next call when they
 * differ.  VM_EINVAL for a NULL context. */
vm_status vm_set_stream(vm_ctx *ctx, void *hip_stream);
/* The message of the context's last failed call (a static string for NULL). */
const char *vm_last_error(const vm_ctx *ctx);

/*
 * FMM evaluation (Sec. 3.1, eqs. 5-15).
 *   n          number of particles, 1 <= n < 2^31
 *   x          device [3][n]: positions; periodic runs take them modulo the box
 *   alpha      device [3][n]: strengths
 *   sigma      Gaussian core radius (> 0), the same for all particles
 *   p          expansion degree, 1..VM_MAX_P ((p+1)^2 real coefficients per component)
 *   level      leaf level of the uniform octree, 0..VM_MAX_LEVEL (8^level leaves);
 *              free space needs level >= 2 for any far field (below that the
 *              evaluation is the direct sum)
 *   u          device [3][n] out: velocity
 *   dalpha_dt  device [3][n] out or NULL: stretching term, opts->scheme form
 *   grad       device [9][n] out or NULL: J[a][b] = d u_b / d x_a at index 3a+b
 * All outputs are in the caller's particle order.  FP64 and mixed forms take
 * and return double precision; the mixed form computes the near field in
 * FP32 with compensated velocity sums and the expansions in FP32 (MFMA),
 * keeping the translation operators' generation and the lattice operator in FP64.
 */
vm_status vm_fmm_eval(vm_ctx *ctx, int64_t n, const double *x, const double *alpha,
                      double sigma, int p, int level, const vm_opts *opts,
                      double *u, double *dalpha_dt, double *grad);

/*
 * The velocity and its gradient that the particles induce at m points y
 * other than the particles (e.g. a lattice for spectra): the same model as
 * vm_fmm_eval -- each point belongs to the leaf its position falls in
 * (periodic: wrapped; free space: clamped into the edge leaf, reported by
 * check_domain), the far field from that leaf's local expansion, the exact
 * regularised sum over its 27 adjacent leaves -- with a second tree over the
 * points.
 *   x, alpha   device [3][n]: particles and strengths
 *   y          device [3][m]: the points, 1 <= m < 2^31
 *   u          device [3][m] out;  grad  device [9][m] out or NULL
 * Precision forms and errors as vm_fmm_eval (no stretching: the points carry
 * no strength).
 */
vm_status vm_fmm_eval_at(vm_ctx *ctx, int64_t n, const double *x, const double *alpha, int64_t m, const double *y,
                         double sigma, int p, int level, const vm_opts *opts, double *u, double *grad);

/*
 * Adaptive hybrid treecode-FMM (Sec. 3.2): the same velocity, gradient and
 * stretching as vm_fmm_eval for particle sets that are far from uniform.
 *   tree     the particles are keyed at max_level exactly as vm_fmm_eval keys
 *            them at `level`; a cell is split when it holds more than ncrit
 *            particles and lies above max_level, and only its non-empty
 *            children exist, so leaves sit at any level and hold at most ncrit
 *            particles except at max_level;
 *   lists    a stack-based dual traversal from the root against itself (and,
 *            periodic, its 26 images) pairs cells: two cells whose closed cubes
 *            (the source shifted by its image) do not touch interact through
 *            expansions -- M2L between cells of one level (cell-cell), M2P from
 *            a finer split source cell to the particles of a leaf and P2L from
 *            the particles of a coarser leaf to a split cell (cell-particle) --
 *            touching leaves, and leaves of different levels that do not touch,
 *            exchange the exact regularised kernel (P2P: for a cell side of at
 *            most ncrit particles the direct sum is the cheaper interaction),
 *            any other touching pair is refined.  Every (target, source,
 *            image) triple is covered once; on a uniform tree the lists are
 *            vm_fmm_eval's.
 *   far field  the cutoff is dropped in all expansion interactions (the cells
 *            are at least one width of the smaller one apart, so at leaves of
 *            width >= 4 sigma as in vm_fmm_eval);
 *   periodic images beyond the 27 of the tree by the same lattice operator.
 * n, x, alpha, sigma, opts, u, dalpha_dt, grad as vm_fmm_eval; p in
 * 1..VM_ADAPTIVE_MAX_P; ncrit >= 1; max_level 0..VM_MAX_LEVEL.  FP64 form and
 * square truncation only (VM_EINVAL otherwise).  Unlike vm_fmm_eval the call
 * synchronises the stream several times (the host sizes each level's cells and
 * the lists) and cannot be captured into a graph.  The context keeps the
 * tree, the lists and the expansions of the last call (vm_debug_adaptive).
 */
#define VM_ADAPTIVE_MAX_P 14   /* the cell-particle kernel holds (p+3)^2 harmonics per particle in LDS */
vm_status vm_fmm_eval_adaptive(vm_ctx *ctx, int64_t n, const double *x, const double *alpha, double sigma, int p,
                               int ncrit, int max_level, const vm_opts *opts, double *u, double *dalpha_dt,
                               double *grad);

/*
 * Auto-tuned leaf size of the adaptive tree (Sec. 3.2: the library picks how
 * many particles a leaf may hold, the user does not): candidates
 * ncrit = 8, 16, ..., 1024 in increasing order, each run once untimed and
 * `reps` times timed (HIP events on the context's stream) with
 * vm_fmm_eval_adaptive, until the time has risen twice in a row.
 *   ncrit  out: the fastest candidate
 *   ms     out or NULL: [VM_NCRIT_CANDIDATES] milliseconds per evaluation of
 *          each candidate tried, -1 for the others
 * Errors as vm_fmm_eval_adaptive; VM_EINVAL for reps outside 1..100.
 */
#define VM_NCRIT_CANDIDATES 8
vm_status vm_tune_ncrit(vm_ctx *ctx, int64_t n, const double *x, const double *alpha, double sigma, int p,
                        int max_level, const vm_opts *opts, int reps, int *ncrit, double *ms);

/*
 * Debug views of the last vm_fmm_eval_adaptive (synchronous copies into host
 * memory `out`, or NULL to query *rows only):
 *   what 0: cells, rows of 6 int32 (Morton key at the cell's level, level,
 *           first sorted particle, particle count, parent cell or -1, leaf 0/1),
 *           level-major, ascending key within a level;
 *   what 1, 2, 3, 4: the P2P, M2L, M2P, P2L lists, rows of 3 int32 (target
 *           cell, source cell, image shift code (sx+1) + 3 (sy+1) + 9 (sz+1));
 *   what 5: the caller index of each sorted particle (n int32).
 */
vm_status vm_debug_adaptive(vm_ctx *ctx, int what, int32_t *out, int64_t *rows);

/*
 * Discrete adjoint of vm_fmm_eval's velocity (the transposed FMM): for a
 * cotangent u_bar of u it returns
 *   alpha_bar = (du/dalpha)^T u_bar,   x_bar = (du/dx)^T u_bar
 * of exactly the map vm_fmm_eval computes (same tree, lists, truncation and
 * lattice operator; the tree is held fixed, since the keys are piecewise
 * constant in x).  Pipeline: L2P^T, L2L^T, M2L^T (MFMA with transposed
 * operators), lattice^T, M2M^T, P2M^T with its source-position derivative,
 * P2P with u_bar as strengths (the pair kernel satisfies K(r)^T = K(-r)),
 * plus the target terms J u_bar.  The forward state (tree, expansions and
 * gradient) is recomputed inside the call rather than stored between calls.
 * x, alpha, u_bar: device [3][n]; x_bar, alpha_bar: device [3][n] out (either
 * may be NULL).  Same precision forms as vm_fmm_eval; the context keeps
 * 30 FP64 words per particle of scratch.
 */
vm_status vm_fmm_adjoint(vm_ctx *ctx, int64_t n, const double *x, const double *alpha, double sigma, int p,
                         int level, const vm_opts *opts, const double *u_bar, double *x_bar, double *alpha_bar);

/*
 * vm_fmm_adjoint without the forward recomputation: the tree (leaf ranges,
 * permutation, sorted records) is taken from the context and the total
 * gradient from `grad` (device [9][n], the grad output of that evaluation).
 * Valid only right after vm_fmm_eval on this context with the same x, alpha
 * (pointers), n, sigma, p, level and opts (box, periodic, precision,
 * truncation), no tree-building call in between, and x, alpha and grad
 * unchanged since (the caller's responsibility); otherwise VM_EINVAL ("the
 * context's last evaluation is not this one") before anything is launched.
 * Further adjoints of the same evaluation may follow.  Results equal
 * vm_fmm_adjoint's bit for bit.
 */
vm_status vm_fmm_adjoint_reuse(vm_ctx *ctx, int64_t n, const double *x, const double *alpha, double sigma, int p,
                               int level, const vm_opts *opts, const double *grad, const double *u_bar,
                               double *x_bar, double *alpha_bar);

/*
 * One step of Heun's method (explicit trapezoidal RK2) for the convection and
 * stretching ODEs (eqs. 7-8; the paper integrates them with forward Euler,
 * Sec. 4.1).  With (u, s) = vm_fmm_eval(x, alpha) (s the opts->scheme form):
 *   x* = x + dt u(x, a),  a* = a + dt s(x, a),
 *   x <- x + dt/2 (u(x, a) + u(x*, a*)),  a <- a + dt/2 (s(x, a) + s(x*, a*)),
 * then, periodic, x wrapped into the box as the keys do.  x and alpha (device
 * [3][n]) are updated in place; sigma stays fixed (no core spreading).
 * u0, grad0: device [3][n] / [9][n] or NULL: the velocity and gradient at the
 * initial state (for diagnostics).  The context keeps four [3][n] FP64
 * scratch arrays (grown on demand).
 */
vm_status vm_rk2_step(vm_ctx *ctx, int64_t n, double *x, double *alpha, double sigma, int p, int level,
                      const vm_opts *opts, double dt, double *u0, double *grad0);

/*
 * Energy and enstrophy in FP64 with a fixed reduction order (deterministic):
 *   out[0] = E     = h3/2 sum_i |u_i|^2
 *   out[1] = Omega = h3/2 sum_i |curl u_i|^2, curl u from grad (0 if grad is NULL)
 *   out[2] = Omega_p = 1/(2 h3) sum_i |alpha_i|^2 (0 if alpha is NULL)
 * u [3][n], grad [9][n], alpha [3][n] and out [3] are device pointers; h3 is
 * the particle volume (h^3).
 */
vm_status vm_diagnostics(vm_ctx *ctx, int64_t n, const double *u, const double *grad, const double *alpha,
                         double h3, double *out);

/*
 * vm_diagnostics for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels, arguments, results (bit for bit) and errors, but the
 * per-block partial sums live in a static device array of the library
 * (3 x 1024 doubles = 24 KiB per device, held until the process ends) instead
 * of the context's workspace, and the call allocates nothing -- no hipMalloc,
 * hipFree or allocating library routine; its first call on a device looks up
 * that device's copy of the array (hipGetSymbolAddress).  The partial-sum
 * pass is grid-strided over at most 1024 blocks, so every n in [1, 2^31)
 * fits; a launch needing more slots would return VM_EINVAL.  Every slot it
 * reads is written by the same call first, so nothing needs clearing between
 * calls.  All calls on one device share that array: two such calls that
 * overlap in time on one device (different streams or contexts, or host
 * threads) race and give wrong results; calls in one stream are ordered.
 */
vm_status vm_diagnostics_noalloc(vm_ctx *ctx, int64_t n, const double *u, const double *grad,
                                 const double *alpha, double h3, double *out);

/*
 * Gaussian smoothing sum over the neighbour list (Sec. 2.2, eqs. 3-4, and the
 * reinitialisation paragraph there): the vorticity the particles carry, at
 * the particles,
 *   omega_i = sum_j gamma_j zeta_sigma(x_i - x_j - n L),
 *   zeta_sigma(r) = (2 pi sigma^2)^(-3/2) exp(-|r|^2 / (2 sigma^2)),
 * with j over the particles of the 27 leaves adjacent to x_i's leaf (itself
 * included) at leaf level `level`: free space skips leaves outside the box;
 * periodic (opts->periodic > 0, any K) wraps the leaf index and shifts the
 * source by its image n L, so a source counts once per adjacent leaf slot
 * (twice or more when 2^level < 3).  No far field: the Gaussian is taken to
 * vanish beyond the neighbour leaves, the truncation the paper makes.
 *   x, gamma   device [3][n]: positions (periodic: modulo the box), strengths
 *   omega      device [3][n] out, caller order
 * opts->precision: VM_FP64 computes in FP64; VM_MIXED takes FP32 differences
 * and exponentials with FP32 sums over each source leaf, added in FP64.
 * opts->scheme is ignored.  Same argument rules and errors as vm_fmm_eval
 * (sigma > 0, 0 <= level <= VM_MAX_LEVEL, ...).  The context's tree
 * workspace and debug tree view are reused (vm_debug_tree shows this call's
 * tree afterwards; the expansion views report no expansions).
 */
vm_status vm_gauss_sum(vm_ctx *ctx, int64_t n, const double *x, const double *gamma, double sigma, int level,
                       const vm_opts *opts, double *omega);

/*
 * The same neighbour-list Gaussian sum at m points y distinct from the
 * particles (the smoothing-function equation evaluated anywhere):
 *   omega(y_i) = sum_j gamma_j zeta_sigma(y_i - x_j - n L),
 * j over the particles in the 27 leaves adjacent to y_i's leaf.  The points
 * get a tree of their own at the same level (periodic: wrapped like the
 * particles; free space: clamped into the edge leaves, reported by
 * check_domain).
 *   x, gamma   device [3][n]: particles and strengths
 *   y          device [3][m]: the points, 1 <= m < 2^31
 *   omega      device [3][m] out, in y's order
 * Precision forms, errors and workspace as vm_gauss_sum.
 */
vm_status vm_gauss_eval(vm_ctx *ctx, int64_t n, const double *x, const double *gamma, int64_t m, const double *y,
                        double sigma, int level, const vm_opts *opts, double *omega);

/*
 * RBF interpolation (Sec. 2.2, the reinitialisation paragraph; initial guess
 * and tolerance as in Sec. 5's solver-tolerance study, default tolerance 1e-3
 * in Sec. 4.1): the strengths gamma that reproduce a given vorticity at the
 * particles, A gamma = omega with A the vm_gauss_sum operator, solved for each
 * component by restarted GMRES(VM_RBF_RESTART) with the matrix-free product.
 *   x, omega   device [3][n]: positions and the vorticity to interpolate
 *   h3         the particle volume h^3: the initial guess is gamma_0 = h3 omega
 *   tol        exit when every component's residual norm has dropped to
 *              tol times its norm at gamma_0 (0 <= tol < 1; 0 runs max_iter)
 *   max_iter   products after the initial residual, 0..VM_RBF_MAX_ITER
 *   gamma      device [3][n] out, caller order
 *   iters      out (may be NULL): the products spent (the three components
 *              share each one)
 *   resid      out (may be NULL): the largest relative residual reached, as
 *              GMRES estimates it (exact at every restart)
 * Orthogonalisation by classical Gram-Schmidt applied twice; dot products
 * reduce in a fixed order, so results are reproducible run to run.  Each
 * iteration reads the dot products back to the host (synchronises the
 * stream).  The context keeps (VM_RBF_RESTART + 3) [3][n] FP64 vectors.
 * Precision forms as vm_gauss_sum (the vectors and the iteration are FP64 in
 * both).  Returns VM_OK also when max_iter ends the iteration first: compare
 * *resid with tol.
 */
#define VM_RBF_RESTART 20
#define VM_RBF_MAX_ITER 100000
vm_status vm_rbf_solve(vm_ctx *ctx, int64_t n, const double *x, const double *omega, double sigma, double h3,
                       int level, const vm_opts *opts, double tol, int max_iter, double *gamma, int *iters,
                       double *resid);

/*
 * Reinitialisation onto the lattice (Sec. 2.2: core spreading grows sigma,
 * and the particles are moved back to a regular lattice with smaller
 * Gaussians by RBF interpolation; Sec. 5 studies how often):
 *   1. the sites y_k = box_lo + (i + 1/2) h of the ng^3 lattice, h = box_len/ng,
 *      k = (i_x ng + i_y) ng + i_z (x index slowest);
 *   2. omega_k = vm_gauss_eval of the particles (x, alpha) with core sigma at y;
 *   3. alpha <- vm_rbf_solve(y, omega, sigma0, h^3, tol, max_iter);
 *   4. x <- y.
 * n must equal ng^3 (one particle per site).  x and alpha (device [3][n]) are
 * replaced in place; iters and resid as vm_rbf_solve (may be NULL).  Errors
 * as vm_rbf_solve, plus VM_EINVAL when n != ng^3 or sigma0 <= 0.
 */
vm_status vm_reinit(vm_ctx *ctx, int64_t n, double *x, double *alpha, double sigma, int ng, double sigma0,
                    int level, const vm_opts *opts, double tol, int max_iter, int *iters, double *resid);

/*
 * The vortex method's time loop (Sec. 2.2: convection eq. 7, stretching
 * eq. 8 and core-spreading diffusion d sigma^2/dt = 2 nu update positions,
 * strengths and core simultaneously; reinitialisation every few steps).
 * Each step from (x, alpha, sigma) with the rates of vm_fmm_eval:
 *   VM_EULER (the paper's integrator): x += dt u, alpha += dt dalpha/dt;
 *   VM_HEUN: the trapezoid of the rates at the start (core sigma) and at the
 *            Euler prediction (core sigma'), as vm_rk2_step;
 * then sigma' = sqrt(sigma^2 + 2 nu dt), periodic positions wrapped, and after
 * every reinit_every-th step vm_reinit onto the ng^3 lattice with the core
 * the loop started with (sigma <- that core).
 */
typedef enum { VM_EULER = 0, VM_HEUN = 1 } vm_integrator;
typedef struct {
    int integrator;    /* vm_integrator */
    double dt;         /* time step, >= 0 */
    double nu;         /* kinematic viscosity, >= 0 */
    int steps;         /* steps to take, >= 0 */
    int reinit_every;  /* 0: never; k > 0: after every k-th step */
    int ng;            /* lattice of the reinitialisation (n = ng^3) */
    double tol;        /* GMRES tolerance of the reinitialisation (as vm_rbf_solve) */
    int max_iter;      /* GMRES products per reinitialisation */
} vm_loop;
/*
 *   x, alpha   device [3][n], advanced in place
 *   sigma      host in/out: the core at the start (also the reinitialisation
 *              core), the core at the end
 *   p, level, opts as vm_fmm_eval (opts->scheme is the stretching form)
 *   diag       device [steps][3] out or NULL: E, Omega, Omega_p (vm_diagnostics,
 *              particle volume box_len^3 / n) of the state each step starts from
 *   products, resid  host out or NULL: GMRES products summed over the
 *              reinitialisations, the largest relative residual they ended with
 * Stream-ordered; each reinitialisation synchronises (GMRES reads its dot
 * products back).  Workspace as vm_rk2_step and vm_reinit.
 */
vm_status vm_run(vm_ctx *ctx, int64_t n, double *x, double *alpha, double *sigma, int p, int level,
                 const vm_opts *opts, const vm_loop *loop, double *diag, int *products, double *resid);

/*
 * Shell energy spectrum of a velocity sampled on the ng^3 lattice of the
 * periodic cube (the diagnostic that the velocity at lattice points, e.g.
 * vm_fmm_eval_at on the grid of a spectral method, makes possible):
 *   E[s] = 1/2 sum over integer wavevectors m with rint(|m|) = s of |u_m|^2,
 *   u_m = ng^-3 sum_x u(x) exp(-i 2 pi m.x / box_len),  s = 0 .. kmax,
 * so that sum_s E[s] = <|u|^2>/2 once kmax >= sqrt(3) ng / 2.
 *   ng    lattice points per side, 2..1290
 *   u     device [3][ng^3]: the velocity at lattice point (i_x ng + i_y) ng + i_z
 *         (x index slowest), any fixed offset of the lattice
 *   kmax  last shell, 0..VM_SPECTRUM_MAX_K
 *   E     device [kmax + 1] out
 * A real-to-complex FFT per component (hipFFT; the plan is created on the
 * first call for an ng and kept), then one fixed-order sum per shell over a
 * host-built list of its entries (deterministic).  The context keeps the
 * plan, (ng^3 + 3 ng^2 (ng/2+1)) doubles and the shell lists.
 */
#define VM_SPECTRUM_MAX_K 4096
vm_status vm_energy_spectrum(vm_ctx *ctx, int ng, const double *u, int kmax, double *E);

/*
 * Auto-tuned leaf level (Sec. 3.2: the number of tree levels that gives the
 * shortest runtime depends on the problem and the hardware, and is chosen
 * without user input).  Candidates are the levels whose leaf width
 * box_len 2^-level is at least min_leaf_sigmas sigma -- the far field drops
 * the cutoff beyond the adjacent leaves, and 4 sigma keeps that model error
 * near 5e-7 on the lattice workloads -- and with no more leaves than
 * particles, tried from the finest towards coarser ones while the time falls.  Each candidate runs vm_fmm_eval once untimed
 * (workspace, caches) and `reps` times timed with HIP events on the context's
 * stream, with the given p and options (velocity and stretching into context
 * scratch).  Synchronises.
 *   level  out: the fastest level tried
 *   ms     out or NULL: [VM_MAX_LEVEL + 1] milliseconds per evaluation of each
 *          level tried, -1 for the others
 * Errors as vm_fmm_eval; VM_EINVAL for min_leaf_sigmas <= 0 or reps outside 1..100.
 */
vm_status vm_tune_level(vm_ctx *ctx, int64_t n, const double *x, const double *alpha, double sigma, int p,
                        const vm_opts *opts, double min_leaf_sigmas, int reps, int *level, double *ms);

/*
 * Device-time accounting (HIP events around every launch, on the stream the
 * launch goes to: vm_fmm_eval runs its near field (VM_PH_P2P) on a second,
 * non-blocking stream of the context, forked after the tree build by an event
 * and joined by L2P, so the P2P phase overlaps P2M and what of the far field
 * the hardware schedules beside it, and the combine of near and far field is
 * part of VM_PH_L2P).  vm_set_timing(ctx, 1) starts a fresh account (and 0 stops it);
 * vm_get_timing reports, summed over every vm_fmm_eval since then, the
 * milliseconds and the number of launches of each phase (at most 32768
 * launches are recorded); it synchronises the stream.  vm_gauss_sum and
 * vm_rbf_solve add their tree build to VM_PH_TREE and their own work to the
 * last two phases.  Phases, in launch order:
 */
enum {
    VM_PH_TREE = 0,   /* keys, radix sort passes, leaf ranges, permutation */
    VM_PH_P2M,
    VM_PH_M2M,
    VM_PH_LATTICE,
    VM_PH_L2L,
    VM_PH_M2L,
    VM_PH_L2P,
    VM_PH_P2P,        /* near field (+ combine and scatter to caller order without a far field) */
    VM_PH_GAUSS,      /* Gaussian sums of vm_gauss_sum / vm_rbf_solve (with the strength packing) */
    VM_PH_KRYLOV,     /* vector work of vm_rbf_solve: dots, updates, gathers and scatters */
    VM_PH_LISTS,      /* adaptive tree: cells, leaves and the dual traversal's lists */
    VM_PH_P2L,        /* adaptive tree: particle-cell interactions */
    VM_PH_M2P,        /* adaptive tree: cell-particle interactions */
    VM_NPHASE
};
vm_status vm_set_timing(vm_ctx *ctx, int enable);
vm_status vm_get_timing(vm_ctx *ctx, double *ms, int *launches);

/*
 * Debug views of the last vm_fmm_eval on this context (stream-ordered
 * device-to-device copies into caller buffers; any pointer may be NULL):
 *   keys        device [n] uint32: Morton keys in sorted order
 *   perm        device [n] int32: caller index of each sorted particle
 *   leaf_start  device [8^level + 1] int32: first sorted index of each leaf
 * Keys follow the oracle's definition bit for bit (periodic wrap
 * s = floor((x - lo) * fl(1/L)), x_w = x - s L; c = floor((x_w - lo) * 2^level fl(1/L))
 * clamped to [0, 2^level - 1]; bit b of c_x, c_y, c_z -> key bits 3b, 3b+1, 3b+2;
 * ties kept in caller order).
 */
vm_status vm_debug_tree(vm_ctx *ctx, uint32_t *keys, int32_t *perm, int32_t *leaf_start);

/*
 * Debug views of the expansions of the last vm_fmm_eval (stream-ordered copies):
 *   which 0: multipoles, 1: locals, at `level`; raw layout [8^level][3][kp] with
 *   kp = (p+1)^2 rounded up to a multiple of 32, element type double (FP64
 *   form) or float (mixed form); *bytes receives the size.  `out` is a device
 *   buffer of at least that size, or NULL to query the size only.
 * vm_debug_far: far-field velocity and gradient per target in sorted order,
 *   device double [12][n] (u_x, u_y, u_z, then J[3a+b]): the last
 *   vm_fmm_eval / vm_fmm_eval_at evaluates it again from its local expansions
 *   (its L2P adds the far field straight into the outputs).
 */
vm_status vm_debug_expansions(vm_ctx *ctx, int which, int level, void *out, int64_t *bytes);
vm_status vm_debug_far(vm_ctx *ctx, double *out);

/*
 * Host-only views of the interaction structure (no device work).
 * vm_debug_offsets: the 316 distinct M2L offsets d = source - target (cells),
 *   sorted by (dz, dy, dx); out int8 [316][3]; returns the count in *count.
 * vm_debug_list: M2L list of one cell `key` at `level` (periodic 0/1): up to
 *   189 entries of source key (int32 src[]), offset (int8 d[][3]) and image
 *   shift (int8 img[][3]) in (dz, dy, dx) order of d; *count receives the length.
 */
vm_status vm_debug_offsets(int8_t *out, int *count);
vm_status vm_debug_list(int level, int periodic, int32_t key, int32_t *src, int8_t *d,
                        int8_t *img, int *count);

/*
 * Host-only: the translation operators in the library's real basis, FP64,
 * row-major C x C with C = (p+1)^2 unless stated (no device work).
 *   kind 0: M2L for offset index `index` (0..315, the vm_debug_offsets order)
 *   kind 1: M2M for child octant `index` (0..7)
 *   kind 2: L2L for child octant `index` (0..7)
 *   kind 3: periodic lattice operator for K = `index` (1..4)
 *   kind 4: derivative table of the multipole basis, 3 p^2 x C (not C x C):
 *           row a p^2 + s (a < 3, s < p^2) holds the coefficients of c_s in
 *           dF/dY_a for F(Y) = sum_t f_t c_t(Y), c = [Rb^0, Re Rb^m, -Im Rb^m]
 *           (index is ignored)
 * The basis: solid harmonics R_n^m = r^n P_n^m(cos t) e^{i m phi} / (n+m)!
 * (P with the Condon-Shortley phase) scaled by sqrt((n+m)!(n-m)!); a cell of
 * width w stores M_n^m = sum_j q_j conj(R_n^m((x_j - c)/w)) and locals with
 * phi(x) = (1/w) sum_n,m L_n^m R_n^m((x - c)/w); real index n^2 holds m = 0,
 * n^2 + 2m - 1 and n^2 + 2m the real and imaginary parts of m > 0.
 */
vm_status vm_debug_operator(int kind, int p, int index, double *out);

#ifdef __cplusplus
}
#endif
#endif /* VMFMM_H */
