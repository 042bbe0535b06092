/*
 * stokes.h -- C ABI of libstokes.so: free-space Stokes kernel sums for
 * slender-body fiber suspensions on one AMD Instinct MI355X (gfx950).
 *
 * Method: Nazockdast, Rahimian, Zorin, Shelley, "A fast platform for
 * simulating flexible fiber suspensions applied to cell mechanics"
 * (arXiv:1602.05650).  The library evaluates, directly and on the GPU, the
 * kernel sums that the paper's solver needs at every GMRES iteration:
 *   - the Stokeslet + source-doublet sum over fiber nodes (section 2,
 *     eq. oseen and eq. main-sb-vel; the fiber-fiber part of the
 *     complementary flow, eq. complementary-uf),
 *   - the stresslet double-layer sum over surface quadrature points
 *     (eq. stresslet, eq. double-layer, with the on-surface singularity
 *     subtraction of section "Singular integrals over surfaces"),
 *   - the local slender-body operator and its inverse (eq. main-sb-local),
 *   - the fiber mobility solve by preconditioned GMRES (section "Linear
 *     solver and preconditioner", eq. prec) and a continuous-batching
 *     serving session that runs many such solves at once.
 *
 * Conventions common to every entry point
 *   Status      every function returns int: STOKES_OK (0) or a positive
 *               STOKES_E_* code.  stokes_status_string() names a code,
 *               stokes_last_error() returns a thread-local message for the
 *               last failure on the calling thread.  No C++ exception
 *               crosses the ABI.  On a validation error nothing is launched
 *               and the outputs are untouched.
 *   Pointers    the *_eval, stokes_local_sbt and stokes_mobility_solve
 *               entry points take DEVICE pointers (memory of the current HIP
 *               device) and a HIP stream passed as void* (NULL = the legacy
 *               default stream).  They are asynchronous on that stream unless
 *               a diagnostics struct or STOKES_CHECK_INPUTS is passed, which
 *               makes the call wait for the stream.  Sessions take HOST
 *               pointers and copy them.
 *   Layout      point sets are structure-of-arrays float64: n points are
 *               three planes x[0..n) y[0..n) z[0..n) stored back to back
 *               (element (c, i) at index c*n + i).  Outputs use the same
 *               layout.
 *   Ownership   the caller owns every input and output buffer and keeps it
 *               alive until the stream work completes.  The library owns a
 *               per-(device, stream) scratch workspace that grows on demand
 *               (growing it waits for that stream) and is freed by
 *               stokes_release_workspace().  Calls on different streams may
 *               run concurrently; calls on one stream are ordered.
 *   Precision   STOKES_PREC_FP64: every pair in FP64.  STOKES_PREC_MIXED:
 *               pairs farther than the near radius in FP32 with
 *               Kahan-compensated FP32 accumulation per target; nearer pairs
 *               (by the same FP32 distance test, so each pair is counted
 *               once) are recomputed in FP64 from the FP64 coordinates.
 *   Results     for fixed inputs and flags every result is bitwise
 *               reproducible: the source partition and the reduction order
 *               depend only on the problem sizes.
 */
#ifndef STOKES_H_
#define STOKES_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define STOKES_OK          0
#define STOKES_E_INVAL     1  /* invalid argument (null pointer with n > 0, n < 0, mu <= 0, eps outside (0, 0.5), ...) */
#define STOKES_E_NOMEM     2  /* device or host allocation failed, or a request can never fit a session's budget */
#define STOKES_E_DEVICE    3  /* a HIP call failed; stokes_last_error() holds hipGetErrorString */
#define STOKES_E_NONFINITE 4  /* STOKES_CHECK_INPUTS found a NaN or Inf in an input */
#define STOKES_E_BUSY      5  /* session queue full */
#define STOKES_E_CANCELED  6  /* request cancelled, or session destroyed with the request pending */
#define STOKES_E_TIMEOUT   7  /* stokes_session_wait timed out; the request is still running */
#define STOKES_E_NOTFOUND  8  /* unknown or already collected ticket */

/* ---- flags ------------------------------------------------------------- */
#define STOKES_PREC_FP64        0u   /* every pair in FP64 (default) */
#define STOKES_PREC_MIXED       1u   /* FP32 far pairs + Kahan, FP64 near pairs */
#define STOKES_EXCL_SELF_POINT  2u   /* skip source trg_self[i] for target i (self-pairs excluded) */
#define STOKES_EXCL_SAME_FIBER  4u   /* skip every source of the target's fiber (eq. complementary-uf) */
#define STOKES_NO_DOUBLET       8u   /* single layer: Stokeslet only (drop the eps^2/2 doublet) */
#define STOKES_ACCUMULATE      16u   /* add into u_out instead of overwriting it */
#define STOKES_CHECK_INPUTS    32u   /* scan device inputs first (finite values, fiber ids); synchronous */
#define STOKES_ONSURF_RAW      64u   /* double layer: no singularity subtraction on the surface */
#define STOKES_NONLOCAL       128u   /* mobility solve: include the nonlocal self term K_delta */
#define STOKES_PRECOND_BLOCK  256u   /* mobility solve: fiber block-Jacobi preconditioner */
#define STOKES_EAGER          512u   /* particle solve: launch each iteration's kernels one by one
                                        instead of replaying a captured HIP graph (same result) */

/* Optional counters filled by the *_eval calls (passing one makes the call synchronous). */
typedef struct stokes_diag {
    int64_t pairs;       /* (target, source) pairs in the sum; excluded pairs are not counted */
    int64_t near_pairs;  /* pairs recomputed in FP64 by the mixed path (0 for FP64) */
    int64_t coincident;  /* non-excluded pairs at zero distance: skipped, never Inf */
} stokes_diag;

/*
 * stokes_sl_eval -- single-layer (Stokeslet + doublet) sum over fiber nodes.
 *
 *   u_i = sum_{j not excluded}  w_j [ G(d) f_j + c_j W(d) f_j ],   d = x_i - y_j
 *   G(d) f = (1/(8 pi mu)) (f/|d| + d (d.f)/|d|^3)           eq. oseen
 *   W(d) f = (1/(8 pi mu)) (f/|d|^3 - 3 d (d.f)/|d|^5)        eq. main-sb-vel (doublet)
 *   c_j    = (eps L_{m(j)})^2 / 2                             eq. main-sb-vel, eps = a/L
 *
 * n_src       number of sources (fiber nodes), >= 0.
 * src_xyz     [3*n_src]  source positions (SoA).
 * src_force   [3*n_src]  force f_j at each node (SoA).
 * src_weight  [n_src] or NULL (all 1): quadrature weight w_j, e.g. Clenshaw-Curtis x L/2.
 * src_fiber   [n_src] or NULL: fiber id of each node, non-decreasing, in [0, n_fib),
 *             nodes of one fiber contiguous.  Required for STOKES_EXCL_SAME_FIBER.
 * n_fib       number of fibers (length of fiber_len); 0 if src_fiber is NULL.
 * fiber_len   [n_fib] or NULL (all 1): fiber lengths L_m.  With src_fiber NULL,
 *             fiber_len[0] (if given) is used for every node.
 * n_trg       number of targets; ignored (= n_src) when trg_xyz is NULL.
 * trg_xyz     [3*n_trg] target positions, or NULL: the targets are the sources.
 * trg_self    [n_trg] or NULL: source index that target i must skip under
 *             STOKES_EXCL_SELF_POINT (-1: none).  NULL means i when the
 *             targets are the sources, none otherwise.
 * trg_fiber   [n_trg] or NULL: fiber id of target i for STOKES_EXCL_SAME_FIBER
 *             (-1: none).  NULL means src_fiber[i] when the targets are the sources.
 * mu          viscosity, > 0.     eps  slenderness a/L, in (0, 0.5).
 * near_r      mixed path only: pairs with |d| < max(near_r, 2 eps L_{m(j)}) are
 *             evaluated in FP64 (the spec rule is two fiber radii; a
 *             larger radius trades speed for accuracy).  <= 0: two radii.
 * flags       STOKES_PREC_*, at most one STOKES_EXCL_*, STOKES_NO_DOUBLET,
 *             STOKES_ACCUMULATE, STOKES_CHECK_INPUTS.
 * u_out       [3*n_trg] velocities (SoA, FP64), written or accumulated.
 * stream      hipStream_t or NULL.     diag  NULL or counters (synchronous).
 */
int stokes_sl_eval(int64_t n_src, const double* src_xyz, const double* src_force,
                   const double* src_weight, const int32_t* src_fiber, int32_t n_fib,
                   const double* fiber_len,
                   int64_t n_trg, const double* trg_xyz, const int64_t* trg_self,
                   const int32_t* trg_fiber,
                   double mu, double eps, double near_r, uint32_t flags,
                   double* u_out, void* stream, stokes_diag* diag);

/*
 * stokes_sl_eval_noalloc -- stokes_sl_eval for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same sum, arguments and layouts, on the same stream rules, but its
 * scratch (tiles, source packs, exclusion ranges, chunk partials) is a static array
 * of 64 MiB per GPU in the library's device code, held until the process ends, and
 * the call allocates nothing (no hipMalloc, hipFree or allocating library routine).
 *   - The caller passes every input and the output, as for stokes_sl_eval.
 *   - No diagnostics argument; STOKES_CHECK_INPUTS is rejected (E_INVAL).
 *   - A problem whose scratch does not fit 64 MiB even with one source chunk is
 *     rejected with E_INVAL (about 5e5 sources and targets together); larger ones
 *     fit with fewer source chunks than stokes_sl_eval takes, so the reduction order
 *     and the last bits of the result can differ from it (within the precision's bound).
 *   - Every call on one GPU uses that GPU's one array and it keeps the last call's
 *     contents: calls that overlap on one GPU (other streams or threads) race.
 */
int stokes_sl_eval_noalloc(int64_t n_src, const double* src_xyz, const double* src_force,
                           const double* src_weight, const int32_t* src_fiber, int32_t n_fib,
                           const double* fiber_len,
                           int64_t n_trg, const double* trg_xyz, const int64_t* trg_self,
                           const int32_t* trg_fiber,
                           double mu, double eps, double near_r, uint32_t flags,
                           double* u_out, void* stream);

/*
 * stokes_dl_eval -- double-layer (stresslet) sum over surface quadrature points.
 *
 *   u_i = (3/(4 pi)) sum_{s != self(i)} w_s (d . qt_s)(d . n_s) d / |d|^5,   d = x_i - y_s
 *
 * eq. double-layer with the stresslet of eq. stresslet.  Sign reading: with
 * the OUTWARD unit normal n, a constant density q gives -q inside the
 * surface, 0 outside and -q/2 on it (principal value): the paper's stresslet
 * with the normal pointing into the fluid enclosed by the periphery, the
 * convention that makes eq. main-cortex-density consistent.  The viscosity
 * factor of eq. stresslet is dropped (q is a velocity).
 *
 * Default (subtraction): for a target with self(i) >= 0 (a surface point),
 * qt_s = q_s - q_{self(i)} and -q_{self(i)}/2 is added afterwards, which
 * returns the principal value (section "Singular integrals over surfaces").
 * STOKES_ONSURF_RAW: qt_s = q_s and the self point is only left out.
 * Off-surface targets (self < 0) always use qt_s = q_s.
 *
 * n_src       number of surface points.   src_xyz [3*n_src] positions.
 * src_normal  [3*n_src] outward unit normals.    src_weight [n_src] area weights.
 * src_q       [3*n_src] density q.
 * n_trg / trg_xyz   targets, or trg_xyz NULL: the targets are the surface points.
 * trg_self    [n_trg] or NULL: surface index of target i (-1: off surface).
 *             NULL means i when the targets are the surface points, else -1.
 * near_r      mixed path only: pairs with |d| < near_r are evaluated in FP64.
 *             <= 0 selects 0.02.
 * flags       STOKES_PREC_*, STOKES_ONSURF_RAW, STOKES_ACCUMULATE, STOKES_CHECK_INPUTS.
 */
int stokes_dl_eval(int64_t n_src, const double* src_xyz, const double* src_normal,
                   const double* src_weight, const double* src_q,
                   int64_t n_trg, const double* trg_xyz, const int64_t* trg_self,
                   double near_r, uint32_t flags,
                   double* u_out, void* stream, stokes_diag* diag);

/*
 * stokes_local_sbt -- local slender-body operator at every node (FP64):
 *   inverse = 0:  out = M f = (1/(8 pi mu)) [ -ln(eps^2 e)(I + t t) + 2 (I - t t) ] f
 *   inverse = 1:  out = M^{-1} f = 8 pi mu [ t t / (2 kappa) + (I - t t)/(kappa + 2) ] f,
 *                 kappa = -ln(eps^2 e)  (the 3x3 node blocks of the block-Jacobi
 *                 preconditioner, eq. prec, for the local operator)
 * eq. main-sb-local.  n nodes; tangent [3*n] unit tangents X_s; f, out [3*n];
 * out may alias f.  Asynchronous on stream.
 */
int stokes_local_sbt(int64_t n, const double* tangent, const double* f, double eps, double mu,
                     int inverse, double* out, void* stream);

/*
 * stokes_nonlocal_sbt -- the regularised nonlocal self-interaction of every
 * fiber (eq. sb-stokes-reg), FP64:
 *   out_i = sum over the other nodes k of node i's fiber of
 *           w_k [ |r|/sqrt(|r|^2 + delta^2) G(r) f_k
 *                 - (I + t_i t_i) f_i / (8 pi mu sqrt((s_i - s_k)^2 + delta^2)) ],
 *   r = X_i - X_k, G(r) = (I/|r| + r r/|r|^3)/(8 pi mu), w_k the Clenshaw-Curtis
 *   weight x L/2 (section "Integration over fiber centerlines") and s_k = (L/2)(1 +
 *   alpha_k) the arc length; the s' = s node contributes nothing (both parts of the
 *   integrand have the same limit there).
 * n_fib, nodes_per_fib (2..64), xyz, tangent, f, out [3*N] SoA as for the mobility
 * solve, fiber_len [n_fib]; delta > 0, mu > 0.  out must not alias f.  Uses the
 * stream's workspace; asynchronous on stream.
 */
int stokes_nonlocal_sbt(int32_t n_fib, int32_t nodes_per_fib, const double* xyz,
                        const double* tangent, const double* fiber_len, const double* f,
                        double delta, double mu, double* out, void* stream);

/*
 * stokes_far -- far field of the u_bar sums of stokes_mobility_solve and
 * stokes_fiber_step through the treecode of stokes_tree_* (section "Matrix-vector
 * products and FMM": the paper evaluates these sums with a fast summation at every
 * GMRES iteration).  A plan is built once per call from the fiber nodes (targets =
 * sources, same-fiber exclusion); every iteration's sum then runs on it.  Its error
 * against the direct sum is set by degree and theta as for stokes_tree_create.
 * Pass NULL for the direct sums.
 */
typedef struct stokes_far {
    int32_t degree;      /* 1..10 */
    double theta;        /* (0, 1) */
    int32_t leaf_size;   /* >= 1; <= 0 selects 128 */
} stokes_far;

/*
 * stokes_mobility_solve -- fiber mobility solve on device pointers.
 *
 * Finds forces f with  M f [+ K_delta f] + u_bar[f] = V  at every fiber node,
 * where M is the local slender-body operator (eq. main-sb-local), K_delta the
 * nonlocal self term (eq. sb-stokes-reg; with STOKES_NONLOCAL) and u_bar[f] the
 * flow of all OTHER fibers (eq. complementary-uf): the Stokeslet + doublet sum
 * with Clenshaw-Curtis weights x L/2 and the own fiber excluded.
 * Right-preconditioned GMRES (section "Linear solver and preconditioner"),
 * x0 = 0, classical Gram-Schmidt applied twice, Givens rotations, in FP64;
 * `iters` iterations unless the Krylov space is exhausted (exact breakdown).
 * Preconditioner: the local node blocks M^{-1}, or with STOKES_PRECOND_BLOCK
 * each fiber's self block M [+ K_delta] inverted once (Gauss-Jordan with partial
 * pivoting, FP64) and applied as a dense product.
 *
 * n_fib, nodes_per_fib   fibers and CGL nodes per fiber (2..64); N = n_fib*nodes_per_fib.
 * xyz, tangent           [3*N] node positions and unit tangents, fiber-contiguous,
 *                        node k of a fiber at alpha_k = cos(k pi/(nodes-1)).
 * fiber_len              [n_fib] lengths.     rhs  [3*N] fiber velocities V.
 * delta                  regularisation of K_delta (> 0 with STOKES_NONLOCAL, else unused).
 * iters                  1..STOKES_MAX_ITERS.  flags: STOKES_PREC_* for the sums,
 *                        STOKES_NO_DOUBLET, STOKES_NONLOCAL, STOKES_PRECOND_BLOCK.
 * f_out                  [3*N] forces.   resid_out: NULL or host double, the final
 *                        least-squares residual norm.  iters_out: NULL or host int.
 * far                    NULL (direct u_bar sums) or the treecode's parameters.
 * Synchronous (waits for the stream at the end).
 */
#define STOKES_MAX_ITERS 128
int stokes_mobility_solve(int32_t n_fib, int32_t nodes_per_fib, const double* xyz,
                          const double* tangent, const double* fiber_len, const double* rhs,
                          double eps, double mu, double delta, int32_t iters, uint32_t flags,
                          double* f_out, double* resid_out, int32_t* iters_out,
                          const stokes_far* far, void* stream);

/*
 * stokes_fiber_step -- one implicit (backward Euler) time step of free elastic
 * fibers (section "Time discretization"), fixed lengths, no rigid bodies.
 *
 * Finds X+ and the tension T+ with (eq. discrete-update, fiber rows)
 *   (X+ - X) / dt = V[f+ + f_ext],   f+ = -E X+_ssss + (T+ X_s)_s   (X_s explicit)
 *   V[f] = M f [+ K_delta f] + u_bar[f]   (eq. main-sb-local, eq. sb-stokes-reg with
 *          STOKES_NONLOCAL, and the other fibers' flow of eq. complementary-uf, all
 *          implicit), the inextensibility constraint in the velocity form of
 *   eq. main-inextensibility, t . (V[f+ + f_ext])_s = 0, taken as a second-order equation
 *   for T: the node-by-node part A = alpha I + beta t t of V (M, and the subtracted
 *   local part of K_delta) is differentiated with the arclength identities
 *   (t . X_ss = 0, t . X_sss = -|X_ss|^2, t . X_ssss = -3 X_ss . X_sss), the rest of V with
 *   D_s; and the free-end conditions of eq. bc-free (X_ss = X_sss = 0, T = 0 at both ends).
 * Discretisation: Chebyshev differentiation on the CGL nodes by the coefficient
 * recursion (section "Fiber representation"); the position equations collocated at
 * nodes_per_fib - 4 and the tension equation at nodes_per_fib - 2 first-kind
 * Chebyshev points, completed by the boundary rows (rectangular collocation).
 * Solved for the increment (X+ - X, T+) by right-preconditioned GMRES in FP64 from
 * zero, with each fiber's self block (its rows without u_bar: 4 n x 4 n) inverted by
 * Gauss-Jordan as block-Jacobi preconditioner (section "Linear solver and
 * preconditioner"); iterations stop after `iters`, at exact breakdown, or when the
 * least-squares residual is <= tol x |rhs|.
 *
 * n_fib, nodes_per_fib   fibers (>= 0) and CGL nodes per fiber (6..48); N = n_fib*nodes.
 * xyz        [3*N] node positions (x of every node, then y, then z), fiber-contiguous,
 *            node k of a fiber at alpha_k = cos(k pi/(nodes-1)) (node 0: s = L).
 * fiber_len  [n_fib] lengths L.    f_ext [3*N] external force density at the nodes.
 * clamp_minus  [n_fib] int32 or NULL: attaches that fiber's minus end (s = 0, node
 *            nodes-1) to a body at rest (U = Omega = 0).  0: both ends free.  2: hinged,
 *            the end keeps its position and is torque free (X_ss = 0, the condition
 *            stated beside eq. BC2-2).  Any other value:
 *            clamped (eq. BC2-1, BC2-2), the end keeps its position and tangent.  An
 *            attached end has no tangential velocity (tangential part of eq. BC2-T).
 * eps        slenderness in (0, 0.5);  E >= 0 bending modulus;  dt > 0;  mu > 0.
 * delta      regularisation of K_delta (> 0 with STOKES_NONLOCAL, else unused).
 * near_r     mixed single-layer sums only (see stokes_sl_eval).
 * iters      1..STOKES_MAX_ITERS;  tol >= 0 (0: run all iterations).
 * flags      STOKES_PREC_* for the u_bar sums, STOKES_NO_DOUBLET, STOKES_NONLOCAL.
 * far        NULL (direct u_bar sums) or the treecode's parameters (stokes_far).
 * xyz_out    [3*N] X+ (must not alias xyz or f_ext).   T_out [N] T+ at the nodes.
 * resid_out, iters_out   NULL or host: final least-squares residual, iterations.
 * All arrays are DEVICE pointers.  The call is synchronous.  Its device memory, about
 * (16 n + 3 iters + 30) N doubles plus 37 n^2 per fiber of a 512-fiber chunk, is kept
 * per (device, stream) for the next call and released by stokes_release_workspace;
 * calls on one stream must therefore not overlap.  The preconditioner's blocks are
 * formed on a side stream that the library creates beside `stream` (one per caller
 * stream, default priority, released with the buffer) and joined back into `stream`.
 */
int stokes_fiber_step(int32_t n_fib, int32_t nodes_per_fib, const double* xyz,
                      const double* fiber_len, const double* f_ext, const int32_t* clamp_minus,
                      double eps, double E,
                      double dt, double mu, double delta, double near_r, int32_t iters,
                      double tol, uint32_t flags, double* xyz_out, double* T_out,
                      double* resid_out, int32_t* iters_out, const stokes_far* far,
                      void* stream);

/*
 * stokes_particle_solve -- mobility of rigid particles in a fixed confining
 * periphery: the second-kind boundary integral equations of sections "The
 * contribution from the periphery" and "The contribution from rigid immersed
 * particles" (eq. main-cortex-density with the rank completion
 * N[q0](x) = n(x) int n.q0 dS, eq. main-nsb-second-kind, constraints
 * eq. main-nsb-rgbt and eq. main-nsb-rgbr), Nystrom on the given surface
 * quadratures with singularity subtraction, external forces and torques
 * through the Stokeslet and rotlet (eq. oseen, eq. rotlet).  With K the double
 * layer of stokes_dl_eval (outward normals), the paper's double layer with the
 * normal into the fluid is +K on the periphery and -K on a particle.  Right-
 * preconditioned GMRES in FP64 with the diagonal of the self blocks (eq. prec).
 *
 * m0, y0, n0, w0     periphery: points, OUTWARD unit normals [3*m0], area weights
 *                    [m0]; m0 = 0 for an unbounded fluid.
 * n_part (>= 1), part_offset   HOST array [n_part+1], part_offset[0] = 0: particle p
 *                    owns points [part_offset[p], part_offset[p+1]) (>= 4 each).
 * yp, np, wp         particle points, outward normals [3*Mp], weights [Mp],
 *                    Mp = part_offset[n_part].
 * centers, force, torque   [3*n_part] (SoA: x of every particle, then y, then z):
 *                    X_p, F_p, L_p.
 * mu > 0; near_r: mixed double-layer sums only (see stokes_dl_eval);
 * iters 1..STOKES_MAX_ITERS; flags: STOKES_PREC_* for the double-layer sums;
 * STOKES_EAGER launches each iteration's kernels one by one instead of replaying the
 * iteration captured into HIP graphs (the default; the results are the same, bit for
 * bit).  The capture runs on a stream the call creates (the caller's may be the null
 * stream) and the replays on `stream`.  The double layers of all surfaces are one sum
 * over all points (each surface's own term in principal value).
 * U_out, Omega_out   [3*n_part] translational and angular velocities (SoA).
 * q_out              NULL or [3*(m0+Mp)] densities (periphery points first).
 * resid_out, iters_out   NULL or host: final least-squares residual, iterations.
 * All arrays except part_offset are DEVICE pointers.  The call allocates its own
 * scratch (about (3 iters + 30)(m0 + Mp) doubles) and is synchronous.  Errors:
 * E_INVAL (sizes, pointers, flags), E_NOMEM, E_DEVICE.
 */
int stokes_particle_solve(int64_t m0, const double* y0, const double* n0, const double* w0,
                          int32_t n_part, const int64_t* part_offset, const double* yp,
                          const double* np, const double* wp, const double* centers,
                          const double* force, const double* torque, double mu, double near_r,
                          int32_t iters, uint32_t flags, double* U_out, double* Omega_out,
                          double* q_out, double* resid_out, int32_t* iters_out, void* stream);

/* ---- far-field acceleration: barycentric Lagrange treecode ---------------
 *
 * The single-layer sum of stokes_sl_eval (Stokeslet + doublet) with the far
 * field approximated, as the paper does with its fast multipole method (section
 * "Matrix-vector products and FMM"), here by a kernel-independent treecode
 * (barycentric Lagrange interpolation at Chebyshev points of the second kind,
 * the published method of Wang, Krasny and Tlupova, 2020).  A source cluster C
 * acts on a target batch B (at most 64 targets) through (degree+1)^3 proxy
 * points when (r_B + r_C) < theta |c_B - c_C| and C holds more sources than
 * proxies; otherwise its children are visited, and leaves (at most leaf_size
 * sources) are summed directly with the pair arithmetic of stokes_sl_eval
 * (mixed: FP32 with FP64 near pairs).  The error against the exact sum is
 * controlled by degree and theta (about 1e-6 relative at degree 6, theta 0.7).
 *
 * stokes_tree_create  builds the trees and interaction lists on the host from
 *   DEVICE positions src_xyz [3*n_src] and trg_xyz [3*n_trg] (NULL: the targets
 *   are the sources); degree 1..10, theta in (0, 1), leaf_size >= 1.  The plan
 *   holds the geometry on the device until stokes_tree_destroy.  Synchronous.
 * stokes_tree_sl_eval  one sum on a plan: src_force [3*n_src], src_weight
 *   [n_src] or NULL, src_fiber / n_fib / fiber_len as in stokes_sl_eval (or
 *   src_fiber and fiber_len both NULL: L = 1; an id outside [0, n_fib) takes L = 1),
 *   mu, eps, near_r; flags STOKES_CHECK_INPUTS (the scan of stokes_sl_eval:
 *   finite forces, weights and lengths, ids in range and non-decreasing;
 *   synchronous), STOKES_PREC_*, STOKES_EXCL_SELF_POINT or
 *   STOKES_EXCL_SAME_FIBER (one of the two; plans built with targets = sources
 *   only; the fiber mode needs src_fiber, non-decreasing as in stokes_sl_eval, and
 *   subtracts exactly the own-fiber sources that the far field took through
 *   proxies), STOKES_NO_DOUBLET, STOKES_ACCUMULATE; u_out [3*n_trg].  Asynchronous on stream; the plan's buffers are reused, so
 *   evaluations on one plan must not overlap.
 * stokes_tree_dl_eval  the double-layer sum of stokes_dl_eval on a plan:
 *   src_normal [3*n_src] outward unit normals, src_weight [n_src] area weights,
 *   src_q [3*n_src] density (all required); near_r as in stokes_dl_eval (mixed
 *   only: direct pairs closer than near_r in FP64; <= 0 selects 0.02); flags
 *   STOKES_PREC_* (mixed: FP32 proxies and direct pairs), STOKES_ONSURF_RAW,
 *   STOKES_ACCUMULATE; u_out [3*n_trg].  A proxy
 *   carries the charges M_k = sum L_k(y_j) q_j (w_j n_j)^T and
 *   N_k = sum L_k(y_j) w_j n_j, so that the singularity subtraction (q_j - q_i)
 *   of a surface target i carries over to the far field.  Plans built with
 *   targets = sources subtract (unless STOKES_ONSURF_RAW); other plans' targets
 *   are off the surface.  Same stream and reuse rules as stokes_tree_sl_eval (the
 *   two share the plan's buffers).
 * stokes_tree_info     pair counts of one evaluation (targets x proxies and
 *   targets x direct sources), proxy clusters and target batches.
 */
typedef struct stokes_tree stokes_tree;
int stokes_tree_create(int64_t n_src, const double* src_xyz, int64_t n_trg, const double* trg_xyz,
                       int32_t degree, double theta, int32_t leaf_size, void* stream,
                       stokes_tree** out);
int stokes_tree_sl_eval(stokes_tree* t, const double* src_force, const double* src_weight,
                        const int32_t* src_fiber, int32_t n_fib, const double* fiber_len, double mu,
                        double eps, double near_r, uint32_t flags, double* u_out, void* stream);
int stokes_tree_dl_eval(stokes_tree* t, const double* src_normal, const double* src_weight,
                        const double* src_q, double near_r, uint32_t flags, double* u_out,
                        void* stream);
int stokes_tree_info(const stokes_tree* t, int64_t* proxy_pairs, int64_t* direct_pairs,
                     int32_t* n_proxy_clusters, int32_t* n_batches);
int stokes_tree_destroy(stokes_tree* t);

/* ---- serving: continuous batching of mobility solves ------------------- */
typedef struct stokes_session stokes_session;

typedef struct stokes_session_cfg {
    int64_t hbm_budget_bytes;  /* device memory the session may hold for requests (> 0) */
    int32_t max_slots;         /* requests in flight at once, 1..256 */
    int32_t max_queue;         /* submitted but not admitted requests, >= 1 */
    uint32_t flags;            /* STOKES_PREC_* and STOKES_NO_DOUBLET for every request */
    int32_t device;            /* HIP device ordinal */
    int64_t step_pairs;        /* pair budget of one request's single-layer work in one
                                  step: a larger matvec is spread over several steps so
                                  that small requests in flight keep advancing every
                                  step (results are unchanged, bit for bit).  0: the
                                  default (STOKES_STEP_PAIRS_DEFAULT); < 0: no limit. */
} stokes_session_cfg;

#define STOKES_STEP_PAIRS_DEFAULT 4000000000LL

typedef struct stokes_solve_req {   /* HOST pointers; copied by stokes_session_submit */
    int32_t n_fib;
    int32_t nodes_per_fib;          /* 2..64 */
    const double* xyz;              /* [3*N] SoA node positions */
    const double* tangent;          /* [3*N] SoA unit tangents */
    const double* fiber_len;        /* [n_fib] */
    const double* rhs;              /* [3*N] SoA fiber velocities V */
    double eps;
    double mu;
    int32_t iters;                  /* GMRES iterations, 1..STOKES_MAX_ITERS */
    uint64_t tag;                   /* returned in the stats */
    uint32_t flags;                 /* STOKES_NONLOCAL, STOKES_PRECOND_BLOCK (or 0) */
    double delta;                   /* K_delta regularisation (> 0 with STOKES_NONLOCAL) */
    const stokes_far* far;          /* NULL (direct u_bar sums) or the treecode's parameters
                                       for this request's u_bar sums (copied at submit).  Its
                                       tree plan is built at admission from the request's
                                       nodes and held outside the HBM budget until the
                                       request finishes; the request then advances one
                                       iteration per step with launches of its own after the
                                       step's graph (paper section 3, "Matrix-vector products
                                       and FMM"). */
} stokes_solve_req;

typedef struct stokes_solve_stats {
    int64_t t_submit_ns;            /* CLOCK_MONOTONIC stamps */
    int64_t t_admit_ns;
    int64_t t_finish_ns;
    int32_t iters;                  /* iterations run */
    int32_t status;                 /* STOKES_OK or an error code */
    double residual;                /* final least-squares residual norm */
    uint64_t tag;
} stokes_solve_stats;

/* Create a session (a worker thread, one stream, device slot memory on demand). */
int stokes_session_create(const stokes_session_cfg* cfg, stokes_session** out);
/* Copy a request and queue it; returns at once.  E_NOMEM if it can never fit the
 * budget, E_BUSY if the queue is full, E_INVAL for bad sizes, E_NONFINITE if an
 * input holds a NaN or Inf. */
int stokes_session_submit(stokes_session* s, const stokes_solve_req* req, uint64_t* ticket);
/* Wait for a ticket (timeout_ms < 0: forever) and collect it: the ticket is
 * released unless the wait times out.  f_out: NULL or host [3*N].  Only one
 * thread may wait for a ticket at a time (a second one gets STOKES_E_BUSY). */
int stokes_session_wait(stokes_session* s, uint64_t ticket, double* f_out,
                        stokes_solve_stats* st, int32_t timeout_ms);
/* Device bytes a request of this shape takes from a session's budget (flags:
 * the session's STOKES_PREC_* and the request's STOKES_PRECOND_BLOCK, whose
 * inverted fiber blocks take 72 nodes_per_fib^2 bytes per fiber).  Returns 0 for
 * invalid shapes. */
int64_t stokes_solve_footprint(int32_t n_fib, int32_t nodes_per_fib, int32_t iters, uint32_t flags);
/* Test hook for failure handling: the session's next step reports a device
 * error for every request then in flight (their waits return STOKES_E_DEVICE);
 * queued requests are not affected and the session keeps serving. */
int stokes_session_inject_fault(stokes_session* s);
/* Cancel a queued or running request; its wait returns STOKES_E_CANCELED. */
int stokes_session_cancel(stokes_session* s, uint64_t ticket);
/* Stop the worker; pending requests finish with STOKES_E_CANCELED. */
int stokes_session_destroy(stokes_session* s);

/* ---- measurement ---------------------------------------------------------- */
/* While enabled, every launch of a main pair-sum kernel (single or double layer,
 * FP64 or mixed, one-shot or batched) is bracketed by two HIP events recorded on
 * the stream it is launched on.  stokes_profile_read waits for those events,
 * returns the summed kernel milliseconds and the number of launches since the
 * last read, and resets both.  Host pointers; either may be NULL. */
int stokes_profile_enable(int on);
int stokes_profile_read(double* ms, int64_t* launches);

/* ---- misc --------------------------------------------------------------- */
const char* stokes_status_string(int status);
const char* stokes_last_error(void);
/* Free every scratch workspace of the calling process (waits for the device), and the
 * pinned tables and events that finished solves leave for the next solve on their
 * device.  Not to be called while another thread's call into the library runs. */
int stokes_release_workspace(void);
/* Library version: major*10000 + minor*100 + patch. */
int stokes_version(void);

#ifdef __cplusplus
}
#endif
#endif /* STOKES_H_ */
