/*
 * semcond.h -- C ABI of the MI355X (gfx950) statically condensed spectral-element
 * Helmholtz solver.
 *
 * Problem (Huismann, Stiller & Froehlich, "Factorizing the factorization",
 * arXiv 1601.08179, Sec. 3, eq. helmholtz_equation):  lambda*u - Laplace(u) = f
 * on a box meshed by n1 x n2 x n3 Cartesian elements with per-axis widths, GLL
 * degree p in every direction, lambda >= 0, Dirichlet or natural conditions per
 * domain face.  The library solves the statically condensed system of Sec. 4
 * (eq. condensation_system) for the element skeleton, with the operator applied
 * in the fast-diagonalisation ("transformed") basis of Sec. 6 (Table 2,
 * Algorithm 4), preconditioned conjugate gradients with the preconditioner that
 * is diagonal in that basis (the "BT" solver of Sec. 8).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Element (e1,e2,e3) has linear number e = e1 + n1*(e2 + n2*e3).
 * - Global GLL node (I1,I2,I3), 0 <= I_a <= n_a*p, has nodal number
 *   I1 + (n1*p+1)*(I2 + (n2*p+1)*I3).  N = prod(n_a*p+1).  "Nodal" arrays are
 *   [k][N] (right-hand side major), FP64 unless stated.
 * - "Skeleton" arrays hold the N_s nodes on element faces, edges and vertices,
 *   entity-major with the right-hand-side index innermost: [N_s][k].  The order
 *   of skeleton slots is fixed by the library; semcond_skeleton_coords() gives
 *   the global (I1,I2,I3) of every slot.  Slots on Dirichlet faces exist and
 *   are ignored on input and written as 0 on output.
 * - A skeleton array is either in the PHYSICAL basis (nodal values) or in the
 *   TRANSFORMED basis of Sec. 6: per face u~ = (S^-1 (x) S^-1) u over its two
 *   interior directions, per edge u~ = S^-1 u, vertices unchanged, where the
 *   n_I x n_I matrix S (n_I = p-1) satisfies S^T M_II S = I, S^T K_II S = Lambda
 *   (Sec. 5, eq. generalized_eigenvalues, in the transpose convention that
 *   makes H_II^-1 = (S(x)S(x)S) D^-1 (S(x)S(x)S)^T hold).
 * - Device pointers are owned by the caller; the library never frees them.
 *   All device work is stream-ordered on the given HIP stream (hipStream_t
 *   passed as void*, NULL = default stream) and asynchronous unless stated.
 * - Every entry point returns an int status.  No C++ exception or abort
 *   crosses the ABI.  semcond_last_error() describes the last failure.
 * - A context may be used by one host thread at a time.
 */
#ifndef SEMCOND_H
#define SEMCOND_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define SEMCOND_OK          0   /* success                                         */
#define SEMCOND_ENOTCONV    1   /* solve hit max_iter; best iterate returned       */
#define SEMCOND_EINVAL     -1   /* invalid argument                                */
#define SEMCOND_ENOMEM     -2   /* device or host allocation failed                */
#define SEMCOND_EDEVICE    -3   /* HIP runtime error                               */
#define SEMCOND_EBREAKDOWN -4   /* p^T A p <= 0 in CG: operator not positive       */
#define SEMCOND_ENONFINITE -5   /* NaN or Inf met in the iteration                 */

/* Scalar type of device arrays. */
#define SEMCOND_F64 0
#define SEMCOND_F32 1

/* Basis of skeleton arrays. */
#define SEMCOND_PHYSICAL    0
#define SEMCOND_TRANSFORMED 1

/* semcond_transform directions (per skeleton entity, see conventions). */
#define SEMCOND_COEF_TO_TRANSFORMED    0  /* u~ = T^-1 u   (S^-1 = S^T M_II per axis) */
#define SEMCOND_COEF_TO_PHYSICAL       1  /* u  = T u~     (S per axis)               */
#define SEMCOND_DUAL_TO_TRANSFORMED    2  /* r~ = T^T r    (S^T per axis)             */
#define SEMCOND_DUAL_TO_PHYSICAL       3  /* r  = T^-T r~  (M_II S per axis)          */

/* Solver precision modes. */
#define SEMCOND_PREC_F64      0   /* FP64 operator and CG                          */
#define SEMCOND_PREC_F32      1   /* FP32 operator and CG vectors, FP64 dots       */
#define SEMCOND_PREC_MIXED_IR 2   /* FP32 inner CG, FP64 iterative refinement      */

typedef struct semcond_ctx semcond_ctx;

/*
 * Mesh and problem (Sec. 3: element widths h_{e,1..3}, degree p, lambda; the
 * metric coefficients d_e = (h1 h2 h3/8)(lambda, 4/h1^2, 4/h2^2, 4/h3^2),
 * eq. metriccoeffelement).  All pointers are HOST pointers, copied at create.
 *   p               2 <= p <= 32
 *   n[3]            elements per axis, each >= 1, n1*n2*n3 <= 2^26
 *   widths[a]       n[a] positive finite widths along axis a
 *   lambda          Helmholtz parameter >= 0 (used when lambda_e is NULL)
 *   lambda_e        optional per-element lambda (n_e entries, >= 0), or NULL
 *   dcoef_e         optional per-element metric override d_e (n_e x 4, row
 *                   per element, entries 1..3 > 0, entry 0 >= 0), or NULL;
 *                   when given it replaces widths/lambda in the operator (the
 *                   RHS mass matrix still uses the widths); when lambda_e is
 *                   given too, d_{e,0} = J_e lambda_e and column 0 is ignored
 *   dirichlet_mask  bit 0: x1-low face, 1: x1-high, 2: x2-low, 3: x2-high,
 *                   4: x3-low, 5: x3-high.  Set bits carry homogeneous
 *                   Dirichlet conditions, clear bits natural ones.  With
 *                   lambda = 0 at least one bit must be set.
 */
typedef struct {
    int p;
    int n[3];
    const double* widths[3];
    double lambda;
    const double* lambda_e;
    const double* dcoef_e;
    unsigned dirichlet_mask;
} semcond_mesh;

/* Options of semcond_solve.  semcond_solve_opts_default() fills defaults. */
typedef struct {
    double tol;             /* stop at ||r~||_2 <= tol*||F^~||_2 (Sec. 8), default 1e-10  */
    int max_iter;           /* CG iterations per RHS (inner for MIXED_IR), default 20000  */
    int precision;          /* SEMCOND_PREC_*, default F64                                */
    int check_every;        /* host polls convergence every this many iterations, def. 8  */
    int recover_interior;   /* 1: also write interior nodes of u_nodal (Alg. 4), def. 1   */
    const void* x0;         /* optional initial guess, TRANSFORMED skeleton [N_s][k] FP64 */
    void* skel_out;         /* optional out: TRANSFORMED skeleton solution [N_s][k] FP64  */
    double inner_tol;       /* MIXED_IR: relative tolerance of each FP32 inner solve,     */
                            /*   default 3e-3 (see ir_restart)                            */
    int max_outer;          /* MIXED_IR: refinement steps, default 30                     */
    int rhs_dual;           /* 0: f are nodal values, F = M_G f (default); 1: f is the   */
                            /* assembled discrete right-hand side itself (R F_L), as in  */
                            /* an adjoint solve H_G a = dL/du                             */
    int persistent;         /* how every CG (inner CG for MIXED_IR) is launched:          */
                            /* SEMCOND_CG_STEPWISE: one launch per step, host polls       */
                            /*   convergence every check_every iterations;               */
                            /* SEMCOND_CG_PERSISTENT: one persistent cooperative launch   */
                            /*   (autotuned grid, else the largest co-resident one);     */
                            /* SEMCOND_CG_AUTO (default): what semcond_autotune chose for */
                            /*   (k, type), else stepwise.  Persistent kernels exist for  */
                            /*   n_I <= 15 and k dividing the workgroup (k <= 32); other  */
                            /*   cases run stepwise                                       */
    const void* g_dirichlet;/* optional, nodal [k][N] FP64: prescribed values u = g on the */
                            /* nodes of the Dirichlet domain faces (other entries are     */
                            /* ignored); NULL: homogeneous.  The known values are moved  */
                            /* to the right-hand side (lifting; Sec. 8's solver test has */
                            /* inhomogeneous Dirichlet conditions).  x0 holds unknowns   */
                            /* only; skel_out returns the full skeleton values           */
    int ir_restart;         /* MIXED_IR: 0 (default): the FP32 CG keeps its search        */
                            /*   direction across refinement steps and only its residual */
                            /*   is replaced by the FP64 one (a reliable update), unless */
                            /*   a step failed to halve the worst residual; 1: every     */
                            /*   inner solve restarts from p = 0.  Either way a step's   */
                            /*   inner tolerance is inner_tol, or looser when a smaller  */
                            /*   reduction (with a factor 4 margin) reaches tol, and     */
                            /*   never below the FP32 operator's rounding level          */
                            /*   (16 K_00 2^-24, K_00 the 1D stiffness corner entry);    */
                            /*   an inner solve whose residual norm has not halved for   */
                            /*   64 iterations ends its refinement step                  */
    int deterministic;      /* 1: bit-reproducible solve (Sec. 3 assembly R in a fixed    */
                            /*   order): the element rows of edges and vertices (and in  */
                            /*   the applies outside the CG also of faces) go to per-side */
                            /*   slots summed in slot order, never through atomics; the  */
                            /*   CG runs with separate reduction launches and one launch */
                            /*   per step.  Two solves of the same input on one device   */
                            /*   then return the same bits.  Default 0 (atomics: results */
                            /*   may differ in the last bits between runs)               */
    int coarse;             /* 1: two-level preconditioner, the BT diagonal (Sec. 8) plus */
                            /*   a coarse correction P A_0^-1 P^T on the trilinear        */
                            /*   functions of the element mesh (values at the free        */
                            /*   element vertices; A_0 the trilinear element matrices     */
                            /*   with the element metrics, Cholesky-factored once per     */
                            /*   context and metric), the two-level direction of the      */
                            /*   multigrid outlook of Sec. 9: iteration counts no longer  */
                            /*   grow with the element count.  One launch per CG step;    */
                            /*   EINVAL above 32768 free vertices.  Default 0 (the paper's */
                            /*   BT preconditioner)                                        */
} semcond_solve_opts;

#define SEMCOND_CG_STEPWISE   0
#define SEMCOND_CG_PERSISTENT 1
#define SEMCOND_CG_AUTO       (-1)

/* Per right-hand-side result of semcond_solve (host array of k entries). */
typedef struct {
    int iters;              /* CG iterations (summed over refinement steps)   */
    int outer;              /* refinement steps (MIXED_IR), else 0            */
    double rel_res;         /* final ||r~||_2 / ||F^~||_2 in FP64             */
    int status;             /* SEMCOND_OK / ENOTCONV / EBREAKDOWN / ENONFINITE */
} semcond_solve_info;

/* Library version string (static storage). */
const char* semcond_version(void);

/* Message of the last failure on ctx (or of the last failed create when ctx
 * is NULL).  Valid until the next call on the same context. */
const char* semcond_last_error(const semcond_ctx* ctx);

/*
 * Host-only 1D tables of degree p (no device needed).  Any output pointer may
 * be NULL.  Arrays are row-major.
 *   x[p+1], w[p+1]     GLL nodes and weights (Sec. 3)
 *   K[(p+1)^2]         stiffness matrix K_ij = int phi_i' phi_j' (Sec. 3)
 *   S[(p-1)^2]         generalized eigenvectors, column m = eigenvector m,
 *                      S^T M_II S = I, S^T K_II S = Lambda (Sec. 5)
 *   lam[p-1]           eigenvalues Lambda in ascending order
 * Returns EINVAL unless 2 <= p <= 32.
 */
int semcond_host_tables(int p, double* x, double* w, double* K, double* S, double* lam);

/*
 * Create a context: validates the mesh, builds the 1D tables on the host,
 * uploads tables, metric data and the preconditioner diagonal (Sec. 8: exact
 * inverse of each face/edge/vertex self-block, diagonal in the transformed
 * basis) to the current HIP device.  stream: where set-up work is queued; the
 * call synchronises it before returning.  *out receives the context.
 * Errors: EINVAL (bad mesh), ENOMEM, EDEVICE.
 */
int semcond_create(const semcond_mesh* mesh, void* stream, semcond_ctx** out);

/* Release a context and its device memory (synchronises the device). */
int semcond_destroy(semcond_ctx* ctx);

/*
 * Deterministic assembly for every later semcond_apply, semcond_condense_rhs
 * and semcond_solve on ctx (on != 0), or atomics where they measured faster
 * (on = 0, the default).  The assembly R of Sec. 3 sums each shared skeleton
 * node's element rows (two per face node, four per edge node, eight per
 * vertex); deterministic mode stores every row into a per-side slot and sums
 * the slots in a fixed order, so that results do not depend on scheduling.
 * The slot workspace holds about 3 N_s k values; calls whose slot workspace
 * would reach 2^31 values fail with EINVAL.  A solve is deterministic when
 * this flag or its opts->deterministic is set.
 */
int semcond_set_deterministic(semcond_ctx* ctx, int on);

/* Sizes: total nodes N, skeleton nodes N_s (layout length), free (unconstrained)
 * skeleton nodes, elements.  Any pointer may be NULL. */
int semcond_sizes(const semcond_ctx* ctx, int64_t* N, int64_t* N_s, int64_t* N_free,
                  int64_t* n_e);

/* Host array ijk[N_s*3] receives (I1,I2,I3) of every skeleton slot, and the
 * optional host array free_mask[N_s] receives 1 for unconstrained slots. */
int semcond_skeleton_coords(const semcond_ctx* ctx, int32_t* ijk, uint8_t* free_mask);

/*
 * Condensed operator apply  v = R H^_L R^T u  on the skeleton (Sec. 4), via the
 * tensor-product factorisation in the transformed basis (Sec. 6, Table 2,
 * Algorithm 3 in transformed form): primary part from the transformed 1D
 * matrices, face -> inner eigenspace, diagonal scaling D^-1, eigenspace -> face.
 *   u, v   device [N_s][k], scalar type dtype (SEMCOND_F64 or SEMCOND_F32),
 *          u and v must not overlap
 *   basis  SEMCOND_TRANSFORMED: u, v in the transformed basis (the operator
 *          T^T H^ T).  SEMCOND_PHYSICAL: u, v nodal (the operator H^ itself;
 *          the library transforms in and out using its workspace).
 * Constrained slots of u are ignored; those of v are written 0.
 */
int semcond_apply(semcond_ctx* ctx, const void* u, void* v, int k, int dtype, int basis,
                  void* stream);

/*
 * semcond_apply without any allocation at call time, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, layouts and results as
 * semcond_apply; its workspace (the basis change and RHS-major copies of the
 * physical-basis and k > 1 forms) is a fixed 32 MiB device array of the
 * library, one per GPU, held until the process ends.
 *   Limit: 2 N_s k values of scalar type dtype must fit 32 MiB (FP64: N_s k
 *          <= 2 Mi; FP32: 4 Mi); larger calls fail with EINVAL, as does a
 *          context in deterministic mode (its slot workspace would need an
 *          allocation).  Launches are not recorded by semcond_profile_enable.
 *   Every call on one GPU shares that GPU's array: calls that overlap in time
 *   on one GPU (other streams, other contexts, other threads) race and must
 *   be ordered by the caller.  The array keeps the last call's contents; the
 *   call overwrites every part of it that it reads.
 * Stream-ordered.  Errors: EINVAL, EDEVICE.
 */
int semcond_apply_noalloc(semcond_ctx* ctx, const void* u, void* v, int k, int dtype, int basis,
                          void* stream);

/*
 * The two other evaluations of the condensed operator compared in Sec. 7
 * (Fig. 4, operation-count table), for measurement and cross-checks; both
 * give the same operator as semcond_apply in the physical basis, FP64.
 *   SEMCOND_VARIANT_TPC: Algorithm 3 in the physical basis with the
 *     tensor-product suboperators of Table 1 (primary part from the 1D
 *     matrices; condensed part through the inner eigenspace with S^T M_II
 *     face transforms), about 12 n_I^3 + 37 n_I^3 multiplications per element.
 *   SEMCOND_VARIANT_MMC: Algorithm 2 with the primary part included: one
 *     precomputed dense element matrix (the Schur complement on all n_B
 *     boundary nodes) per class of elements with equal metric, applied by one
 *     DGEMM per class (rocBLAS), 2 n_B^2 flops per element.
 * semcond_variant_setup does the precomputation (MMC: the class matrices,
 * n_classes n_B^2 doubles of device memory, EINVAL above 16 GiB; TPC:
 * nothing) and must precede semcond_apply_variant for MMC; it synchronises
 * the stream.  semcond_apply_variant: u, v device [N_s][k] FP64 in the
 * physical basis, must not overlap; constrained slots of u are ignored and
 * those of v written 0.  Stream-ordered.  Errors: EINVAL, ENOMEM, EDEVICE.
 */
#define SEMCOND_VARIANT_TPC 1
#define SEMCOND_VARIANT_MMC 2
int semcond_variant_setup(semcond_ctx* ctx, int variant, void* stream);
int semcond_apply_variant(semcond_ctx* ctx, const void* u, void* v, int k, int variant, void* stream);

/* Basis change of skeleton arrays (direction: SEMCOND_COEF_TO_TRANSFORMED, ...).
 * in, out: device [N_s][k] of dtype, must not overlap. */
int semcond_transform(semcond_ctx* ctx, const void* in, void* out, int k, int dtype,
                      int direction, void* stream);

/* Diagonal of the transformed condensed operator restricted to free slots,
 * diag(R H~^_L R^T) (Sec. 8: the BT preconditioner), device [N_s] of dtype;
 * constrained slots receive 0. */
int semcond_precond_diag(semcond_ctx* ctx, void* diag, int dtype, void* stream);

/*
 * Condensed right-hand side in the transformed basis (Algorithm 4, first loop):
 * F_e = J_e (W(x)W(x)W) f_e (GLL-lumped mass, J_e = h1 h2 h3/8), F~_e = T^T F_e,
 * F^~ = R (F~_B - H~_BI H~_II^-1 F~_I).
 *   f_nodal  device [k][N] FP64, nodal right-hand sides
 *   fhat     device [N_s][k] of dtype, TRANSFORMED basis
 */
int semcond_condense_rhs(semcond_ctx* ctx, const void* f_nodal, void* fhat, int k, int dtype,
                         void* stream);

/* Copy skeleton values into a nodal array (skeleton nodes only; other entries
 * of nodal untouched), or gather them from a nodal array.  FP64.
 *   skel device [N_s][k], nodal device [k][N]. */
int semcond_skeleton_to_nodal(semcond_ctx* ctx, const void* skel, void* nodal, int k,
                              void* stream);
int semcond_nodal_to_skeleton(semcond_ctx* ctx, const void* nodal, void* skel, int k,
                              void* stream);

/* Fill *opts with the defaults documented in semcond_solve_opts. */
void semcond_solve_opts_default(semcond_solve_opts* opts);

/*
 * Solve lambda*u - Laplace(u) = f for k right-hand sides (Algorithm 4 with the
 * BT conjugate-gradient solver of Sec. 8, x0 = 0 unless opts->x0).
 *   f_nodal  device [k][N] FP64
 *   u_nodal  device [k][N] FP64; skeleton nodes always written (physical
 *            basis), interior nodes too when opts->recover_interior
 *   opts     host, NULL = defaults
 *   info     host array of k entries, may be NULL
 * Synchronises the stream before returning.  Returns OK when every RHS
 * converged, ENOTCONV when some hit max_iter (their best iterate is returned),
 * EBREAKDOWN / ENONFINITE on numerical failure.
 */
int semcond_solve(semcond_ctx* ctx, const void* f_nodal, void* u_nodal, int k,
                  const semcond_solve_opts* opts, semcond_solve_info* info, void* stream);

/*
 * Interior recovery (Algorithm 4, second loop) from a skeleton solution:
 * skeleton nodes u = T u~ (Sec. 6 basis change), interior nodes
 * u_I = (S(x)S(x)S) D^-1 (F~_I - H~_IB u~_B) per element (Sec. 4, Sec. 5).
 *   f_nodal  device [k][N] FP64, the nodal right-hand sides of the solve
 *   u_skel   device [N_s][k] FP64, TRANSFORMED skeleton values including those
 *            of the Dirichlet entities (zero for homogeneous conditions), e.g.
 *            the skel_out of semcond_solve
 *   u_nodal  device [k][N] FP64, every node written
 *   dtype    SEMCOND_F64 (only)
 * Stream-ordered.  Errors: EINVAL, ENOMEM, EDEVICE.
 */
int semcond_recover_interior(semcond_ctx* ctx, const void* f_nodal, const void* u_skel, void* u_nodal,
                             int k, int dtype, void* stream);

/*
 * Pre-size the context's device workspace and the host side of its
 * convergence polls for applies, transforms, solves (any launch kind, with
 * prescribed Dirichlet values or dual right-hand sides) and interior recovery
 * of up to k_max right-hand sides; dtype SEMCOND_F64 covers FP64 solves,
 * SEMCOND_F32 also FP32 and MIXED_IR ones.  Later calls with k <= k_max then
 * allocate nothing (profiling, autotuning and semcond_update_coefficients
 * adding per-element tables excepted).  Synchronises the device.
 * Errors: EINVAL (k_max, dtype), ENOMEM, EDEVICE.
 */
int semcond_reserve(semcond_ctx* ctx, int k_max, int dtype);

/*
 * Replace the Helmholtz parameter / metric coefficients of an existing context
 * (Sec. 3: d_e = (h1 h2 h3/8)(lambda, 4/h1^2, 4/h2^2, 4/h3^2); Sec. 8 notes that
 * lambda changes between time steps) and rebuild the preconditioner.  Same
 * meaning and validation as the semcond_mesh fields (host pointers, copied;
 * lambda_e and dcoef_e may be NULL).  Widths and the RHS mass are unchanged.
 * Synchronises the stream.
 */
int semcond_update_coefficients(semcond_ctx* ctx, double lambda, const double* lambda_e,
                                const double* dcoef_e, void* stream);

/* Assembled GLL-lumped mass M_G = R (J_e W(x)W(x)W) R^T as a nodal array
 * (Sec. 3; J_e = h1 h2 h3 / 8).  mass: device [N] FP64. */
int semcond_nodal_mass(semcond_ctx* ctx, void* mass, void* stream);

/* out = M_G (x) in, or in / M_G when inverse != 0, for nodal [k][N] FP64
 * arrays (the assembled GLL-lumped mass of Sec. 3; dL/df = M_G a in the
 * adjoint method).  in and out may coincide. */
int semcond_mass_apply(semcond_ctx* ctx, const void* in, void* out, int k, int inverse, void* stream);

/*
 * Element gradients for the adjoint method: with u the solution of the full
 * discrete system H_G u = M_G f and a the adjoint (H_G a = dL/du), the
 * derivative of L with respect to the metric coefficient d_{e,m} (Sec. 3, eq.
 * helmholtz_operator, H_e = sum_m d_{e,m} A_m) is -a_e^T A_m u_e.
 *   u_nodal, a_nodal  device [k][N] FP64, full nodal vectors (interior included)
 *   grad              device [n_e][5] FP64, summed over the k right-hand sides:
 *                     columns 0..3 dL/dd_{e,0..3}, column 4 dL/dlambda_e =
 *                     J_e dL/dd_{e,0} (d_{e,0} = J_e lambda_e)
 */
int semcond_element_grads(semcond_ctx* ctx, const void* u_nodal, const void* a_nodal, void* grad,
                          int k, void* stream);

/*
 * The same element terms per right-hand side: grad[e][m][r] = -a_{e,r}^T A_m
 * u_{e,r} (Sec. 3, eq. helmholtz_operator), m = 0..3, for the adjoint pairs
 * (u_r, a_r) of k right-hand sides, i.e. dL_r/dd_{e,m} of per-RHS losses
 * L_r (their sum over r is semcond_element_grads' columns 0..3; dL_r/dlambda_e
 * = J_e grad[e][0][r]).
 *   u_nodal, a_nodal  device [k][N] FP64
 *   grad              device [n_e][4][k] FP64, every entry written
 * Stream-ordered.  Errors: EINVAL.
 */
int semcond_element_grads_rhs(semcond_ctx* ctx, const void* u_nodal, const void* a_nodal, void* grad,
                              int k, void* stream);

/*
 * Right-hand sides per workgroup of the batched right-hand-side condensation
 * and interior recovery kernels (Algorithm 4, first and second loops; used for
 * 8 <= p - 1 <= 12 and N < 2^32).  A workgroup takes one element and R
 * right-hand sides, setting up the element's tables, addresses and D^-1 once.
 * R > 0 fixes the batch for every k (capped at k) and R = -1 selects the
 * per-item kernels (one workgroup per element and right-hand side); R = 0, the
 * default, lets the library time the per-item kernels and R = 1, 2, 4, 8, 16
 * (up to k) on the first condensation and the first recovery of each k of this
 * context (synchronising the stream there) and keep the fastest.  Every
 * batched R gives bitwise the same recovery, and the same condensation up to
 * the order of its atomic additions (bitwise the same in deterministic mode);
 * the per-item kernels differ from them by rounding.  Errors: EINVAL for R
 * outside [-1, 256].
 */
int semcond_set_rhs_batch(semcond_ctx* ctx, int R);

/*
 * The batch sizes in use for k right-hand sides: R_condense, R_recover
 * (nullable) receive R, 0 for the per-item kernels, -1 while not yet timed.
 * Errors: EINVAL for k outside [1, 256].
 */
int semcond_get_rhs_batch(const semcond_ctx* ctx, int k, int* R_condense, int* R_recover);

/*
 * Autotuner of the CG launch (k right-hand sides of scalar type dtype): times
 * one launch per step and the candidate persistent grids (workgroup count G,
 * element groups per workgroup S) for a few CG iterations on this context's
 * problem and keeps the fastest for later SEMCOND_CG_AUTO solves; (S, G) =
 * (0, 0) denotes one launch per step.  When cache_path is non-NULL the choice
 * is read from / appended to that text file (one line "p n1 n2 n3 k dtype S G").
 * S_out, G_out (nullable) receive the choice.  Returns EINVAL when no
 * persistent kernel exists for (p, k).  Synchronises the device.
 */
int semcond_autotune(semcond_ctx* ctx, int k, int dtype, const char* cache_path, int* S_out, int* G_out);

/*
 * Kernel tracing.  While enabled, every launch of the condensed-apply kernel
 * (inside semcond_apply and the stepwise CG; SEMCOND_KERNEL_APPLY for FP64
 * operands, SEMCOND_KERNEL_APPLY_F32 for FP32) and of the persistent CG
 * kernel (SEMCOND_KERNEL_PCG) is bracketed by two HIP events
 * recorded on the launch stream.  semcond_profile_enable resets the counters;
 * semcond_profile_read synchronises the recorded events and returns the summed
 * kernel time in milliseconds and the number of launches of `kernel` since the
 * reset, and for SEMCOND_KERNEL_PCG the CG iterations those launches ran
 * (summed over right-hand sides' maximum per launch) in *iters (nullable).
 */
#define SEMCOND_KERNEL_APPLY 0
#define SEMCOND_KERNEL_PCG   1
#define SEMCOND_KERNEL_APPLY_F32 2
int semcond_profile_enable(semcond_ctx* ctx, int enable);
int semcond_profile_read(semcond_ctx* ctx, int kernel, double* ms, int64_t* launches, int64_t* iters);

#ifdef __cplusplus
}
#endif

#endif /* SEMCOND_H */
