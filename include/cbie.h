/*
 * cbie.h -- C-ABI of the MI355X (gfx950) H-matrix direct solver for the
 * Chebyshev-based Nystrom boundary integral equation (CBIE), after
 * Hu, Sever, Babazadeh, Jeffrey, Okhmatovski, Sideris, "H-Matrix Accelerated
 * Direct Matrix Solver for Maxwell's Equations using the Chebyshev-based
 * Nystrom Boundary Integral Equation Method" (arXiv 2408.17116).
 *
 * Problem (Sec. II).  A closed PEC surface is cut into curved quadrilateral
 * patches; on each patch the contravariant components F^u, F^v of the
 * surface current (eq. 11) are sampled on a q x q grid of first-kind
 * Chebyshev (Fejer) points (eqs. 12, 13).  The MFIE (eq. 10, second row,
 * with the sign fixed by eqs. 2, 5, 6:  J/2 - n x curl S[J] = n x H_inc),
 * tested with sqrt(G) a^u, sqrt(G) a^v (eqs. 17, 18), gives the dense complex
 * system of eq. (22).  Far entries use the plain Fejer rule; self and near
 * entries (eq. 20) are integrals against the Chebyshev basis computed with a
 * singularity-cancelling change of variables.  The matrix is held as an
 * H-matrix (Sec. III: cluster tree, admissibility eq. 21, leaf size n_leaf,
 * ACA for admissible blocks), factorized by H-LU and solved by forward/back
 * substitution (eqs. 23-28), in the "entire matrix" ordering with
 * interleaved u/v unknowns at repeated points (Sec. III-B).
 *
 * Conventions
 *  - Units are normalized: eps0 = mu0 = 1, eta0 = 1, omega = k0.  Time
 *    dependence e^{j omega t}.  The mu_1 row factor of eq. (22) is dropped.
 *  - Vectors crossing the ABI are complex128 (two doubles, re then im),
 *    column-major with leading dimension ld >= n_unknowns, device pointers
 *    on the context's device, in the ORIGINAL unknown order: object-major,
 *    then patch p, node (k, l) with l the u-index, then component (u, v):
 *    index = 2 * ((p * q + k) * q + l) + a within an object.
 *  - Every call is ordered on the context stream and returns after the
 *    work has completed, so the status reflects device errors.  Nothing is
 *    printed, thrown or aborted across the ABI; a failing call leaves the
 *    context valid and sets cbie_last_error().
 *  - Ownership: the caller owns every buffer it passes; the library never
 *    frees them and never keeps them after the call returns.  The library
 *    owns everything it allocates and frees it in cbie_destroy().
 *  - State machine: create -> build_tree -> fill -> compress -> factor ->
 *    solve.  matvec is valid after compress.  factor may be repeated with
 *    another precision.  Calls out of order return CBIE_ESTATE.  A stage
 *    call (build_tree, fill, compress, factor) that fails after its argument
 *    checks leaves the context in the state that precedes the stage, so the
 *    stage and every later one must be run again before their results are
 *    used.
 */
#ifndef CBIE_H
#define CBIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CBIE_OK = 0,
    CBIE_EINVAL = -1,     /* bad argument (null pointer, size, range)      */
    CBIE_ENOMEM = -2,     /* device or host allocation failed              */
    CBIE_EHIP = -3,       /* a HIP runtime call or kernel failed           */
    CBIE_ESTATE = -4,     /* call out of order                             */
    CBIE_ENOCONV = -5,    /* iterative refinement did not reach tolerance  */
    CBIE_ESINGULAR = -6,  /* zero pivot in a diagonal leaf                 */
    CBIE_EINTERNAL = -7   /* unsupported internal case (reported, no UB)   */
} cbie_status;

typedef struct cbie_ctx cbie_ctx;

typedef enum { CBIE_MFIE_PEC = 0, CBIE_NMULLER = 1 } cbie_formulation;
typedef enum { CBIE_PREC_C128 = 0, CBIE_PREC_C64_IR = 1 } cbie_precision;
typedef enum { CBIE_RANK_ADAPTIVE = 0, CBIE_RANK_PREDICTED = 1 } cbie_rank_mode;
typedef enum { CBIE_ORDER_ENTIRE = 0, CBIE_ORDER_COMPONENT = 1 } cbie_ordering;

/* One patch of the equiangular cube sphere mapped onto an ellipsoid:
 * face f (0..5 = +x,-x,+y,-y,+z,-z), sub-square (i, j) of split x split,
 * r(u,v) = center + diag(axes) c/|c|, c = e_n + tan(pi xi/4) e_1 +
 * tan(pi eta/4) e_2, xi = (2i+1+u)/split - 1, eta = (2j+1+v)/split - 1.  */
typedef struct {
    int face, i, j, split;
} cbie_patch;

typedef struct {
    cbie_formulation form;     /* CBIE_MFIE_PEC (perfect conductor, 2 unknowns
                                  per node) or CBIE_NMULLER (homogeneous
                                  dielectric, 4 unknowns per node); every
                                  object of a context has the same form   */
    double k0;                 /* exterior wavenumber, rad/m, > 0           */
    double axes[3];            /* ellipsoid semi-axes, > 0                   */
    double center[3];
    int q;                     /* Chebyshev points per direction: 2..11 for
                                  CBIE_MFIE_PEC (2 q^2 <= 256, one patch per
                                  leaf at most), 2..8 for CBIE_NMULLER       */
    int n_patches;
    const cbie_patch* patches; /* host array of n_patches, copied at create  */
    double eps_r, mu_r;        /* N-Mueller: interior relative permittivity and
                                  permeability (real, > 0; the exterior is
                                  vacuum); ignored for CBIE_MFIE_PEC        */
    /* Chebyshev-interpolated patches (generic surfaces, the form a CAD
     * surface is handed over in; eqs. 11-14 on patches of any shape):
     * patch_degree d in 1..16 and patch_coeffs, a host array of
     * n_patches x 3 x (d+1) x (d+1) doubles, coefficient [p][c][n][m]
     * multiplying T_n(u) T_m(v) in coordinate c of patch p's r(u, v) on
     * [-1, 1]^2, with a_u x a_v pointing outward; copied at create.  Then
     * patches, axes and center are ignored (patches may be NULL).
     * patch_degree 0: the cube-sphere patches above.                      */
    int patch_degree;
    const double* patch_coeffs;
} cbie_object;

/* Create a context for n_objs independent objects (block-diagonal system,
 * no coupling between objects).  hip_stream: a hipStream_t, or NULL for
 * the null stream.  Copies the patch tables.  Errors: EINVAL, ENOMEM, EHIP. */
cbie_status cbie_create(const cbie_object* objs, int n_objs, void* hip_stream,
                        cbie_ctx** out);

/* Geometry of the nodes (eqs. 11, 14, 17, 18), near classification (eq. 20:
 * patch p is near node i iff dist(r_i, p) < near_delta * diam(p), diam =
 * longer corner diagonal, dist by projection; the owner patch is "self"),
 * cluster tree by patch-atomic bisection of node bounding boxes until a
 * cluster holds <= leaf_size unknowns or one patch, and block cluster tree
 * with admissibility min(diam_t, diam_s) <= eta dist(t, s) on bounding
 * boxes (eq. 21); a block holding a near pair is never admissible.
 * Errors: EINVAL (leaf_size below the unknowns of one patch, upn q^2 with
 * upn = 2 (MFIE) or 4 (N-Mueller), or above 256; eta <= 0, near_delta <= 0),
 * ENOMEM, EHIP. */
cbie_status cbie_build_tree(cbie_ctx* ctx, int leaf_size, double eta, double near_delta);

/* Fill the inadmissible (dense) blocks: far entries by the Fejer rule,
 * self/near entries by the change-of-variables quadrature, plus the identity
 * term (1/2 for the MFIE; (mu1 + mu2)/2 and -(eps1 + eps2)/2 for N-Mueller).
 * n_ang / n_rad: points of the singular rule per angular / radial direction
 * (0 = defaults: 40 / 32 up to q = 8, max(40, 6 q - 8) / max(32, 5 q - 8)
 * for the largest order q of the context).  Errors: ESTATE, ENOMEM, EHIP. */
cbie_status cbie_fill(cbie_ctx* ctx, int n_ang, int n_rad);

/* Compress the admissible blocks by partial-pivot ACA (Sec. III-A) to the
 * relative Frobenius tolerance aca_tol; each block keeps its ACA factors
 * U (m x r) and V (n x r) at the rank where ACA stopped (at most 512).
 * mode CBIE_RANK_ADAPTIVE sizes each block's workspace at full width,
 * CBIE_RANK_PREDICTED at the width the rank model predicts (see
 * cbie_set_rank_model); both give the same factors.  Blocks are processed in
 * rounds whose ACA workspace fits a quarter of the device memory free when
 * the call starts, at most 2^32 complex elements (environment variable
 * CBIE_ACA_BUDGET: another element count), so the workspace stays bounded at
 * any problem size; N-Mueller blocks compressed from explicit copies keep
 * those within an eighth of the free memory, at most 2^31 entries
 * (CBIE_ACA_DENSE).  Errors: ESTATE, EINVAL (aca_tol outside (0, 1),
 * CBIE_RANK_PREDICTED without a model), ENOMEM, EHIP. */
cbie_status cbie_compress(cbie_ctx* ctx, double aca_tol, cbie_rank_mode mode);

/* H-LU factorization (eqs. 23-28): partial pivoting inside diagonal leaves,
 * none across blocks; formatted updates truncated at the compress tolerance
 * (or the tolerance set by cbie_set_factor_tolerance) in the relative
 * Frobenius norm of each block, with the range basis of every truncation
 * built in FP64 in both precisions; a complex64 factor is truncated at no
 * less than 1e-5 (closer to its rounding noise, the noise would be kept as
 * rank).
 * CBIE_PREC_C128: complex128 on FP64 MFMA.  CBIE_PREC_C64_IR: complex64 on
 * FP32 MFMA (FP32 accumulation); solve() then refines in FP64.
 * Errors: ESTATE, ENOMEM, EHIP, ESINGULAR. */
cbie_status cbie_factor(cbie_ctx* ctx, cbie_precision prec);

/* Truncation tolerance of the formatted sums of later factorizations
 * (an addition to the paper, which truncates at the ACA tolerance): tol in
 * (0, 1), or 0 for the compress tolerance (the default).  A looser factor
 * is a cheaper preconditioner; the refinement of cbie_solve or
 * cbie_solve_gmres still converges to the stored FP64 operator's solution
 * while it contracts.  Errors: EINVAL. */
cbie_status cbie_set_factor_tolerance(cbie_ctx* ctx, double tol);

/* Ordering of the unknowns for later factorizations (Sec. III, Fig. 3).
 * CBIE_ORDER_ENTIRE (the default, Sec. III-B): one cluster tree over the
 * nodes, every block holding all components of its nodes interleaved.
 * CBIE_ORDER_COMPONENT (Sec. III-A, eqs. 22-28): per object, the unknowns
 * ordered component by component and one H-matrix per component
 * interaction block (MFIE: uu, uv, vu, vv; N-Mueller: the 16 of eq. 19),
 * factored as the 2 x 2 block LU of eq. 23 (N-Mueller: nested twice) with
 * the substitutions of eqs. 26-28.  The component blocks are taken from
 * the compressed operator: dense leaves as strided copies, low-rank blocks
 * as the matching rows of U and V, truncated at the factorization's
 * truncation tolerance (t_factor_reorder in cbie_stats, part of t_factor).  Leaves hold a
 * single component, so diagonal leaves are leaf_size / unknowns-per-node
 * unknowns.  cbie_solve and cbie_solve_gmres take and return the original
 * order either way.  Errors: EINVAL. */
cbie_status cbie_set_factor_ordering(cbie_ctx* ctx, cbie_ordering ordering);

/* Solve A x = b for nrhs right-hand sides (per object).  b_dev, x_dev:
 * complex128 device arrays, n_unknowns x nrhs, leading dimension ld,
 * original order; b_dev is not modified; x_dev may not alias b_dev.
 * x = LU^{-1} b; then, for ir_maxit > 0, iterate r = b - A x (FP64, stored
 * operator), x += LU^{-1} r.  The residual is checked before every sweep and
 * after the last one: the call succeeds once max_j ||r_j|| / ||b_j|| <= ir_tol
 * (2-norms per right-hand side j) and returns ENOCONV after ir_maxit sweeps
 * without it, or at once when a residual is not finite (x then holds the
 * last iterate).  ir_maxit = 0 returns the plain substitution with no
 * residual check.  ir_iters_out (may be NULL) receives the sweep count.
 * The substitution program (eqs. 26-28) is recorded once per factorization
 * and number of right-hand sides, captured into a HIP graph on a private
 * stream, and replayed for every later substitution (the refinement sweeps
 * and later solves); the context stream waits on the replay through events.
 * Errors: ESTATE, EINVAL, ENOCONV, EHIP. */
cbie_status cbie_solve(cbie_ctx* ctx, int nrhs, const void* b_dev, void* x_dev, long ld,
                       double ir_tol, int ir_maxit, int* ir_iters_out);

/* The same system solved by GMRES-based refinement (an addition to the
 * paper's direct solve, for operators close to a resonance where the
 * stationary refinement of cbie_solve stops contracting): restarted GMRES in
 * FP64 on A M y = b, x = M y, with A the stored FP64 operator and M the
 * forward/back substitutions with the factorization (either precision) as
 * a right preconditioner, one right-hand side at a time, starting from
 * x = M b.  Each column stops when ||b - A x|| <= tol ||b|| (true residual,
 * recomputed) or after maxit Krylov steps; every cycle builds at most
 * `restart` basis vectors (device memory: restart + 2 vectors of
 * n_unknowns complex128 per cycle).  iters_out (may be NULL) receives the
 * Krylov steps summed over the columns.  Errors: ESTATE, EINVAL (restart
 * <= 0, maxit < 0, tol <= 0), ENOCONV (x holds the last iterates), EHIP. */
cbie_status cbie_solve_gmres(cbie_ctx* ctx, int nrhs, const void* b_dev, void* x_dev, long ld, double tol,
                             int restart, int maxit, int* iters_out);

/* y = A_H x with the compressed operator in FP64 arithmetic (complex128),
 * nrhs columns, original order, leading dimension ld.  Errors: ESTATE, EINVAL, EHIP. */
cbie_status cbie_matvec(cbie_ctx* ctx, int nrhs, const void* x_dev, void* y_dev, long ld);

/* The same product as cbie_matvec, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the call allocates nothing and works in a scratch array
 * that the library holds on each GPU for the life of the process, 2^23
 * complex128 elements (128 MiB).  One call needs (2 n_unknowns + sum of the
 * low-rank ranks) * nrhs elements (the ranks from compress: cbie_stats
 * sum_rank); larger calls return EINVAL and do nothing.  Every context on a
 * GPU shares that GPU's array, which keeps the last call's contents: calls
 * that overlap on one GPU (other threads, other streams) race and must be
 * serialized by the caller.  Errors: ESTATE, EINVAL, EHIP. */
cbie_status cbie_matvec_noalloc(cbie_ctx* ctx, int nrhs, const void* x_dev, void* y_dev, long ld);

/* Right-hand sides of eq. (22) for nw plane waves E = pol e^{-j k khat.r},
 * H = khat x E: b_u = -a_v . H, b_v = a_u . H per node; N-Mueller objects
 * (eq. 19, exterior vacuum) add the electric rows -a_v . E, a_u . E after
 * them.  khat, pol: host arrays of 3*nw doubles.  b_dev: complex128 device array n_unknowns x nw, ld.
 * Errors: ESTATE (before build_tree), EINVAL, EHIP. */
/* Right-hand sides for n_dipoles point electric dipoles in free space (the
 * x-polarized dipole feeding the spiral antenna of Sec. IV-A): each
 * dipole's fields replace the plane wave's in the rows of eq. (22) (and the
 * electric rows of eq. 19 for N-Mueller objects).  pos, moment: host arrays
 * of 3*n_dipoles doubles, position r0 and current moment m (I l) of each
 * dipole; in the normalized units eps = mu = 1, omega = k0, time factor
 * e^{j omega t}, with d = r - r0, R = |d|, e = d / R, G = e^{-j k0 R} / (4 pi R):
 * H = (1 + j k0 R) (G / R) m x e and
 * E = G [(-1/R + j (1/(k0 R^2) - k0)) (m - (m.e) e) + (2/R - 2j/(k0 R^2)) (m.e) e].
 * b_dev: complex128 device array n_unknowns x n_dipoles, leading dimension
 * ld, original order.  Errors: ESTATE (before build_tree), EINVAL (also
 * when a dipole sits exactly on a node), EHIP. */
cbie_status cbie_rhs_dipole(cbie_ctx* ctx, int n_dipoles, const double* pos, const double* moment, void* b_dev,
                            long ld);

cbie_status cbie_rhs_planewave(cbie_ctx* ctx, int nw, const double* khat, const double* pol,
                               void* b_dev, long ld);

/* Far field r e^{j k r} E_s = -j k (N_perp - rhat x L) / (4 pi), N = sum_nodes
 * w (F^u a_u + F^v a_v) e^{j k rhat.r} from the electric current and L the
 * same sum from the magnetic current (N-Mueller objects; L = 0 on a
 * conductor), for nrhs solutions x_dev (device,
 * ld) at ndir directions rhat (host, 3*ndir doubles).  E_out: host array of
 * 3 * ndir * nrhs complex128 (x,y,z fastest, then direction, then rhs).
 * Errors: ESTATE, EINVAL, EHIP. */
cbie_status cbie_farfield(cbie_ctx* ctx, int nrhs, const void* x_dev, long ld, int ndir,
                          const double* rhat, void* E_out);

/* Statistics.  Fills as many leading fields of cbie_stats as `bytes` allows. */
typedef struct {
    int64_t n_unknowns, n_nodes, n_patches, n_objects;
    int64_t n_clusters, n_leaves, n_dense_blocks, n_lr_blocks;
    int64_t n_near_pairs;            /* (target node, patch) pairs incl. self */
    int64_t dense_entries;           /* stored dense entries                  */
    int64_t lr_entries;              /* stored low-rank entries (m + n) r     */
    int64_t max_rank, sum_rank;
    double compression_rate;         /* 1 - stored / N^2 (Sec. IV-A)          */
    double t_tree, t_fill, t_compress, t_factor, t_solve;  /* seconds          */
    int64_t factor_flops;            /* algorithmic flops of the last factor:
                                        products 8 m n k, leaf LU 8/3 b^3, a
                                        leaf triangular solve (n x n, k
                                        columns) 4 n^2 k although it runs as a
                                        product with the explicit inverse      */
    int64_t n_kernel_launches;       /* launches in the last factor           */
    int64_t ir_iterations;           /* sweeps of the last solve              */
    double quad_seconds;             /* near/self quadrature kernel time      */
    /* batched complex GEMM (the H-LU's dense contractions) since create:
     * launches, algorithmic flops (8 m n k per product) and, with
     * profiling on, the summed kernel time from HIP events recorded around
     * each launch on the context stream (0 otherwise)                        */
    int64_t gemm_launches;
    double gemm_flops;
    double gemm_seconds;
    /* compress: admissible blocks redone with the full width because the
     * predicted width was too small; ACA workspace the widths asked for,
     * bytes, summed over every round of both passes (at any time at most
     * one round's budget is allocated) */
    int64_t aca_fallbacks;
    double aca_workspace_bytes;
    /* solve: substitutions run as a replay of the captured HIP graph of the
     * program recorded by the first solve with this factorization and this
     * number of right-hand sides (cumulative over the factorization) */
    int64_t solve_replays;
    /* compress: admissible blocks whose ACA stopped at the rank cap (512),
     * below the block's full rank min(m, n), without meeting aca_tol (last
     * compress only; a block that reached min(m, n) is reproduced exactly) */
    int64_t aca_unconverged;
    /* algorithmic flops of the batched GEMM launches since create (leaf
     * solves through explicit inverses counted as triangular solves,
     * 4 n^2 k); gemm_flops counts what the launches execute, 8 m n k */
    double gemm_flops_alg;
    /* flops the last factor executed: every product at 8 m n k and every
     * leaf at LU plus both inverses (16/3 b^3) */
    int64_t factor_flops_executed;
    /* batched leaf LU launches since create, their algorithmic flops
     * (8/3 b^3 per leaf) and, with profiling on, their summed kernel time */
    int64_t leaf_lu_launches;
    double leaf_lu_flops;
    double leaf_lu_seconds;
    /* fill: quadrature points of the near/self rule summed over the pairs,
     * and the FP64 flops of their basis contraction (per point and source
     * node 16 for the MFIE, 64 for N-Mueller; the kernel evaluations come
     * on top), done in quad_seconds */
    double quad_points;
    double quad_flops;
    /* factor: bytes one forward/back substitution reads (explicit leaf
     * inverses, off-diagonal dense blocks, low-rank factors, in the factor
     * precision) */
    double solve_factor_bytes;
    /* fill: kernel time of the far (Fejer-rule) entries of the dense blocks,
     * dense_entries complex128 values written */
    double far_fill_seconds;
    /* algorithmic bytes of the batched GEMM launches since create: per
     * product A (m k), B (k n), C read when beta != 0 and C written (m n),
     * in the factor precision */
    double gemm_bytes_alg;
    /* matrix-core flops of the batched GEMM launches since create: 8 m n k
     * per product, 6 m n k for complex64 products on 64 x 64 tiles, which
     * form the complex product from three real ones (P1 = Ar Br,
     * P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi); Cr = P1 - P2, Ci = P3 - P1 - P2;
     * CBIE_GEMM_3M=0 selects the four-product form) */
    double gemm_flops_mfma;
    /* last factor: recompressions of every pending block forced by storage
     * pressure (the factors grew by more than half the device memory free
     * when the factorization started, or by CBIE_FACTOR_MEM bytes) */
    int64_t factor_mem_flushes;
    /* last factor in CBIE_ORDER_COMPONENT: seconds spent truncating the
     * component blocks taken from the low-rank blocks (0 otherwise) */
    double t_factor_reorder;
} cbie_stats;
cbie_status cbie_get_stats(cbie_ctx* ctx, void* stats_out, size_t bytes);

/* ------------------------------------------------------------------
 * Rank predictor (an addition to the paper's method).  A fully connected
 * network 8 -> 64 -> 64 -> 1 with ReLU maps geometric features of an
 * admissible block to the natural log of its adaptive ACA rank.  Parameters
 * (CBIE_MLP_NPARAMS float32): W1 (64 x 8, row-major), b1 (64), W2 (64 x 64,
 * row-major), b2 (64), W3 (64), b3 (1).  Inputs are standardized by a
 * per-feature mean and standard deviation (8 float32 each).
 * Features of block (t, s), object wavenumber k, boxes of the node clusters:
 *   log m, log n (unknowns), k diam_t, k diam_s, k dist, max(diam)/dist,
 *   log10(ACA tol), k diam_t diam_s / dist  (diam: box diagonal, dist: box gap)
 * ------------------------------------------------------------------ */
#define CBIE_MLP_NFEAT 8
#define CBIE_MLP_NPARAMS 4801

/* After build_tree: features of every admissible block (host, count x 8
 * float32, low-rank block order) and, after compress, their ranks (host,
 * count int32; -1 before compress).  cap: rows the arrays hold (either may
 * be NULL); count_out: number of admissible blocks.  Errors: ESTATE, EINVAL. */
cbie_status cbie_get_block_features(cbie_ctx* ctx, double aca_tol, int64_t cap, float* feat, int32_t* ranks,
                                    int64_t* count_out);

/* The model used by compress(CBIE_RANK_PREDICTED) (host arrays, copied).
 * A block's ACA then starts with width ceil(exp(y) (1 + margin)) + 2
 * (y: predicted log-rank); a block that fills it without converging is
 * redone with the full width, so the factors equal the adaptive ones.
 * Errors: EINVAL. */
cbie_status cbie_set_rank_model(cbie_ctx* ctx, const float* params, const float* mean, const float* sdev,
                                float margin);

/* Network kernels on a HIP stream; every array is device float32 (order:
 * int32).  X: n x 8 row-major raw features.
 * forward: y[i] = network((X[i] - mean) / sdev).
 * grad: loss[0] = mean_i (y_i - t_i)^2 and grad (CBIE_MLP_NPARAMS) its
 *   gradient with respect to the parameters.
 * train: Adam (beta1 0.9, beta2 0.999, eps 1e-8, rate lr) for nsteps steps,
 *   step s on samples order[s * batch .. (s + 1) * batch); params updated in
 *   place, losses[s] = that batch's loss before the step.  One work-group.
 * Errors: EINVAL (sizes), EHIP. */
cbie_status cbie_mlp_forward(void* hip_stream, const float* params, const float* mean, const float* sdev,
                             const float* X, int64_t n, float* y);
cbie_status cbie_mlp_grad(void* hip_stream, const float* params, const float* mean, const float* sdev,
                          const float* X, const float* t, int64_t n, float* grad, float* loss);
cbie_status cbie_mlp_train(void* hip_stream, float* params, const float* mean, const float* sdev, const float* X,
                           const float* t, const int32_t* order, int64_t nsteps, int batch, float lr,
                           float* losses);

/* Kernel timing: on != 0 brackets every batched GEMM launch and every
 * batched leaf LU launch of the factorization with HIP events on the context
 * stream (their sums are reported as gemm_seconds and leaf_lu_seconds).
 * Costs a little host time per launch; off by default.  Errors: EINVAL, EHIP. */
cbie_status cbie_set_profiling(cbie_ctx* ctx, int on);

/* Parity hooks (small problems; no effect on the solver state).
 * Near pairs after build_tree: for each pair, target node and patch index
 * (original numbering).  cap: capacity of the host arrays; count_out gets
 * the total (the arrays hold min(cap, total), sorted by (target, patch)).  */
cbie_status cbie_get_near_pairs(cbie_ctx* ctx, int64_t cap, int32_t* targets, int32_t* patches,
                                int64_t* count_out);
/* After fill (dense blocks) and compress (low-rank blocks): the full matrix,
 * N x N complex128, device, column-major with leading dimension ld, original
 * order.  Admissible blocks not yet compressed are filled with the plain
 * Fejer rule.  Errors: ESTATE, EINVAL, ENOMEM, EHIP. */
cbie_status cbie_export_dense(cbie_ctx* ctx, void* a_dev, long ld);

const char* cbie_last_error(const cbie_ctx* ctx);
void cbie_destroy(cbie_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* CBIE_H */
