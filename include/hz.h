/*
 * hz.h -- C-ABI of the nested polarized-traces Helmholtz solver for one AMD
 * MI355X (gfx950).
 *
 * Method: L. Zepeda-Nunez and L. Demanet, "Nested domain decomposition with
 * polarized traces for the 2D Helmholtz equation" (arXiv 1510.01831).
 *
 * Problem (Sec. 2, App. A).  -Laplace(u) - omega^2 m u = f on the unit square
 * discretised by the 5-point stencil on n interior nodes per side
 * (h = 1/(n+1)), truncated by a quadratic stretched-coordinate PML of n_pml
 * nodes per side (sigma = (C/delta)(d/delta)^2, C = pml_beta * omega * delta,
 * homogeneous Dirichlet beyond), with m = 1/c^2 extended into the PML by
 * copying the nearest physical value.  Rows are scaled by 1/(alpha_x alpha_z)
 * so the operator H is complex symmetric; inside the physical square the
 * rows are exactly the paper's stencil.  A point source is f = 1/h^2 at a node
 * (the discrete delta of Sec. 2.1).
 *
 * Method (Sec. 3-4).  The extended grid is cut into `layers` slabs in depth
 * and each slab into `cells` in x; every cell is factorised (offline), every
 * layer's Green's integrals are factorised through its cells (eq.
 * factorization + block LU of the inner SIE, Sec. 4.2.2), and the polarized
 * SIE on the layer interfaces is solved by GMRES preconditioned with the
 * Gauss-Seidel sweeps (Sec. 3.1, Alg. 6).
 *
 * Conventions for every entry point.
 *  - Arrays are row-major; a field on the physical grid is f[z][x] with z the
 *    depth index (x fastest, Sec. 2.1 ordering).  A batch of B fields is
 *    f[b][z][x], i.e. each right-hand side contiguous.
 *  - Complex data are interleaved (re, im) pairs of double, i.e. the memory
 *    layout of `double _Complex` / torch.complex128.
 *  - Pointers named *_dev are device pointers (hipMalloc'd or torch CUDA
 *    tensors); *_host are host pointers.  The caller owns every pointer it
 *    passes; the library copies what it keeps.  The context owns all device
 *    memory it allocates and frees it in hz_destroy.
 *  - All device work is enqueued on the context's stream (default: a stream
 *    of default priority that hz_setup creates, blocking with respect to the
 *    null stream; see hz_set_stream).  Every call returns only after its work has
 *    completed on that stream, unless stated otherwise.
 *  - No call throws across the ABI.  Errors are returned as hz_status; the
 *    text of the last error of the calling thread is in hz_last_error().
 *  - Environment (read by hz_setup / per launch; for experiments, results do
 *    not depend on them beyond rounding):
 *      HZ_TUNE=0     fixed kernel heuristics instead of the autotuner (which
 *                    times the GEMM kernels of every solve plan and the
 *                    cell-solve batch width once per batch size);
 *      HZ_GEMM_KIND=k  one matrix-core GEMM kernel for every solve launch
 *                    (2: 32x32 tiles, 32-deep chunks; 3: 64x64, 16-deep;
 *                    4: 32x32, 16-deep; 5: 32x32, 32-deep, two chunks in
 *                    flight; 6: 64x64, two chunks in flight; 7: 32 rows x
 *                    64 columns, 8: 64 x 32, both 32-deep; 9 / 10: 64x64
 *                    with each tile's k range split over 2 / 4 workgroups
 *                    and the partial tiles added by a second kernel;
 *                    11 / 12 / 13: the same split over 2 / 4 / 8
 *                    workgroups of 32x32 tiles; 14: 64x64 split 8 ways;
 *                    15 / 16: 32 x 64 split 4 / 8 ways; 17 / 18: kind
 *                    5 split 4 / 8 ways), no tuning;
 *      HZ_COMPOSE=0  inner SIE solved by block LU substitutions at every layer
 *                    application instead of the composed output operators;
 *      HZ_GRAPHS=0   plans launched kernel by kernel instead of replayed HIP
 *                    graphs;
 *      HZ_CELL_NB=w  force w right-hand sides per cell-solve workgroup
 *                    (1, 2, 4, 16 or 32).
 */
#ifndef HZ_H
#define HZ_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hz_ctx hz_ctx;

typedef enum {
    HZ_OK = 0,
    HZ_EINVAL = -1,     /* bad argument: sizes, NaN / non-positive model, partition */
    HZ_ENOMEM = -2,     /* device allocation failed */
    HZ_ESTATE = -3,     /* call out of order (e.g. hz_solve before hz_factor) */
    HZ_ENOCONV = -4,    /* some right-hand side missed tol within max_iter */
    HZ_ESINGULAR = -5,  /* a block of a factorisation is singular to working precision */
    HZ_EDEVICE = -6     /* a HIP runtime error */
} hz_status;

typedef enum {
    HZ_FP64 = 0,        /* everything in complex128 */
    HZ_MIXED = 1,       /* the Gauss-Seidel preconditioner (the sequential
                           sweeps) applies complex64 copies of the interface
                           operators with FP32 accumulation; the SIE matrix,
                           the volume solves and the flexible GMRES stay in
                           complex128 (Sec. 5: a low-accuracy operator for the
                           preconditioner, a high-accuracy one for M) */
    HZ_MIXED_REFINE = 2 /* every local operator (cell factors, interface
                           operators, sweeps) computed and applied in
                           complex64 with FP32 accumulation (the offline
                           stage too) as an approximate inverse, wrapped in
                           FP64 iterative refinement on the volume:
                           u += Hhat^{-1}(f - H u) */
} hz_precision;

typedef enum {
    HZ_MODEL_VELOCITY = 0,   /* model array holds c */
    HZ_MODEL_SLOWNESS2 = 1   /* model array holds m = 1/c^2 */
} hz_model_kind;

typedef enum {
    HZ_PRECOND_GS = 0,       /* block Gauss-Seidel, eq. preconditioner_GS: downward sweep,
                                up-going reflections, upward sweep (Algs. 3-5) */
    HZ_PRECOND_JACOBI = 1    /* block Jacobi, eq. preconditioner_Jac: the two sweeps
                                without the reflections */
} hz_precond;

typedef enum {
    HZ_KRYLOV_GMRES = 0,     /* GMRES (Alg. 6): left-preconditioned in HZ_FP64, flexible
                                right-preconditioned in HZ_MIXED */
    HZ_KRYLOV_BICGSTAB = 1   /* right-preconditioned Bi-CGstab (Sec. 5, Table 3): two
                                applications of M and P per iteration, stopping on the
                                unpreconditioned SIE residual */
} hz_krylov;

typedef enum {
    HZ_INNER_LU = 0,         /* inner SIE of each layer by block LU without pivoting,
                                inverted diagonal blocks (Sec. 4.2.2) */
    HZ_INNER_PT = 1          /* nested polarized traces (Sec. 4.2.1): the inner SIE as a
                                polarized system over the cells, iterated by GMRES with the
                                inner Gauss-Seidel sweeps; no inner factorisation.  Needs
                                HZ_FP64, HZ_KRYLOV_GMRES (run flexible: the preconditioner's
                                inner solves stop at inner_tol) */
} hz_inner;

typedef struct {
    int n_x, n_z;            /* physical nodes per side (must be equal) */
    double h;                /* grid step; must equal 1/(n+1) (unit square) */
    double omega;            /* angular frequency, > 0 */
    int n_pml;               /* PML nodes per side, >= 0 (>= 1 when layers or cells > 1) */
    double pml_beta;         /* sigma_max = pml_beta * omega at the Dirichlet node; <= 0 -> 2 */
    int layers;              /* L: 1..n_z, each layer >= 2 rows */
    int cells;               /* L_c: 1..n_x, each cell >= 2 columns */
    hz_precision precision;
    hz_model_kind model_kind;
    int max_batch;           /* largest B accepted by hz_solve; <= 0 -> 1 */
    hz_precond precond;      /* preconditioner of the polarized SIE (0: Gauss-Seidel) */
    hz_krylov krylov;        /* Krylov method for the polarized SIE (0: GMRES) */
    hz_inner inner;          /* inner solver of the layers (0: block LU) */
    double inner_tol;        /* HZ_INNER_PT: relative tolerance of the inner GMRES inside the
                                preconditioner (<= 0 -> 1e-6, the paper's value; also used by
                                hz_apply_precond); inside hz_solve / hz_adjoint the inner
                                solves of the SIE matrix, the right-hand side and the
                                reconstruction use min(1e-10, max(1e-13, tol / 100)), and the
                                other building blocks 1e-12 */
    int plr;                 /* 1: the Gauss-Seidel preconditioner of single-right-hand-side
                                solves (B = 1) applies the interface operators in partitioned
                                low-rank form (eq. factorization and its PLR footnote; accuracy
                                of the caption of Fig. 9), compressed by hz_factor; the SIE
                                matrix stays dense.  Needs HZ_INNER_LU.  0: dense. */
    double plr_eps;          /* relative Frobenius accuracy of every compressed operator block,
                                ||A - A_plr||_F <= plr_eps ||A||_F (<= 0 -> 1e-8) */
} hz_params;

typedef struct {
    int iters;               /* outer GMRES iterations (summed over refinement steps) */
    double rel_resid;        /* final preconditioned relative residual of the SIE */
    double vol_resid;        /* ||f - H u|| / ||f|| on the extended grid (FP64) */
    int refine_steps;        /* HZ_MIXED_REFINE: refinement steps; otherwise 0 */
    double err_est;          /* HZ_MIXED_REFINE: estimated relative error of u from the
                                observed contraction of the updates; otherwise 0 */
} hz_rhs_stats;

typedef struct {
    double t_setup, t_factor;          /* seconds, last hz_setup / hz_factor */
    double t_rhs, t_gmres, t_recon;    /* seconds, last hz_solve, by phase */
    double t_solve;                    /* seconds, whole last hz_solve */
    int gmres_iters;                   /* max over the batch, last hz_solve */
    int inner_iters;                   /* HZ_INNER_PT: largest inner GMRES iteration count,
                                          last hz_solve (at most 40 per inner solve) */
} hz_timing;

typedef struct {
    int n, n_pml, W;                   /* W = n + 2 n_pml, the trace width */
    int layers, cells;
    int trace_len;                     /* 4 (L-1) W: length of a polarized vector */
    int max_batch;
    long long device_bytes;            /* device memory held by the context */
    long long plr_bytes;               /* device bytes of the compressed operators (0 if none) */
    long long plr_dense_bytes;         /* the same operators stored dense */
    double min_pivot_ratio;            /* smallest |pivot| / largest |pivot| over the block
                                          inversions of the last hz_factor (cell Schur
                                          complements, inner SIE diagonal blocks); 0 before */
} hz_info_t;

/* ---- life cycle ------------------------------------------------------- */

/* Validate prm and the model (n_z x n_x doubles on the device: c or m per
 * prm->model_kind; NaN or <= 0 -> HZ_EINVAL), copy the model, build the
 * coefficients of the global, layer and cell grids (App. A, Fig. 1 and 5).
 * *out receives a new context; on error *out is NULL. */
hz_status hz_setup(const double* model_dev, const hz_params* prm, hz_ctx** out);

/* Offline stage (Sec. 4.3.1, Table 2 rows 1-2): factor every cell
 * (block-tridiagonal Schur recursion along x with explicitly inverted
 * diagonal blocks), precompute every cell's interface operators (eq.
 * factorization: M_f, M_u and the cell-local term) and factor every layer's
 * inner SIE by block LU without pivoting (Sec. 4.2.2).  The block recursions
 * have no pivoting across blocks (Sec. 4.2.2), so a singular block cannot be
 * avoided: HZ_ESINGULAR when a block inversion meets an exactly zero pivot or
 * a smallest pivot magnitude at most 2^-26 times its largest (singular to
 * working precision; hz_get_info reports the smallest ratio seen).  The
 * context is then left set up but not factored (hz_solve returns
 * HZ_ESTATE until a hz_factor succeeds).  May be called again after
 * hz_update_model. */
hz_status hz_factor(hz_ctx* ctx);

/* Online stage (Alg. 6): solve H u = f for B right-hand sides.
 * rhs_dev: B x n_z x n_x complex128 (physical grid, zero-extended into the
 * PML); u_dev: B x n_z x n_x complex128 output (may not alias rhs_dev).
 * tol: per RHS, relative tolerance of the preconditioned SIE residual
 * (HZ_FP64, left-preconditioned GMRES), of the unpreconditioned SIE residual
 * (HZ_MIXED, flexible right-preconditioned GMRES), or of the estimated
 * relative error of the refined volume solution (HZ_MIXED_REFINE).
 * max_iter: GMRES iterations per solve (also the Krylov dimension).
 * stats_host: B entries or NULL.  timing: or NULL.
 * HZ_EINVAL (nothing launched, the context unchanged): a NULL rhs_dev or
 * u_dev, B < 1 or B > max_batch, tol <= 0 or NaN, max_iter < 1.
 * HZ_ESTATE: the context is not factored.
 * HZ_ENOCONV: u_dev holds the last iterate; stats say which RHS failed. */
hz_status hz_solve(hz_ctx* ctx, const void* rhs_dev, int B, void* u_dev,
                   double tol, int max_iter, hz_rhs_stats* stats_host,
                   hz_timing* timing);

/* Adjoint solve H^H lam = rhs (same layout and semantics as hz_solve), the
 * second solve of an adjoint-state misfit gradient (hz_misfit).  The
 * five-point discretisation of App. A, each row divided by the PML factors
 * alpha_x alpha_z of its node, is complex symmetric (H = H^T), so
 * H^H lam = rhs is solved as lam = conj(H^{-1} conj(rhs)) on the same
 * factors. */
hz_status hz_adjoint(hz_ctx* ctx, const void* rhs_dev, int B, void* lam_dev,
                     double tol, int max_iter, hz_rhs_stats* stats_host);

/* Same as hz_solve / hz_adjoint, but the output holds the whole extended
 * grid: B x W x W complex128 with W = n + 2 n_pml (PML nodes included). */
hz_status hz_solve_ext(hz_ctx* ctx, const void* rhs_dev, int B, void* u_ext_dev,
                       double tol, int max_iter, hz_rhs_stats* stats_host,
                       hz_timing* timing);
hz_status hz_adjoint_ext(hz_ctx* ctx, const void* rhs_dev, int B, void* lam_ext_dev,
                         double tol, int max_iter, hz_rhs_stats* stats_host);

/* Adjoint-state gradient of J = 1/2 sum_b ||P u_b - d_b||^2 with respect to
 * m on the physical grid (derived from H's dependence on m, the diagonal term
 * -omega^2 m / (alpha_x alpha_z)):
 *   g[k] = omega^2 Re sum_b sum_{e -> k} w_e u_b[e] conj(lam_b[e]),
 * with w = 1/(alpha_x alpha_z), e running over the extended nodes whose m
 * copies physical node k (PML nodes fold onto the edge nodes they copy),
 * u_b the forward fields and lam_b the adjoint fields
 * H^H lam_b = P^T (P u_b - d_b), both B x W x W complex128 on the extended
 * grid (from hz_solve_ext / hz_adjoint_ext).  g_dev: n_z x n_x double,
 * overwritten.  Needs state "set up" or later. */
hz_status hz_misfit_gradient(hz_ctx* ctx, const void* u_ext_dev, const void* lam_ext_dev,
                             int B, double* g_dev);

/* Least-squares data misfit for receivers on every physical node of depth
 * row rec_row (1-based): r_b = P u_b - d_b, J = 1/2 sum_b ||r_b||^2.
 * u_ext_dev: B x W x W complex128 (from hz_solve_ext); d_obs_dev: B x n_x
 * complex128; adj_src_dev: B x n_z x n_x complex128, overwritten with the
 * adjoint source P^T r_b (zero off the receiver row); *J_host receives J. */
hz_status hz_misfit(hz_ctx* ctx, const void* u_ext_dev, const void* d_obs_dev, int rec_row,
                    int B, void* adj_src_dev, double* J_host);

/* Allocation-free variant of hz_misfit, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same inputs and adjoint source as
 * hz_misfit; J is written to device memory (*J_dev, one double) instead of
 * the host.  The kernel's partial sums live in a library-owned file-scope
 * device array of 256 doubles (2 KB), one copy per device that the library
 * runs on, held until the process ends; its size does not depend on B or n,
 * so no input size is rejected for it, and every call overwrites all of it
 * (nothing needs clearing).  The call allocates nothing (no hipMalloc /
 * hipFree), enqueues its work on the context's stream and returns without
 * waiting: synchronise that stream before reading *J_dev or adj_src_dev.
 * J equals hz_misfit's value bit for bit (the partials are added in the same
 * order).  Calls that overlap on one GPU (from any context, any stream)
 * race on the shared array.  Errors: HZ_EINVAL as hz_misfit (or J_dev NULL),
 * HZ_ESTATE before hz_setup, HZ_EDEVICE on a HIP error. */
hz_status hz_misfit_noalloc(hz_ctx* ctx, const void* u_ext_dev, const void* d_obs_dev,
                            int rec_row, int B, void* adj_src_dev, double* J_dev);

/* Replace the model (same size and kind) and rebuild the coefficients; the
 * context returns to the "set up" state (hz_factor must be called again).
 * HZ_EINVAL for a bad model (checked first: the context is then unchanged). */
hz_status hz_update_model(hz_ctx* ctx, const double* model_dev);

/* Local re-factorisation after a model update (Sec. 6: in an inversion loop
 * the solver is modified only where the medium changed).  ctx must be
 * factored.  model_dev: the new model, same size, kind and device layout as
 * for hz_setup.  The coefficients are rebuilt; the cells whose local
 * operators changed (bitwise) get new Schur factors and interface operators,
 * and the inner SIE factors and composed operators are rebuilt for the
 * layers holding a changed cell.  The result equals that of
 * hz_update_model followed by hz_factor (in every precision form).
 * ncells_refactored: host int, or NULL; receives the number of cells redone.
 * Errors: HZ_ESTATE if ctx is not factored; HZ_EINVAL for a bad model (NaN,
 * infinite or non-positive entries: checked first, ctx unchanged);
 * HZ_ESINGULAR as hz_factor. */
hz_status hz_update_model_local(hz_ctx* ctx, const double* model_dev, int* ncells_refactored);

/* Enqueue all further work of ctx on `hip_stream` (a hipStream_t, or NULL for
 * the null stream).  Waits for the work already enqueued; captured plans are
 * rebuilt for the new stream. */
hz_status hz_set_stream(hz_ctx* ctx, void* hip_stream);

/* Kernel timing for roofline measurements.  While profiling is on, every
 * launch of the solver's dense kernels is bracketed by HIP events on the
 * context's stream, and its algorithmic traffic (each operator entry and
 * vector element the method must read or write, counted once per launch)
 * and flops are accumulated per kernel family.  hz_profile(ctx, 1) clears
 * the counters; hz_profile_read fills up to `max` records. */
typedef struct {
    char name[32];           /* kernel family (one record per family and launch shape) */
    int launches;
    double ms;               /* summed launch durations (event to event) */
    double bytes;            /* summed algorithmic bytes */
    double flops;            /* summed algorithmic flops */
} hz_kstat;
hz_status hz_profile(hz_ctx* ctx, int on);
hz_status hz_profile_read(hz_ctx* ctx, hz_kstat* out, int max, int* count);

hz_status hz_get_info(const hz_ctx* ctx, hz_info_t* info);
hz_status hz_get_timing(const hz_ctx* ctx, hz_timing* timing);

void hz_destroy(hz_ctx* ctx);
const char* hz_strerror(hz_status s);
const char* hz_last_error(void);

/* ---- building blocks, exposed for parity tests ----------------------------
 * These run single steps of the online path on the factors of a context in
 * state "factored".  Polarized vectors use the layout
 *   x[i][b], i in [0, 4 (L-1) W): (d_0, ..., d_{L-2}, q_0, ..., q_{L-2}),
 * each d_k / q_k a pair (trace on row a, trace on row b) of length 2W;
 * interface k lies between layers k and k+1 (0-based), row a is the last row
 * of layer k and row b the first row of layer k+1.  B is the fastest index. */

/* R_side (H^l)^{-1}[T_l(top) + B_l(bot)]: layer l's Green's integrals
 * applied to a top pair and a bottom pair (App. C equivalent sources),
 * sampled on the top rows (side = 0: local rows 0, 1) or bottom rows
 * (side = 1: local rows n_l, n_l + 1).  top/bot/out: [2][W][B] complex128;
 * top or bot may be NULL (absent). */
hz_status hz_apply_layer(hz_ctx* ctx, int layer, const void* top_dev,
                         const void* bot_dev, int side, void* out_dev, int B);

/* y = M x, the polarized SIE matrix (eq. M_polarized, jump conditions). */
hz_status hz_apply_sie(hz_ctx* ctx, const void* x_dev, void* y_dev, int B);

/* y = P^GS x, the Gauss-Seidel preconditioner (eq. preconditioner_GS):
 * downward sweep, up-going reflections, upward sweep. */
hz_status hz_apply_precond(hz_ctx* ctx, const void* x_dev, void* y_dev, int B);

/* Right-hand side of the polarized system (Alg. 6 lines 2-7) for the B
 * sources rhs_dev (B x n_z x n_x): y = (R_bot N^k f ; R_top N^{k+1} f). */
hz_status hz_sie_rhs(hz_ctx* ctx, const void* rhs_dev, void* y_dev, int B);

/* (H^{l,c})^{-1} g on the full grid of cell c of layer l.  g, x:
 * [HL][Wc][B] complex128, HL = rows of the layer grid, Wc = columns of the
 * cell grid (cell-local, artificial PML included). */
hz_status hz_cell_solve(hz_ctx* ctx, int layer, int cell, const void* g_dev,
                        void* x_dev, int B);

/* Grid sizes of layer l / cell c: *HL, *Wc. */
hz_status hz_cell_shape(const hz_ctx* ctx, int layer, int cell, int* HL, int* Wc);

/* r = f - H u on the extended grid (W x W per RHS), complex128, [b][z][x]. */
hz_status hz_residual(hz_ctx* ctx, const void* u_ext_dev, const void* f_ext_dev,
                      void* r_ext_dev, int B);

#ifdef __cplusplus
}
#endif
#endif /* HZ_H */
