/*
 * eft.h -- C ABI of the MI355X hot path of the fully Eulerian phase-field
 * fluid-structure method of Mao & Jaiman (arXiv 2402.10348): one partitioned
 * nonlinear iteration of a time step, i.e.
 *   (a) assembly of the unified, phase-interpolated momentum/mass residual and
 *       Jacobian (eq. PG_NS, tau_m/tau_c, Newtonian and left-Cauchy-Green
 *       stress, elastic tangent of eq. Bext / Appendix B),
 *   (b) the sparse Krylov solve of eq. LS_NS (BSR SpMV + FGMRES),
 *   (c) the Allen-Cahn order-parameter transport of every indicator
 *       (eqs. Allen-Cahn, tdm-num, PPV_AC) and the B-tensor transport of every
 *       solid (eq. semiCGT), restricted to a grid-cell band around each
 *       interface, with the stop rule of Sec. 2.4.
 *
 * Conventions
 *   - Plain C types only.  Mesh, material and parameter arguments of
 *     eft_create are HOST pointers and are copied.  Every field, vector and
 *     matrix array argument of the other calls is a DEVICE pointer (HIP device
 *     memory, FP64 unless stated) owned by the caller; the library never frees
 *     caller memory.
 *   - Dimension d is 2 (triangles) or 3 (tetrahedra).  Nodal blocks are
 *     interleaved: vp is [N][d+1] = (v_0..v_{d-1}, p) per node.
 *   - Symmetric tensors use the Voigt order [11,22,33,12,23,13] (d = 3) or
 *     [11,22,12] (d = 2), Sec. 2.5 remark; nv = 6 or 3.
 *   - All work is enqueued on the HIP stream given to eft_create; calls that
 *     return host-visible results (info structs, status) synchronize it.
 *   - A context is not thread-safe; one stream per context.
 *   - The return code is the only error channel; eft_last_error gives text.
 */
#ifndef EFT_H
#define EFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EFT_OK = 0,
    EFT_EINVAL = 1,          /* bad argument (null, size, unsupported value)       */
    EFT_ENOMEM = 2,          /* device or host allocation failed                   */
    EFT_EDEVICE = 3,         /* a HIP call failed                                  */
    EFT_ENOTCONV = 4,        /* Krylov solve hit its iteration cap (best iterate
                                returned, info filled)                             */
    EFT_EBREAKDOWN = 5,      /* singular system: the point-block Jacobi or ILU(0)
                                preconditioner met a singular diagonal block, or
                                FGMRES could make no progress                      */
    EFT_ENAN = 6,            /* NaN/Inf met; fields keep the last good iterate     */
    EFT_EBAND_OVERFLOW = 7,  /* max|v| dt exceeds the band halo width              */
    EFT_EUNSUPPORTED = 8     /* valid request the library does not implement       */
} eft_status;

typedef struct eft_ctx eft_ctx;        /* opaque; owns every internal buffer */
typedef struct eft_matrix eft_matrix;  /* opaque BSR matrix owned by a ctx   */

/* Fixed Eulerian mesh of P1 simplices (Sec. 2.1.2), HOST arrays. */
typedef struct {
    int32_t dim;                 /* 2 or 3                                         */
    int64_t n_nodes, n_elems;
    const double *xyz;           /* [n_nodes][dim]                                 */
    const int32_t *conn;         /* [n_elems][dim+1], positive orientation         */
    int64_t n_dir;               /* Dirichlet nodes of the momentum/mass block     */
    const int32_t *dir_node;     /* [n_dir]                                        */
    const uint8_t *dir_mask;     /* [n_dir]: bit k<dim velocity k, bit dim pressure */
    const double *dir_val;       /* [n_dir][dim+1] prescribed values               */
    int32_t grid[3];             /* structured cell counts of the box (band grid)  */
} eft_mesh;

/* One phase (Sec. 2.1.1): fluid (Newtonian, Sec. 2.2) or Neo-Hookean solid
 * (Sec. 2.3).  Exactly the transported phases carry an order parameter; at
 * most one non-transported phase fills the complement. */
typedef struct {
    int32_t kind;                /* 0 fluid, 1 solid                               */
    int32_t transported;         /* 1: own order parameter; 0: background          */
    double rho, mu, mu_L;        /* density, dynamic viscosity, shear modulus      */
} eft_phase;

typedef struct {
    int32_t n_phases;            /* <= 65 (at most 64 order parameters)            */
    const eft_phase *phase;      /* HOST [n_phases]                                */
    double g[3];                 /* gravity; body force rho g                      */
} eft_materials;

typedef struct {
    double dt;                   /* time step                                      */
    double rho_inf;              /* generalized-alpha spectral radius (paper: 0)   */
    double eps;                  /* interface thickness parameter                  */
    double eta;                  /* mobility regularization eta                    */
    double C_I;                  /* inverse-estimate constant in tau_m             */
    double di_cut;               /* diffuse-interface cut |phi| <= 0.9             */
    double nl_rtol;              /* stop rule ||dx||/||x|| (paper: 5e-4)           */
    int32_t nl_max;              /* nonlinear iteration cap (paper: 20)            */
    int32_t nl_fixed;            /* >0: run exactly this many iterations           */
    double lin_rtol;             /* FGMRES relative residual target                */
    int32_t restart;             /* FGMRES restart length m (<= 512)               */
    int32_t lin_maxit;           /* FGMRES iteration cap per solve                 */
    int32_t precond;             /* 0 point-block Jacobi; 1 geometric multigrid V-
                                    cycle for the momentum/mass block when the mesh
                                    is a structured Kuhn box with even cell counts
                                    (point-block Jacobi otherwise, and always for
                                    the band systems); 2 learned preconditioner
                                    (a network correction of block Jacobi or of the
                                    V-cycle, see nn_base and eft_nn_init) for the
                                    momentum/mass block; 3
                                    block ILU(0) of the momentum/mass matrix in the
                                    natural row order (factors on the matrix
                                    pattern, level-scheduled factorization and
                                    triangular solves; point-block Jacobi for the
                                    band systems).  The factors' storage (one more
                                    copy of the matrix values) is reserved by
                                    eft_create / eft_set_params.                   */
    int32_t precision;           /* 0 FP64; 1 FP32 Jacobian values + FP64 rest     */
    double band_flat;            /* band seed: |phi^n| < 1 - band_flat; a negative
                                    value seeds every cell, so the transport runs
                                    on the whole mesh (no band)                   */
    int32_t band_cell;           /* mesh cells per grid cell and axis              */
    int32_t band_halo;           /* grid-cell layers added around the seeds        */
    int32_t mg_nu;               /* multigrid: smoothing sweeps before the coarse
                                    correction, the first from x = 0 (1..16)       */
    double mg_omega;             /* multigrid: damping of the block-Jacobi sweeps  */
    int32_t mg_bf16;             /* multigrid: 1 stores the finest level's matrix
                                    copy in BF16 (block inverses from the FP64
                                    diagonal blocks), 0 in FP32                    */
    int32_t mg_nu_post;          /* multigrid: smoothing sweeps after the coarse
                                    correction (1..16)                             */
    int32_t mg_smoother;         /* multigrid: 0 damped node-block Jacobi; 1 node-
                                    block Gauss-Seidel over the parity colours of
                                    the Kuhn mesh (forward before, backward after
                                    the coarse correction)                         */
    int32_t band_sweeps;         /* preconditioner of the Allen-Cahn and B band
                                    systems: this many damped point-block Jacobi
                                    sweeps from z = 0 (1..8; 1 with band_omega = 1
                                    is plain point-block Jacobi).  The sweeps read
                                    FP32 copies of the values and block inverses
                                    (FP64 vectors and arithmetic); the Krylov
                                    products stay FP64                             */
    double band_omega;           /* damping of those sweeps (0 < omega <= 1.5)      */
    int32_t mg_galerkin;         /* multigrid coarse operators: 0 rediscretized (the
                                    element kernels on node fields injected from
                                    the fine mesh), 1 Galerkin products P^T A P of
                                    the fine operator with the V-cycle's transfers */
    int32_t nn_maxit;            /* learned preconditioner: Krylov iterations of
                                    one momentum solve after which the rest of the
                                    solve uses its base (block Jacobi or the
                                    V-cycle), its fallback (<= 0: lin_maxit / 2)  */
    double band_reserve;         /* band storage reserved at eft_create and
                                    eft_set_params: the bands of all indicators
                                    together may hold this many times the mesh's
                                    elements (with band_flat < 0 at least the
                                    indicator count); <= 0 picks 1, but never less
                                    than 2^20 elements or every band the whole
                                    mesh, the smaller of the two.  A step whose
                                    bands need
                                    more returns EFT_ENOMEM with the state
                                    unchanged; eft_step itself never allocates.   */
    int32_t graphs;              /* 1: each column of a multigrid-preconditioned
                                    momentum solve (V-cycle, SpMV, Gram-Schmidt)
                                    is captured once into a HIP graph and replayed
                                    (not while kernel timing, pair harvesting or
                                    the learned preconditioner is on); 0: every
                                    launch enqueued from the host.  Same kernels,
                                    same results.  The graphs are kept until the
                                    parameters or the workspace change.           */
    int32_t nn_base;             /* learned preconditioner (precond = 2): the
                                    vector the network corrects, z = b + s m NN(b/s,
                                    m): 0 the point-block Jacobi vector D^-1 r; 1
                                    the multigrid V-cycle's output (structured
                                    meshes; EFT_EINVAL without a hierarchy).  With
                                    a zero output layer the preconditioner is
                                    exactly that base, which is also its fallback.
                                    Harvested pairs store the base of A z_j.      */
    int32_t mg_lag;              /* multigrid inside eft_step: 0 every assembly
                                    refreshes the whole hierarchy; 1 the coarse
                                    levels (Galerkin products or rediscretized
                                    operators, their block inverses, the coarsest
                                    inverse) are refreshed at the first nonlinear
                                    iteration of a step only, the finest level
                                    (copy of J, block inverses) at every one.  The
                                    preconditioner changes, the answer does not. */
    int32_t mg_cnu;              /* multigrid coarse levels (all but the finest and
                                    the coarsest with its dense solve): smoothing
                                    sweeps before the coarse correction, the first
                                    from x = 0 (1..32; 0: mg_nu)                   */
    int32_t mg_cnu_post;         /* ... and after it (1..32; 0: mg_nu_post)         */
} eft_params;

/* State at time level n (Sec. 2.1.2): values and rates.  DEVICE arrays. */
typedef struct {
    double *vp;                  /* [N][d+1]                                       */
    double *vdot;                /* [N][d]                                         */
    double *phi;                 /* [n_ind][N]                                     */
    double *phidot;              /* [n_ind][N]                                     */
    double *B;                   /* [n_s][N][nv]                                   */
    double *Bdot;                /* [n_s][N][nv]                                   */
    double t;
    int64_t step;
} eft_state;

/* Current nonlinear iterate x^{n+1,(k)}.  DEVICE arrays, shapes as above. */
typedef struct {
    double *vp;
    double *phi;
    double *B;
} eft_iterate;

typedef struct {
    int32_t iters;               /* Krylov iterations                              */
    int32_t restarts;            /* completed restart cycles                       */
    int32_t converged;           /* 1 if ||b - A x|| <= lin_rtol ||b||             */
    int32_t fallback_used;       /* 1: the requested preconditioner gave way to a
                                    plain one: point-block Jacobi for an
                                    unavailable multigrid (mesh not a structured
                                    Kuhn box, or the matrix not assembled by
                                    eft_assemble/eft_step), or the learned one's
                                    base (block Jacobi or the V-cycle) where it
                                    produced a non-finite value (those nodes) or
                                    after nn_maxit iterations (the rest of the
                                    solve)                                        */
    double rel_res0;             /* ||b - A x0|| / ||b|| (x0 = 0: 1)               */
    double rel_res;              /* final true relative residual                   */
} eft_solve_info;

typedef struct {
    int32_t n_ind, n_solid;
    double gamma[64];            /* mobility per indicator                         */
    double beta[64];             /* Lagrange multiplier per indicator              */
    int64_t band_nodes[64];      /* band size per indicator                        */
    int64_t band_elems[64];
    int32_t lin_iters[128];      /* per indicator, then per solid: iterations of
                                    the solve the system took part in             */
    double ratio[128];           /* ||dx||/||x|| per indicator, then per solid     */
    int32_t ac_iters, b_iters;   /* Krylov iterations of the batched Allen-Cahn
                                    solve (all indicators) and B solve (all solids)*/
} eft_transport_info;

typedef struct {
    int32_t nl_iters;            /* nonlinear iterations taken                     */
    int32_t converged;           /* stop rule met (or nl_fixed reached)            */
    int32_t lin_iters_total;     /* Krylov iterations over all blocks              */
    int32_t n_blocks;            /* 1 + n_ind + n_s                                */
    double block_ratio[129];     /* last ||dx||/||x|| per block: [v,p], phi_i, B_s */
    double t_assemble, t_solve, t_transport;   /* seconds (host clock)            */
    int32_t lin_iters_block[129];/* Krylov iterations per block over the step      */
} eft_step_info;

typedef struct {
    int64_t launches;            /* timed launches of the kernel role              */
    int64_t active;              /* of these, launches that did work (launches of
                                    Krylov columns past convergence return at once) */
    double seconds;              /* summed HIP-event durations                     */
    double bytes;                /* summed algorithmic bytes: every unique byte the
                                    kernel must read or write, once (matrix values,
                                    indices, vectors; for the assembly J, R, the
                                    connectivity and the node fields it reads)     */
} eft_kernel_time;

/* Create a context: copies the mesh to the device, builds the node graph
 * (BSR pattern of eq. LS_NS) and every workspace.  hip_stream may be NULL
 * (default stream).  EFT_EINVAL on inconsistent sizes or orientation. */
eft_status eft_create(const eft_mesh *mesh, const eft_materials *mat, const eft_params *par,
                      void *hip_stream, eft_ctx **out);
eft_status eft_destroy(eft_ctx *ctx);
const char *eft_last_error(const eft_ctx *ctx);

/* Replace the solver parameters (dt, tolerances, band definition ...). */
eft_status eft_set_params(eft_ctx *ctx, const eft_params *par);

/* The context-owned Jacobian of the momentum/mass block (bs = d+1). */
eft_status eft_ns_matrix(eft_ctx *ctx, eft_matrix **out);
eft_status eft_matrix_shape(const eft_matrix *A, int64_t *n_rows, int64_t *nnzb, int32_t *bs);
/* Copy pattern and FP64 values (FP32 values are widened) into caller DEVICE
 * buffers: rowptr [n_rows+1], col [nnzb], val [nnzb][bs][bs] row-major. */
eft_status eft_matrix_export(eft_ctx *ctx, const eft_matrix *A, int32_t *rowptr, int32_t *col, double *val);

/* Overwrite the values of a context matrix with caller values val
 * [nnzb][bs][bs] (FP64, DEVICE, row-major blocks in the pattern of
 * eft_matrix_export; narrowed when the matrix holds FP32 values).  The
 * matrix is then no longer the assembled Jacobian: until the next assembly
 * its solves use point-block Jacobi (the multigrid hierarchy is built by the
 * assembly).  For solving other systems of the same pattern, and tests. */
eft_status eft_matrix_import(eft_ctx *ctx, eft_matrix *A, const double *val);

/* Block ILU(0) factors of the current momentum/mass matrix (test hook,
 * precond = 3): factors it and copies the factors into DEVICE buffers lu
 * [nnzb][bs][bs] (the strictly lower blocks hold L, whose diagonal blocks
 * are the identity and not stored; the others U) and dinv [n][bs][bs] =
 * U_ii^-1; either may be null.  L U equals the matrix on its pattern
 * (standard block ILU(0), natural order).  Synchronizes the context stream.
 * EFT_EINVAL without precond = 3, EFT_EBREAKDOWN on a singular U_ii. */
eft_status eft_ilu_export(eft_ctx *ctx, double *lu, double *dinv);

/* Multigrid hierarchy of the momentum/mass preconditioner (test hook):
 * level 0 is the mesh itself; level l has cells of 2^l mesh cells.  With
 * null buffers: *levels, and for level `level` (when valid) its rows n and
 * pattern size nnzb.  Otherwise copies the level's pattern and operator into
 * DEVICE buffers rowptr [n+1], col [nnzb], val [nnzb][bs][bs] (FP64; FP32
 * levels are widened; level 0 gives the FP64 Jacobian).  The operators are
 * those of the last assembly.  EFT_EINVAL without a hierarchy. */
eft_status eft_mg_export(eft_ctx *ctx, int32_t level, int32_t *levels, int64_t *n, int64_t *nnzb, int32_t *rowptr,
                         int32_t *col, double *val);

/* (a) Momentum/mass residual R [N][d+1] (FP64) and Jacobian J of eq. (PG_NS)
 * at the iterate, with the elastic tangent of eq. (Bext), Dirichlet rows
 * replaced by unit rows and zero residual.  J may be NULL (residual only). */
eft_status eft_assemble(eft_ctx *ctx, const eft_state *level_n, const eft_iterate *it, double *R,
                        eft_matrix *J);

/* (b) y = A x for a context matrix; x, y [n_rows][bs]. */
eft_status eft_spmv(eft_ctx *ctx, const eft_matrix *A, const double *x, double *y);

/* (b) Solve A x = b with right-preconditioned FGMRES(restart), x0 = 0, the
 * preconditioner chosen by par.precond (point-block Jacobi, the multigrid
 * V-cycle, the learned one with its base as fallback, or block ILU(0));
 * classical Gram-Schmidt with a conditional second pass, all in FP64.  x is
 * output only.  EFT_ENOTCONV if lin_maxit is reached (x = best iterate);
 * EFT_EBREAKDOWN on a singular diagonal block (point-block Jacobi, ILU(0));
 * EFT_ENAN on a non-finite right-hand side or iterate; EFT_EINVAL for a
 * learned preconditioner without parameters, or nn_base = 1 without a
 * multigrid hierarchy. */
eft_status eft_fgmres(eft_ctx *ctx, const eft_matrix *A, const double *b, double *x, eft_solve_info *info);

/* Allocation-free variant of eft_fgmres, for callers that cannot allocate
 * device memory (code under HIP stream capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, preconditioner, result
 * and errors as eft_fgmres, but the Krylov workspace (basis V, Z, w, r, the
 * block inverses, reduction partials, Hessenberg data, flags) lives in one
 * fixed device array of 64 MiB that the library holds on each GPU it runs on
 * until the process ends; nothing is allocated or freed.  Limit:
 * (2 restart + 3) n bs + n bs^2 + the reduction partials <= 8 Mi doubles
 * (e.g. restart 50, bs 4: up to about 40,000 nodes); larger systems get
 * EFT_EINVAL.  Every call on one GPU shares the array and leaves its last
 * contents there: calls that overlap on one GPU (two streams, two threads)
 * race.  Harvesting of training pairs must be off (EFT_EINVAL otherwise). */
eft_status eft_fgmres_noalloc(eft_ctx *ctx, const eft_matrix *A, const double *b, double *x, eft_solve_info *info);

/* (c) Build the transport band of every indicator from phi^n (grid cells of
 * band_cell mesh cells seeded by |phi^n| < 1 - band_flat, dilated by band_halo
 * layers; nodes touched by a non-band element keep their value). */
eft_status eft_bands_build(eft_ctx *ctx, const eft_state *level_n);

/* Export the band of indicator k: band_elem [E] and free_node [N] as 0/1
 * bytes, DEVICE buffers (test hook). */
eft_status eft_band_export(eft_ctx *ctx, int32_t k, uint8_t *band_elem, uint8_t *free_node);

/* Assemble one band system at the iterate and copy it out (test hook):
 * kind 0 = Allen-Cahn system of indicator `index` (with its gamma and beta),
 * kind 1 = B system of solid `index`.  Rows of kept nodes are unit rows with
 * zero residual.  Call once with null buffers to get n (band nodes) and nnz
 * (pattern size); then node [n] (global ids), rowptr [n+1], col [nnz]
 * (band-local ids), R [n][bs] and J [nnz][bs][bs] (bs = 1 or nv) are DEVICE
 * buffers; gamma_beta [2] is a HOST buffer (kind 0).  Requires
 * eft_bands_build. */
eft_status eft_band_system(eft_ctx *ctx, const eft_state *level_n, const eft_iterate *it, int32_t kind,
                           int32_t index, int64_t *n, int64_t *nnz, int32_t *node, int32_t *rowptr, int32_t *col,
                           double *R, double *J, double *gamma_beta);

/* (c) One transport pass of the partitioned iteration (eqs. LS_AC, LS_MC):
 * for every indicator the mobility gamma (eq. tdm-num, RMS over |phi| <= 0.9),
 * beta, one Allen-Cahn solve on its band; then for every solid one B solve on
 * the band of its indicator with the updated phi.  The systems of one kind
 * are solved together, as one block-diagonal system whose member rows are
 * scaled by 1/||b_k||, to lin_rtol / sqrt(members), so that every member
 * meets lin_rtol.  Updates it->phi and it->B
 * in place.  Requires eft_bands_build for the current level. */
eft_status eft_transport_solids(eft_ctx *ctx, const eft_state *level_n, eft_iterate *it,
                                eft_transport_info *info);

/* Centre of mass of the region of each order parameter (Sec. 3, rotating
 * disk case): x_c = int x alpha dOmega / int alpha dOmega with alpha =
 * clamp((1 + phi)/2, 0, 1) at the nodes, interpolated linearly; per element
 * the degree-2 simplex rule (exact here); partial sums reduced in a fixed
 * order.  phi [n_ind][N] is a DEVICE array; xc [n_ind][3] (components past
 * dim are 0; xc = 0 where the measure is 0) and mass [n_ind] (int alpha
 * dOmega) are HOST arrays.  Synchronizes the context stream. */
eft_status eft_center_of_mass(eft_ctx *ctx, const double *phi, double *xc, double *mass);

/* Particle tracking (Appendix, parallel particle tracking): for each of the
 * n_p particles x [n_p][dim] (HOST, in/out) every element is tested; the
 * particle lies in an element when all its P1 shape functions at x are in
 * [-tol, 1 + tol] (the lowest element index wins on shared faces); it then
 * moves by dt sum_a N_a(x) v_a with the velocities of vp [N][dim+1]
 * (DEVICE; one explicit Euler step).  elem [n_p] (HOST) receives the
 * element, or -1 when none contains x (x unchanged).  n_p <= 4096, tol >=
 * 0; EFT_EINVAL otherwise.  Synchronizes the context stream. */
eft_status eft_track_particles(eft_ctx *ctx, const double *vp, int32_t n_p, double dt, double tol, double *x,
                               int32_t *elem);

/* Closed triangle surface mesh (HOST arrays): vert [n_vert][3], tri
 * [n_tri][3] vertex indices. */
typedef struct {
    int32_t n_vert, n_tri;
    const double *vert;
    const int32_t *tri;
} eft_surface;

/* Order parameter of the solid bounded by a closed surface mesh, on the
 * mesh nodes (the paper's phase-field interface processing: grid cells,
 * Algorithm "distance", ray casting with non-duplicated plane partitioning,
 * Algorithm "sign"; 3D only, EFT_EUNSUPPORTED in 2D).  ncell[3] grid cells
 * over the nodes' bounding box; a triangle belongs to the cells its bounding
 * box grown by 3 eps overlaps.  Nodes of cells with triangles: |phi| =
 * tanh(|d| / (sqrt2 eps)), |d| the shortest distance to those triangles'
 * vertices; other nodes |phi| = 1.  Sign by a +X ray, crossings in the Y-Z
 * projection when A1 + A2 + A3 - A0 <= 2 chi (areas), classified as element,
 * edge or node crosses and counted once per vertex-id combination; odd:
 * inside, phi > 0.  A ray that only touches the surface at a vertex counts
 * as a crossing (the method's limit).  phi [N] is a DEVICE array (output).
 * crossings [2] (HOST, may be NULL): the most distinct crossings of one ray
 * and 1 when a ray had more than 32 (its count truncated).  Allocates and
 * frees its own temporaries; synchronizes the context stream. */
eft_status eft_init_phase(eft_ctx *ctx, const eft_surface *surf, double eps, const int32_t *ncell, double chi,
                          double *phi, int32_t *crossings);

/* One time step (Sec. 2.4): predictor, bands, nonlinear iterations
 * NS -> indicators -> solids until every block satisfies ||dx||/||x|| <
 * nl_rtol or nl_max (exactly nl_fixed when > 0), corrector.  Advances *st in
 * place (t += dt, step += 1).  A non-converged nonlinear loop still returns
 * EFT_OK with info->converged = 0 (the paper continues after 20 iterations). */
eft_status eft_step(eft_ctx *ctx, eft_state *st, double dt, eft_step_info *info);

/* ---- Autotuner of the solver's run-time knobs (not part of the method).
 * The multigrid sweep counts before/after the coarse correction (on the
 * finest level and on the coarse levels), its damping,
 * smoother kind (Jacobi or multicolour Gauss-Seidel) and coarse operators
 * (rediscretized or Galerkin), and the sweeps and
 * damping of the band systems' preconditioner are chosen by measurement: on
 * the state st (as the first nonlinear iteration of a step sees it) the
 * momentum/mass system is assembled once and solved once per candidate (a
 * candidate's solve stops at three times the best one's iterations, the entry
 * settings' at 400; one that does not converge there is not chosen), and
 * one transport pass is timed per band candidate (on copies of phi and B; st
 * is not changed).  None of these knobs changes the converged answer; the
 * definition parameters (band_cell, band_halo, band_flat, eps, eta, dt,
 * tolerances) are never changed.  The best set is kept in the context's
 * parameters.  cache_path (HOST string, may be NULL): a text file of
 * "key|knobs" lines, the key made of the GPU architecture and the problem's
 * sizes, materials and solver settings; a key found there is applied without
 * a search, a new result is appended.  budget: most momentum candidates
 * timed (<= 0: 96).  info (HOST, may be NULL) receives the outcome. */
typedef struct {
    int32_t evaluated;           /* solves and transport passes timed              */
    int32_t from_cache;          /* 1: knobs read from the cache file              */
    double default_seconds;      /* one momentum solve with the entry knobs        */
    double best_seconds;         /* ... with the chosen knobs                      */
    int32_t default_iters, best_iters;
    double band_default_seconds; /* one transport pass with the entry knobs        */
    double band_best_seconds;
    int32_t mg_nu, mg_nu_post, mg_smoother;
    double mg_omega;
    int32_t mg_galerkin;
    int32_t band_sweeps;
    double band_omega;
    int32_t mg_cnu, mg_cnu_post;
} eft_tune_info;
eft_status eft_tune(eft_ctx *ctx, const eft_state *st, const char *cache_path, int32_t budget, eft_tune_info *info);

/* Measurement hook, not part of the method: time every launch of the kernel
 * roles set in role_mask with a pair of HIP events on the context's stream.
 * Bit 1 = fine-level multigrid smoother sweep (x + omega D^-1 (b - A x) with
 * the finest level's copy of the momentum Jacobian: BF16 with mg_bf16 = 1,
 * the default, FP32 otherwise), bit 2 = SpMV of the momentum
 * Jacobian inside FGMRES, bit 3 = momentum/mass assembly on the mesh (not the
 * coarse levels).  0 turns timing off.  Resets the counters; two event records
 * per timed launch are added to the stream.  EFT_EINVAL for other bits. */
eft_status eft_time_kernel(eft_ctx *ctx, int32_t role_mask);

/* Counters of one role (1, 2 or 3, as the bits above) since eft_time_kernel
 * (synchronizes the context's stream).  *out is a HOST struct.  EFT_EINVAL
 * for another role. */
eft_status eft_kernel_time_read(eft_ctx *ctx, int32_t role, eft_kernel_time *out);

/* ---- Learned right preconditioner (not in the paper).  FGMRES admits any
 * variable right preconditioner M in eq. (LS_NS), so the network changes the
 * iteration count only, never the converged answer.  With the base u = D^-1 r
 * (node-block Jacobi, nn_base = 0) or u = the multigrid V-cycle applied to r
 * (nn_base = 1), s = sqrt(mean(u^2)) and m the free-dof mask:
 *   z = u + s (m * NN(u / s, m)),
 * NN = a message-passing network on the matrix graph: input layer 2 bs -> H,
 * L layers h <- relu([h, mean of neighbours' h] W_l + b_l), output H -> bs
 * (H = 64, L = 4).  Parameters: one FP32 vector, W_in [2bs][H], b_in [H],
 * then per layer W_l [2H][H], b_l [H], then W_out [H][bs].  The dense layers
 * run on MFMA with BF16 operands and FP32 accumulation.  Training pairs
 * (u = base of r, e) with A e = r are harvested from the context's own
 * momentum FGMRES solves.  The parameters do not depend on the mesh size:
 * a network trained on a small mesh applies to a large one (eft_nn_params). */

/* Allocate (first call) and initialize the parameters from a seed; W_out = 0,
 * so the preconditioner starts as its base.  Adam moments are reset. */
eft_status eft_nn_init(eft_ctx *ctx, uint64_t seed);

/* hidden width, layer count, parameter count (0 before eft_nn_init) and the
 * number of harvested pairs held; any pointer may be NULL. */
eft_status eft_nn_shape(eft_ctx *ctx, int32_t *hidden, int32_t *layers, int64_t *n_params, int64_t *pairs);

/* Copy the parameters to (direction 0) or from (1) the HOST array host[n];
 * n must equal the parameter count.  EFT_EINVAL otherwise or before init. */
eft_status eft_nn_params(eft_ctx *ctx, float *host, int64_t n, int32_t direction);

/* Keep the last `capacity` training pairs of the momentum FGMRES solves that
 * follow: every Krylov column j gives (base of A z_j, z_j), every converged
 * solve (base of b, x), the base after nn_base (with nn_base = 1 one more
 * V-cycle per column).  0 stops harvesting and frees the ring.  The pairs
 * take 2 capacity N (d+1) FP32 values of device memory. */
eft_status eft_nn_harvest(eft_ctx *ctx, int32_t capacity);

/* Train on the harvested pairs: `steps` Adam steps (beta 0.9, 0.999), each on
 * the summed gradient of `batch` pairs drawn with a xorshift generator seeded
 * by `seed`, loss ||m (z(u) - e)||^2 / ||m e||^2.  losses (HOST, may be NULL)
 * receives the loss of the first pair of every step.  EFT_EINVAL without
 * pairs or before init. */
eft_status eft_nn_train(eft_ctx *ctx, int32_t steps, int32_t batch, double lr, uint64_t seed, double *losses);

/* Loss and gradient of one pair (u, e) (DEVICE FP64 [N][d+1]) at the current
 * parameters; grad_host (HOST, parameter count, may be NULL) and loss (HOST)
 * receive them.  For tests of the backward pass. */
eft_status eft_nn_loss_grad(eft_ctx *ctx, const double *u, const double *e, float *grad_host, double *loss);

/* z = u + s (m * NN(u / s, m)) for a DEVICE base vector u (already block-
 * Jacobi or V-cycle preconditioned), z DEVICE; both FP64 [N][d+1]. */
eft_status eft_nn_apply(eft_ctx *ctx, const double *u, double *z);

#ifdef __cplusplus
}
#endif

#endif /* EFT_H */
