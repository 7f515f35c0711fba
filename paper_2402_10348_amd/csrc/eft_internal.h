// Internal declarations of the HIP library behind include/eft.h.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "eft.h"

#define EFT_MAX_IND 64
#define EFT_MAX_PHASE 65
#define EFT_MAX_SOLID 64
#define EFT_MAX_RESTART 512

// ------------------------------------------------------------ matrices ----

// BSR matrix with row-major bs x bs blocks.  Values live in val (FP64) or,
// for the reduced-precision Jacobian, in val32 (FP32).
struct eft_matrix {
    int32_t bs = 0;
    int64_t n = 0, nnzb = 0;
    int32_t *rowptr = nullptr, *col = nullptr, *diag = nullptr;  // device
    double *val = nullptr;
    float *val32 = nullptr;
    uint16_t *val16 = nullptr;   // BF16 values (the finest multigrid level's copy)
    const double *bcmp = nullptr;  // B systems: the blocks in compact form (s1, M), see eft_bcmp_*
    // the pattern in stencil form, or null: every column of row r is r +
    // stn_off[s] for the set bits s of stn_mask[r] (ascending), see eft_stencil_form
    uint16_t *stn_mask = nullptr;
    int32_t *stn_off = nullptr;
    // band systems: FP32 copies for the Jacobi preconditioner (values or
    // compact blocks, block inverses), written by the solve's set-up; null:
    // the preconditioner reads the FP64 arrays
    float *pc32 = nullptr;
    float *dinv32 = nullptr;
    bool fp32 = false;
    bool bf16 = false;
};

// FGMRES workspace for vectors of length nd = n*bs and restart m.
struct KrylovWs {
    int64_t cap_nd = 0;
    int32_t cap_m = 0;
    int64_t cap_n = 0;
    int32_t cap_bs = 0;
    double *V = nullptr;        // [m+1][nd]
    double *Z = nullptr;        // [m][nd]
    double *w = nullptr;        // [nd]
    double *r = nullptr;        // [nd]
    double *Dinv = nullptr;     // [n][bs*bs]
    double *part = nullptr;     // reduction partials
    double *small = nullptr;    // device scalars: H, cs, sn, g, y, h, norms
    int32_t *flag = nullptr;    // [8]: active, columns done, breakdown, second-pass gate, -,
                                // learned fallback, singular diagonal block, -
    int32_t nblk = 0;           // blocks of the reduction kernels
};

// Block ILU(0) factors of the momentum/mass matrix and their level schedule
// (rows grouped by the longest chain of lower, resp. upper, dependencies).
struct IluState {
    double *lu = nullptr, *dinv = nullptr;      // [nnzb][bs*bs] L below, U on and above the diagonal; [n][bs*bs] U_ii^-1
    int32_t *lrows = nullptr, *urows = nullptr;  // rows by level (device)
    std::vector<int32_t> loff, uoff;            // level offsets (host)
};

// Compact system on the band of one indicator.  Its arrays are slices of
// the context's band pool (BandPool), reserved at creation.
struct Band {
    int64_t n = 0, ne = 0, nnz = 0;            // band nodes, band elements, pattern size
    int32_t *node = nullptr;                   // [n] global id of band node
    int32_t *elem = nullptr;                   // [ne] global id of band element
    int32_t *epos = nullptr;                   // [ne][nn*nn] position in band pattern
    int32_t *bconn_ = nullptr;                 // [ne][nn] band-local node ids
    uint8_t *fre = nullptr;                    // [n] 1 if the node is solved for
    uint8_t *eflag = nullptr;                  // [E] 1 for band elements
    int32_t *rowptr = nullptr, *col = nullptr, *diag = nullptr;
};

// Storage of the bands of all indicators, sized once (eft_create,
// eft_set_params) for band_reserve x the mesh's elements, so that building
// the bands inside a time step allocates nothing.  Band k takes the next
// slices of each array.
struct BandPool {
    int64_t cap_e = 0, cap_n = 0, cap_nnz = 0;     // elements, nodes, pattern entries of all bands
    int64_t used_n = 0;                            // nodes of the bands built last
    int32_t *elem = nullptr, *epos = nullptr, *bconn = nullptr;       // [cap_e], [cap_e nn^2], [cap_e nn]
    int32_t *node = nullptr, *rowptr = nullptr, *diag = nullptr;      // [cap_n], [cap_n + n_ind], [cap_n]
    uint8_t *fre = nullptr;                                           // [cap_n]
    int32_t *col = nullptr;                                           // [cap_nnz]
    uint8_t *eflag = nullptr;                                         // [n_ind][E]
};

// One level of the mesh with the node fields the element kernels read.
struct MeshView {
    int64_t N = 0, E = 0;
    const int32_t *conn = nullptr, *epos = nullptr;
    const double *xyz = nullptr;
    const double *va = nullptr, *acc = nullptr, *rho = nullptr, *mu = nullptr, *as = nullptr, *Ba = nullptr;
    const uint64_t *smask = nullptr;                 // [N] bit s: solid s has a non-zero fraction at the node
    int64_t n_dir = 0;
    const int32_t *dir_node = nullptr;
    const uint8_t *dir_mask = nullptr;
    const int32_t *iptr = nullptr, *ient = nullptr;  // node -> (element << 2 | local node)
    const uint32_t *islot = nullptr;  // per incidence entry: its row's block slots, see eft_build_graph
    int maxc = 0, rpb = 1;                           // longest matrix row, rows per workgroup
    const uint8_t *fmask = nullptr;                  // [N] bit c set when dof c is free (others: unit rows)
    // node records staged per assembly workgroup (null: read from the node arrays), see eft_ns_stage_build
    const int32_t *wnptr = nullptr, *wnode = nullptr;
    const uint32_t *iloc = nullptr;
    int maxnl = 0, maxpw = 0;
};

// One level of the geometric multigrid hierarchy on nested Kuhn meshes.
// Level 0 is the momentum/mass mesh itself (its mesh arrays and matrix are
// the context's); coarser levels own theirs.
struct MGLevel {
    int n[3] = {1, 1, 1};            // cells per axis
    int64_t N = 0, E = 0;
    int32_t *conn = nullptr, *epos = nullptr, *inj = nullptr;  // inj: fine-mesh node of each node
    int32_t *iptr = nullptr, *ient = nullptr;
    uint32_t *islot = nullptr;
    int maxc = 0, rpb = 1;
    double *xyz = nullptr;
    double *va = nullptr, *acc = nullptr, *rho = nullptr, *mu = nullptr, *as = nullptr, *Ba = nullptr;
    uint64_t *smask = nullptr;       // [N] solids present at each node (injected from the fine level)
    double *vp = nullptr, *R = nullptr;
    int64_t n_dir = 0;
    int32_t *dir_node = nullptr;
    uint8_t *dir_mask = nullptr;
    uint8_t *fmask = nullptr;        // [N]: bit c set when dof c is free (not Dirichlet)
    eft_matrix A;                    // FP32 values (level 0: FP32 copy of the Jacobian)
    double *Dinv = nullptr;          // [N][bs*bs] (levels with FP64 values)
    float *Dinv32 = nullptr;         // [N][bs*bs] (the level with FP32 values)
    double *x = nullptr, *x2 = nullptr, *b = nullptr, *r = nullptr;  // [N*bs]
    float *xf = nullptr, *xf2 = nullptr, *rf = nullptr;   // [N*bs] the finest level's FP32 iterate and residual
    uint16_t *Dinv16 = nullptr;      // [N][bs*bs] the finest level's block inverses in BF16 (its FP32-vector cycle)
    int32_t *crow = nullptr;         // rows ordered by parity colour (i%2, j%2, k%2)
    int64_t coff[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // colour c: crow[coff[c] .. coff[c+1])
    int64_t cnnz[8] = {0, 0, 0, 0, 0, 0, 0, 0};     // blocks of the rows of each colour
    int ncolor = 0;
};

// Learned right preconditioner (not in the paper; the learned form of the
// right preconditioner of the FGMRES solve): parameters, Adam moments,
// activations of one vector, and harvested training pairs.
struct NNState {
    int H = 64, L = 4, bs = 0, F = 0;
    int64_t np = 0;                     // parameters
    int64_t cap_n = 0;                  // nodes the activations are sized for
    float *theta = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
    int64_t adam_t = 0;
    float *mask = nullptr;              // [N][bs]: 1 free dof, 0 Dirichlet dof
    float *f = nullptr;                 // [N][F] input features
    float *pre = nullptr, *h = nullptr; // [L+1][N][H] pre-activations, activations
    float *g = nullptr;                 // [L][N][H] neighbour means
    float *d1 = nullptr, *d2 = nullptr; // [N][2H] backward scratch
    float *delta = nullptr;             // [N][bs] network output
    float *part = nullptr;              // split-K and column-sum partials
    int64_t cap_part = 0;
    double *u = nullptr;                // [N][bs] base vector of the input (block Jacobi or V-cycle)
    int32_t *on = nullptr;              // a device flag that reads 1 (ungated V-cycles of the harvest)
    double *red = nullptr;              // reduction partials; scalars at the end
    double *losses = nullptr;           // [cap_steps] training losses
    int64_t cap_steps = 0;
    int32_t cap_pairs = 0;              // harvest ring (0: harvesting off)
    int64_t stored = 0, next = 0;       // pairs written so far, next ring slot
    float *hu = nullptr, *he = nullptr; // [cap_pairs][N][bs]: u = D^-1 r and e (A e = r)
    bool ready = false;
};

// Optional HIP-event timing of kernel roles (a measurement hook): each
// launch of a timed role is bracketed by two events on the context's stream
// and carries its algorithmic bytes.  Launches inside a Krylov chunk are
// tagged with their column; columns the solve never reached ran gated off and
// are counted with zero bytes.
enum { EFT_KT_SMOOTH = 1, EFT_KT_SPMV = 2, EFT_KT_ASSEMBLE = 3, EFT_KT_NROLE = 4 };
struct KTimer {
    uint32_t mask = 0;              // bit r: role r is timed
    int tag = -1;                   // Krylov column being enqueued (-1: none)
    std::vector<hipEvent_t> ev;     // event pool, two per pending launch
    std::vector<double> pbytes;     // bytes of each pending launch
    std::vector<int> ptag, prole;   // tag and role of each pending launch
    int64_t pend = 0;
    int64_t launches[EFT_KT_NROLE] = {}, active[EFT_KT_NROLE] = {};
    double seconds[EFT_KT_NROLE] = {}, bytes[EFT_KT_NROLE] = {};
};

struct eft_ctx {
    hipStream_t stream = nullptr;
    std::string err;
    int dim = 0, nn = 0, bs = 0, nv = 0;
    int64_t N = 0, E = 0;
    // materials
    int n_phase = 0, n_ind = 0, n_s = 0, bg = -1;
    std::vector<eft_phase> phase;
    std::vector<int> ind_phase;     // phase of indicator k
    std::vector<int> solid_phase;   // phase of solid s
    std::vector<int> solid_ind;     // indicator of solid s
    double g[3] = {0, 0, 0};
    eft_params par{};
    KTimer kt;
    NNState net;                    // learned preconditioner
    // device mesh
    double *xyz = nullptr;
    int32_t *conn = nullptr;
    int32_t *epos = nullptr;        // [E][nn*nn] position of (a,b) in the NS pattern
    int32_t *iptr = nullptr, *ient = nullptr;  // node -> incident (element << 2 | local node)
    uint32_t *islot = nullptr;      // per incidence entry: its row's block slots (eft_build_graph)
    uint8_t *fmask0 = nullptr;      // [N] bit c set when dof c of the node is free (not Dirichlet)
    int maxc = 0, rpb = 1;          // longest row of the node graph, rows per band-assembly workgroup
    int rpb_ns = 1;                 // rows per momentum/mass assembly workgroup
    // per assembly workgroup: its nodes (wnode[wnptr[w] .. wnptr[w + 1])) and per
    // incidence entry the list positions of the element's nodes (null: not staged)
    int32_t *wnptr = nullptr, *wnode = nullptr;
    uint32_t *iloc = nullptr;
    int maxnl = 0, maxpw = 0;
    int32_t *cell_of = nullptr;     // [E] band grid cell of each element
    int64_t n_dir = 0;
    int32_t *dir_node = nullptr;
    uint8_t *dir_mask = nullptr;
    double *dir_val = nullptr;
    double *phase_tab = nullptr;    // [5][EFT_MAX_PHASE]: kind, transported, rho, mu, mu_L
    int32_t *ind_of_phase = nullptr;   // [n_phase] indicator index or -1
    // band grid
    int ng[3] = {1, 1, 1};
    // momentum/mass matrix and node fields
    eft_matrix J;
    double *va = nullptr, *acc = nullptr;      // [N][d]
    double *rho = nullptr, *mu = nullptr;      // [N]
    uint64_t *smask = nullptr;                 // [N] bit s: solid s has a non-zero fraction at the node
    int32_t *solid_ind_d = nullptr;            // [n_s] indicator of each solid (device)
    // the level-n and iterate arrays eft_props last read: the element kernels
    // compute solid fractions and B at n+alpha from them for the solids
    // present, instead of reading full per-solid arrays
    const double *src_lphi = nullptr, *src_iphi = nullptr, *src_lB = nullptr, *src_iB = nullptr;
    double *R = nullptr, *dx = nullptr;        // [N][max(bs,nv)]
    // level-n copies used by eft_step
    double *l_vp = nullptr, *l_vdot = nullptr, *l_phi = nullptr, *l_phidot = nullptr, *l_B = nullptr,
           *l_Bdot = nullptr;
    // transport
    std::vector<Band> band;                    // per indicator
    BandPool bp;
    double band_node_ratio = 1.0;              // most nodes per element over the band grid's cells
    double h_min = 0.0;                        // smallest mesh spacing of the box (band overflow test)
    bool bands_valid = false;
    // block-diagonal union of the band systems of one kind (all Allen-Cahn
    // systems, all B systems), solved together; rebuilt with the bands
    struct BandUnion {
        int64_t n = 0, nnz = 0, cap_n = 0, cap_nnz = 0;
        int32_t *rowptr = nullptr, *col = nullptr, *diag = nullptr;
        std::vector<int> band_of;              // band of each member system
        std::vector<int64_t> roff, noff;       // row / block offsets of each member
    } u_ac, u_b;
    double *tsc = nullptr;                     // [1024] device transport scalars
    double *htsc = nullptr;                    // [1024] pinned host copy
    uint8_t *seed = nullptr, *active = nullptr;  // [n_cells]
    uint8_t *nin = nullptr, *nout = nullptr;     // [N]
    uint8_t *ein = nullptr;                      // [E]
    int32_t *g2b = nullptr;                      // [N] global -> band id
    int32_t *gpos2b = nullptr;                   // [nnzb] global pattern pos -> band pos
    int32_t *scan_tmp = nullptr;                 // scan workspace
    int64_t scan_cap = 0;
    double *bR = nullptr, *bX = nullptr;         // band system rhs / solution [cap][nv]
    double *bval = nullptr;                      // band matrix values [cap_nnz][nv*nv]
    double *bcmp = nullptr;                      // B blocks in compact form [cap_nnz][1 + dim^2]
    double *bdiag = nullptr;                     // B systems: diagonal blocks [cap_n][nv^2] by union row
    float *bpc32 = nullptr;                      // FP32 copy of bval / bcmp for the Jacobi preconditioner
    float *bdinv32 = nullptr;                    // FP32 block inverses of the band system [cap_n][nv^2]
    void *hmem = nullptr, *dmem = nullptr;       // member descriptors and unit tables of the batched
                                                 // transport launches (pinned host, device)
    double *tpart = nullptr;                     // partial sums of the batched mobility / beta
    int64_t tpart_cap = 0;
    int32_t *iota = nullptr;                     // [cap_n]: i (diagonal index of bdiag)
    double *tnum = nullptr, *tden = nullptr;     // mobility projection sums [cap_n]
    // reductions and host mirror
    double *red = nullptr;                       // partial sums
    double *dscal = nullptr;                     // device scalars
    double *hscal = nullptr;                     // pinned host scalars
    int32_t nred = 0;
    KrylovWs kw;
    IluState ilu;
    // HIP graphs of the columns of a multigrid-preconditioned momentum solve,
    // one per column index, with what they were captured on
    struct ColGraphs {
        std::vector<hipGraphExec_t> exec;
        eft_params par{};
        std::vector<const void *> key;
        hipStream_t cap = nullptr;   // the stream they are recorded on (the caller's may be the null stream)
    } colg;
    // geometric multigrid (structured Kuhn meshes with even cell counts)
    bool structured = false;
    std::vector<MGLevel> mg;
    double *mg_dense = nullptr, *mg_inv = nullptr;   // coarsest level [nd][nd] over its free dofs
    int32_t *mg_fidx = nullptr, *mg_free = nullptr;  // dof -> free index, free index -> dof
    int32_t *mg_miss = nullptr;                      // Galerkin product found no slot (consistency flag)
    int64_t mg_nd = 0;
    bool mg_f32_fresh = false;   // the finest level's FP32 or BF16 copy was written by the assembly
    bool mg_valid = false;       // the hierarchy belongs to the Jacobian now in J (set by eft_mg_setup)
    int nl_k = 0;                // nonlinear iteration of the running eft_step (1-based; 0 outside)
    // diagnostics workspace (centre of mass partials, particles)
    double *dg = nullptr;
    int64_t dg_cap = 0;
    // bounding box of the mesh nodes (host)
    double bb_lo[3] = {0, 0, 0}, bb_hi[3] = {0, 0, 0};
    // device address of the fixed workspace array on this context's GPU
    // (eft_fgmres_noalloc), and the guard that makes a workspace reservation
    // fail instead of allocating while that entry point runs
    double *scratch = nullptr;
    bool no_alloc = false;
};

// ------------------------------------------------------------- helpers ----

#define EFT_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);               \
            return EFT_EDEVICE;                                                         \
        }                                                                               \
    } while (0)

#define EFT_TRY(expr)                      \
    do {                                   \
        eft_status s_ = (expr);            \
        if (s_ != EFT_OK) return s_;       \
    } while (0)

static inline int eft_grid(int64_t n, int block) { return (int)((n + block - 1) / block); }

// generalized-alpha constants (Sec. 2.1.2)
struct GA {
    double alpha, alpha_m, vs, dt, ct, kappa;
};
static inline GA ga_of(double rho_inf, double dt)
{
    GA g;
    g.alpha = 1.0 / (1.0 + rho_inf);
    g.alpha_m = 0.5 * (3.0 - rho_inf) / (1.0 + rho_inf);
    g.vs = 0.5 + g.alpha_m - g.alpha;
    g.dt = dt;
    g.ct = g.alpha_m / (g.vs * dt);
    g.kappa = g.alpha * g.vs * dt / g.alpha_m;
    return g;
}

// ------------------------------------------------- kernels (launchers) ----

// k_assemble.hip
eft_status eft_props(eft_ctx *ctx, const eft_state *lvl, const eft_iterate *it);
eft_status eft_ns_kernels(eft_ctx *ctx, const eft_iterate *it, double *R, eft_matrix *J);
// (J32, J16: when given, an FP32 or BF16 copy of the values written by the
// same launch)
eft_status eft_ns_level(eft_ctx *ctx, const MeshView &M, const double *vp, double *R, eft_matrix *J,
                        float *J32 = nullptr, uint16_t *J16 = nullptr);

bool eft_stencil_form(int64_t n, const std::vector<int32_t> &rowptr, const std::vector<int32_t> &col, int maxs,
                      std::vector<int32_t> &soff, std::vector<uint16_t> &smask);
bool eft_ns_stage_build(int64_t N, int nn, const int32_t *conn, const std::vector<int32_t> &iptr,
                        const std::vector<int32_t> &ient, int rpb, std::vector<int32_t> &wnptr,
                        std::vector<int32_t> &wnode, std::vector<uint32_t> &iloc, int &maxnl, int &maxpw);

// k_mg.hip
eft_status eft_mg_create(eft_ctx *ctx, const int32_t *grid, const std::vector<uint8_t> &dmask0);
eft_status eft_mg_setup(eft_ctx *ctx, const double *vp, bool coarse = true);
eft_status eft_mg_vcycle(eft_ctx *ctx, const double *b0, double *z, const int32_t *flag);
void eft_mg_free(eft_ctx *ctx);
// the multigrid preconditioner is requested and possible for A / and its
// hierarchy belongs to the Jacobian now in A
bool eft_mg_enabled(const eft_ctx *ctx, const eft_matrix *A);
bool eft_mg_active(const eft_ctx *ctx, const eft_matrix *A);
eft_status eft_ilu_reserve(eft_ctx *ctx);
void eft_ilu_free(eft_ctx *ctx);
eft_status eft_ilu_setup(eft_ctx *ctx, const eft_matrix *A, int32_t *sing);
eft_status eft_ilu_apply(eft_ctx *ctx, const double *r, double *z, const int32_t *flag);
eft_status eft_mg_reserve(eft_ctx *ctx);
eft_status eft_build_graph(int64_t N, int64_t E, int nn, const int32_t *conn, std::vector<int32_t> &rowptr,
                           std::vector<int32_t> &col, std::vector<int32_t> &diag, std::vector<int32_t> &epos,
                           std::vector<int32_t> &iptr, std::vector<int32_t> &ient, std::vector<uint32_t> &islot,
                           int &maxc, int &rpb, int &rpb_ns, std::string &err);
eft_status eft_fill(eft_ctx *ctx, double *p, int64_t n, double v);
eft_status eft_fill32(eft_ctx *ctx, float *p, int64_t n, float v);
eft_status eft_fill_u8(eft_ctx *ctx, uint8_t *p, int64_t n);

// k_sparse.hip
eft_status eft_spmv_dev(eft_ctx *ctx, const eft_matrix *A, const double *x, double *y);
// (sing: optional device flag set to 1 when a diagonal block is singular; its
// inverse is then replaced by the identity)
eft_status eft_bj_setup(eft_ctx *ctx, const eft_matrix *A, double *Dinv, int32_t *sing = nullptr);
eft_status eft_bj_setup32(eft_ctx *ctx, const eft_matrix *A, float *Dinv, int32_t *sing = nullptr);
// the Jacobi preconditioner of a band system reads its FP32 copies (values
// or compact blocks in pc32, block inverses in dinv32)
inline bool eft_jacobi_narrow(const eft_matrix *A)
{
    return A->pc32 && A->dinv32 && (A->bs == 1 || A->bcmp);
}
eft_status eft_bj_apply(eft_ctx *ctx, int bs, int64_t n, const double *Dinv, const double *x, double *z,
                        const int32_t *active);
// z = M v with M = `sweeps` damped point-block Jacobi sweeps from z = 0
// (tmp: scratch of the size of v; sweeps = 1, omega = 1 is block Jacobi;
// the products read the compact blocks A->bcmp when they are set)
eft_status eft_jacobi_apply(eft_ctx *ctx, const eft_matrix *A, const double *Dinv, const double *v, double *z,
                            double *tmp, int sweeps, double omega, const int32_t *active);
eft_status eft_spmv_flag(eft_ctx *ctx, const eft_matrix *A, const double *x, double *y, const int32_t *active);
// B-system products from the compact blocks (A->bcmp, bs 3 or 6): y = A x,
// and one damped Jacobi sweep zo = z + omega D^-1 (v - A z)
eft_status eft_bcmp_spmv(eft_ctx *ctx, const eft_matrix *A, const double *x, double *y, const int32_t *active);
eft_status eft_bcmp_sweep(eft_ctx *ctx, const eft_matrix *A, const double *Dinv, double omega, const double *v,
                          const double *z, double *zo, const int32_t *active);

// k_krylov.hip
eft_status eft_krylov_reserve(eft_ctx *ctx, int64_t n, int bs, int m);
eft_status eft_fgmres_dev(eft_ctx *ctx, const eft_matrix *A, const double *b, double *x, eft_solve_info *info,
                          double rtol = 0.0);   // rtol <= 0: par.lin_rtol
eft_status eft_norm2(eft_ctx *ctx, const double *x, int64_t n, double *out_host);
// looks up (once per device) the address of the fixed workspace array on the
// current device and records it in the context
eft_status eft_scratch_attach(eft_ctx *ctx);

// k_transport.hip
eft_status eft_bands_build_dev(eft_ctx *ctx, const double *phi_n);
eft_status eft_transport_dev(eft_ctx *ctx, const eft_state *lvl, eft_iterate *it, eft_transport_info *info);
eft_status eft_band_system_dev(eft_ctx *ctx, const eft_state *lvl, const eft_iterate *it, int kind, int index,
                               int64_t *n, int64_t *nnz, int32_t *node, int32_t *rowptr, int32_t *col, double *R,
                               double *J, double *gamma_beta);

// band pool and band-system workspaces for band_reserve (frees the old ones;
// invalidates the bands)
eft_status eft_band_reserve(eft_ctx *ctx);
void eft_band_free(eft_ctx *ctx);

// kernel timing hook (abi.hip)
int64_t eft_kt_begin(eft_ctx *ctx, int role);
void eft_kt_end(eft_ctx *ctx, int64_t slot, double bytes, int role);
void eft_kt_void_from(eft_ctx *ctx, int tag0);
eft_status eft_kt_harvest(eft_ctx *ctx);

// learned preconditioner (k_nn.hip)
eft_status eft_nn_alloc(eft_ctx *ctx);
void eft_nn_free(eft_ctx *ctx);
// (flag[5] is set to 1 when a network output was not finite and the node
// fell back to block Jacobi)
eft_status eft_nn_precond(eft_ctx *ctx, const double *Dinv, const double *v, double *z, int32_t *flag);
eft_status eft_nn_store_pair(eft_ctx *ctx, const double *Dinv, const double *r, const double *e, int64_t slot,
                             const int32_t *flag);
