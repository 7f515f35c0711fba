// C ABI of include/eft.h: context set-up (node graph, element-to-block map,
// band grid), the entry points of the hot path, and the time step of Sec. 2.4
// (predictor, partitioned nonlinear iterations NS -> order parameters -> B
// tensors with the stop rule, corrector).
#include <chrono>
#include <climits>
#include <cstring>
#include <numeric>

#include "dev_common.h"
#include "eft_internal.h"

namespace {

__global__ void k_apply_dirichlet(int64_t n_dir, const int32_t *node, const uint8_t *mask, const double *val, int BS,
                                  double *vp)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_dir) return;
    const int64_t n = node[t];
    for (int i = 0; i < BS; ++i)
        if ((mask[t] >> i) & 1) vp[n * BS + i] = val[t * BS + i];
}

__global__ void k_neg(double *x, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = -x[i];
}

__global__ void k_add(double *x, const double *d, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] += d[i];
}

// rate at n+1 from x^n, xdot^n and x^{n+1} (update formula of Sec. 2.1.2);
// value stride sx, rate stride sd, ncomp components per entity
__global__ void k_rates(int64_t n, int ncomp, int sx, int sd, const double *xn, const double *xdn, const double *x1,
                        double *xd1, double dt, double vs)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * ncomp) return;
    const int64_t p = t / ncomp;
    const int c = (int)(t - p * ncomp);
    const double a = xn[p * sx + c], ad = xdn[p * sd + c], b = x1[p * sx + c];
    xd1[p * sd + c] = ad + (b - a - dt * ad) / (vs * dt);
}

__global__ void k_widen(const float *a, double *b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (double)a[i];
}

__global__ void k_scatter_one(int64_t n, const int32_t *idx, uint8_t *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[idx[i]] = 1;
}

__global__ void k_scatter_u8(int64_t n, const int32_t *idx, const uint8_t *v, uint8_t *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[idx[i]] = v[i];
}

int sgrid(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(8192, (n + 255) / 256)); }

template <typename T> eft_status dalloc(eft_ctx *ctx, T **p, int64_t count)
{
    *p = nullptr;
    if (count <= 0) count = 1;
    if (hipMalloc((void **)p, sizeof(T) * (size_t)count) != hipSuccess) {
        ctx->err = "out of device memory";
        return EFT_ENOMEM;
    }
    return EFT_OK;
}

template <typename T> eft_status upload(eft_ctx *ctx, T **p, const T *h, int64_t count)
{
    EFT_TRY(dalloc(ctx, p, count));
    if (count > 0) EFT_HIP(hipMemcpy(*p, h, sizeof(T) * (size_t)count, hipMemcpyHostToDevice));
    return EFT_OK;
}

void free_all(eft_ctx *ctx)
{
    auto fr = [](void *p) {
        if (p) (void)hipFree(p);
    };
    fr(ctx->xyz); fr(ctx->conn); fr(ctx->epos); fr(ctx->iptr); fr(ctx->ient); fr(ctx->islot); fr(ctx->wnptr); fr(ctx->wnode); fr(ctx->iloc); fr(ctx->cell_of); fr(ctx->dir_node); fr(ctx->dir_mask); fr(ctx->fmask0);
    fr(ctx->dir_val); fr(ctx->phase_tab); fr(ctx->ind_of_phase);
    fr(ctx->J.rowptr); fr(ctx->J.col); fr(ctx->J.stn_mask); fr(ctx->J.stn_off); fr(ctx->J.diag); fr(ctx->J.val); fr(ctx->J.val32);
    fr(ctx->va); fr(ctx->acc); fr(ctx->rho); fr(ctx->mu); fr(ctx->smask); fr(ctx->solid_ind_d); fr(ctx->R); fr(ctx->dx);
    fr(ctx->l_vp); fr(ctx->l_vdot); fr(ctx->l_phi); fr(ctx->l_phidot); fr(ctx->l_B); fr(ctx->l_Bdot);
    eft_band_free(ctx);
    fr(ctx->seed); fr(ctx->active); fr(ctx->nin); fr(ctx->nout); fr(ctx->ein); fr(ctx->g2b); fr(ctx->gpos2b);
    fr(ctx->red);
    fr(ctx->dscal);
    eft_mg_free(ctx);
    eft_ilu_free(ctx);
    KrylovWs &K = ctx->kw;
    fr(K.V); fr(K.Z); fr(K.w); fr(K.r); fr(K.Dinv); fr(K.part); fr(K.small); fr(K.flag);
    for (hipGraphExec_t g : ctx->colg.exec)
        if (g) (void)hipGraphExecDestroy(g);
    ctx->colg.exec.clear();
    if (ctx->colg.cap) (void)hipStreamDestroy(ctx->colg.cap);
    ctx->colg.cap = nullptr;
    if (ctx->hscal) (void)hipHostFree(ctx->hscal);
    if (ctx->htsc) (void)hipHostFree(ctx->htsc);
    fr(ctx->tsc);
    fr(ctx->dg);
    for (hipEvent_t e : ctx->kt.ev) (void)hipEventDestroy(e);
    ctx->kt.ev.clear();
    eft_nn_free(ctx);
}

eft_status check_params(eft_ctx *ctx, const eft_params *p)
{
    if (!(p->dt > 0.0) || !(p->eta > 0.0) || p->restart < 1 || p->restart > EFT_MAX_RESTART || p->lin_maxit < 1 ||
        p->band_cell < 1 || p->band_halo < 0 || p->nl_max < 1 || !(p->lin_rtol > 0.0) || p->rho_inf < 0.0 ||
        p->rho_inf > 1.0 || (p->precision != 0 && p->precision != 1) || (p->precond < 0 || p->precond > 3) ||
        p->mg_nu < 1 || p->mg_nu > 16 || !(p->mg_omega > 0.0) || p->mg_omega > 1.5 ||
        (p->mg_bf16 != 0 && p->mg_bf16 != 1) || p->mg_nu_post < 1 || p->mg_nu_post > 16 ||
        (p->mg_smoother != 0 && p->mg_smoother != 1) || p->band_sweeps < 1 || p->band_sweeps > 8 ||
        !(p->band_omega > 0.0 && p->band_omega <= 1.5) || (p->mg_galerkin != 0 && p->mg_galerkin != 1) ||
        (p->graphs != 0 && p->graphs != 1) || (p->nn_base != 0 && p->nn_base != 1) ||
        (p->mg_lag != 0 && p->mg_lag != 1) || p->mg_cnu < 0 || p->mg_cnu > 32 || p->mg_cnu_post < 0 ||
        p->mg_cnu_post > 32) {
        ctx->err = "invalid eft_params (dt, eta, lin_rtol > 0; 1 <= restart <= 512; band_cell >= 1; "
                   "0 <= rho_inf <= 1; precision 0/1; precond 0/1/2/3; 1 <= mg_nu <= 16; 0 < mg_omega <= 1.5; mg_bf16 0/1; 1 <= mg_nu_post <= 16; mg_smoother 0/1; 1 <= band_sweeps <= 8; 0 < band_omega <= 1.5; mg_galerkin 0/1; graphs 0/1; nn_base 0/1; mg_lag 0/1; 0 <= mg_cnu, mg_cnu_post <= 32)";
        return EFT_EINVAL;
    }
    return EFT_OK;
}

eft_status alloc_jacobian_values(eft_ctx *ctx)
{
    const int64_t n = ctx->J.nnzb * ctx->bs * ctx->bs;
    if (ctx->J.val) (void)hipFree(ctx->J.val);
    if (ctx->J.val32) (void)hipFree(ctx->J.val32);
    ctx->J.val = nullptr;
    ctx->J.val32 = nullptr;
    ctx->J.fp32 = ctx->par.precision == 1;
    if (ctx->J.fp32) return dalloc(ctx, &ctx->J.val32, n);
    return dalloc(ctx, &ctx->J.val, n);
}

// True when the mesh is the structured Kuhn (Freudenthal) split of a box:
// nodes numbered lexicographically (x fastest) on a uniform grid and every
// simplex a monotone lattice path from a cell corner to the opposite corner.
bool structured_kuhn(int d, const int32_t *grid, int64_t N, int64_t E, const double *xyz, const int32_t *conn)
{
    int64_t np = 1, nc = 1;
    for (int k = 0; k < d; ++k) {
        np *= grid[k] + 1;
        nc *= grid[k];
    }
    if (np != N || E != nc * (d == 3 ? 6 : 2)) return false;
    double lo[3], hi[3];
    for (int k = 0; k < d; ++k) {
        lo[k] = 1e300;
        hi[k] = -1e300;
    }
    for (int64_t p = 0; p < N; ++p)
        for (int k = 0; k < d; ++k) {
            lo[k] = std::min(lo[k], xyz[p * d + k]);
            hi[k] = std::max(hi[k], xyz[p * d + k]);
        }
    auto idx = [&](int64_t p, int k) -> int64_t {
        if (k == 0) return p % (grid[0] + 1);
        if (k == 1) return (p / (grid[0] + 1)) % (grid[1] + 1);
        return p / ((int64_t)(grid[0] + 1) * (grid[1] + 1));
    };
    for (int64_t p = 0; p < N; ++p)
        for (int k = 0; k < d; ++k) {
            const double x = lo[k] + (hi[k] - lo[k]) * (double)idx(p, k) / grid[k];
            if (std::fabs(xyz[p * d + k] - x) > 1e-9 * (hi[k] - lo[k])) return false;
        }
    const int nn = d + 1;
    for (int64_t e = 0; e < E; ++e) {
        int64_t mn[3] = {INT64_MAX, INT64_MAX, INT64_MAX};
        for (int a = 0; a < nn; ++a)
            for (int k = 0; k < d; ++k) mn[k] = std::min(mn[k], idx(conn[e * nn + a], k));
        int off[4][3], sum[4];
        for (int a = 0; a < nn; ++a) {
            sum[a] = 0;
            for (int k = 0; k < d; ++k) {
                off[a][k] = (int)(idx(conn[e * nn + a], k) - mn[k]);
                if (off[a][k] < 0 || off[a][k] > 1) return false;
                sum[a] += off[a][k];
            }
        }
        // one node per lattice level 0..d, each adding one unit vector
        int at[4] = {-1, -1, -1, -1};
        for (int a = 0; a < nn; ++a) {
            if (sum[a] > d || at[sum[a]] >= 0) return false;
            at[sum[a]] = a;
        }
        for (int l = 1; l <= d; ++l)
            for (int k = 0; k < d; ++k)
                if (off[at[l]][k] < off[at[l - 1]][k]) return false;
    }
    return true;
}

eft_status create_impl(eft_ctx *ctx, const eft_mesh *mesh, const eft_materials *mat, const eft_params *par)
{
    const int d = mesh->dim;
    if (d != 2 && d != 3) {
        ctx->err = "dim must be 2 or 3";
        return EFT_EINVAL;
    }
    if (mesh->n_nodes <= 0 || mesh->n_elems <= 0 || !mesh->xyz || !mesh->conn ||
        mesh->n_nodes > 2000000000LL || mesh->n_elems > 2000000000LL ||
        (mesh->n_dir > 0 && (!mesh->dir_node || !mesh->dir_mask || !mesh->dir_val))) {
        ctx->err = "invalid mesh";
        return EFT_EINVAL;
    }
    for (int k = 0; k < d; ++k)
        if (mesh->grid[k] < 1) {
            ctx->err = "grid cell counts must be >= 1";
            return EFT_EINVAL;
        }
    EFT_TRY(check_params(ctx, par));
    ctx->par = *par;
    ctx->dim = d;
    ctx->nn = d + 1;
    ctx->bs = d + 1;
    ctx->nv = d == 3 ? 6 : 3;
    const int64_t N = mesh->n_nodes, E = mesh->n_elems;
    const int nn = ctx->nn, bs = ctx->bs, nv = ctx->nv;
    ctx->N = N;
    ctx->E = E;
    // materials
    if (!mat || mat->n_phases < 1 || mat->n_phases > EFT_MAX_PHASE || !mat->phase) {
        ctx->err = "invalid materials";
        return EFT_EINVAL;
    }
    ctx->n_phase = mat->n_phases;
    ctx->phase.assign(mat->phase, mat->phase + mat->n_phases);
    for (int k = 0; k < 3; ++k) ctx->g[k] = mat->g[k];
    std::vector<int32_t> iop(EFT_MAX_PHASE + EFT_MAX_SOLID, -1);
    std::vector<double> tab(5 * EFT_MAX_PHASE + EFT_MAX_SOLID, 0.0);
    int nbg = 0;
    for (int ph = 0; ph < ctx->n_phase; ++ph) {
        const eft_phase &P = ctx->phase[ph];
        if (!(P.rho > 0.0) || P.mu < 0.0 || P.mu_L < 0.0 || (P.kind != 0 && P.kind != 1)) {
            ctx->err = "phase needs rho > 0, mu >= 0, mu_L >= 0, kind 0/1";
            return EFT_EINVAL;
        }
        tab[0 * EFT_MAX_PHASE + ph] = P.kind;
        tab[1 * EFT_MAX_PHASE + ph] = P.transported ? 1.0 : 0.0;
        tab[2 * EFT_MAX_PHASE + ph] = P.rho;
        tab[3 * EFT_MAX_PHASE + ph] = P.mu;
        tab[4 * EFT_MAX_PHASE + ph] = P.mu_L;
        if (P.transported) {
            iop[ph] = ctx->n_ind++;
            ctx->ind_phase.push_back(ph);
        } else {
            ++nbg;
            ctx->bg = ph;
            if (P.kind == 1) {
                ctx->err = "a solid phase must carry its own order parameter";
                return EFT_EINVAL;
            }
        }
    }
    if (nbg > 1 || ctx->n_ind > EFT_MAX_IND) {
        ctx->err = "at most one background phase and 64 order parameters";
        return EFT_EINVAL;
    }
    for (int ph = 0; ph < ctx->n_phase; ++ph)
        if (ctx->phase[ph].kind == 1) {
            const int s = ctx->n_s++;
            ctx->solid_phase.push_back(ph);
            ctx->solid_ind.push_back(iop[ph]);
            iop[EFT_MAX_PHASE + s] = iop[ph];
            tab[5 * EFT_MAX_PHASE + s] = ctx->phase[ph].mu_L;
        }
    // mesh checks and the node graph (host)
    const int32_t *conn = mesh->conn;
    for (int64_t t = 0; t < E * nn; ++t)
        if (conn[t] < 0 || conn[t] >= N) {
            ctx->err = "connectivity index out of range";
            return EFT_EINVAL;
        }
    for (int64_t e = 0; e < E; ++e) {
        double M[3][3] = {{0}};
        for (int i = 0; i < d; ++i)
            for (int k = 0; k < d; ++k) M[i][k] = mesh->xyz[(int64_t)conn[e * nn + k + 1] * d + i] - mesh->xyz[(int64_t)conn[e * nn] * d + i];
        const double det = d == 2 ? M[0][0] * M[1][1] - M[0][1] * M[1][0]
                                  : M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                                        M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                                        M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
        if (!(det > 0.0)) {
            ctx->err = "element " + std::to_string(e) + " has non-positive orientation";
            return EFT_EINVAL;
        }
    }
    std::vector<int32_t> rowptr, col, diag, epos, iptr, ient;
    std::vector<uint32_t> islot;
    EFT_TRY(eft_build_graph(N, E, nn, conn, rowptr, col, diag, epos, iptr, ient, islot, ctx->maxc, ctx->rpb, ctx->rpb_ns,
                            ctx->err));
    const int64_t nnzb = (int64_t)col.size();
    // band grid: cells of band_cell mesh cells, element -> cell of its centroid
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int i = 0; i < d; ++i) {
        lo[i] = 1e300;
        hi[i] = -1e300;
    }
    for (int64_t p = 0; p < N; ++p)
        for (int i = 0; i < d; ++i) {
            lo[i] = std::min(lo[i], mesh->xyz[p * d + i]);
            hi[i] = std::max(hi[i], mesh->xyz[p * d + i]);
        }
    for (int i = 0; i < d; ++i) {
        ctx->bb_lo[i] = lo[i];
        ctx->bb_hi[i] = hi[i];
    }
    double hg[3] = {1, 1, 1};
    for (int i = 0; i < 3; ++i) ctx->ng[i] = 1;
    for (int i = 0; i < d; ++i) {
        ctx->ng[i] = (mesh->grid[i] + par->band_cell - 1) / par->band_cell;
        hg[i] = par->band_cell * (hi[i] - lo[i]) / mesh->grid[i];
    }
    std::vector<int32_t> cell_of(E);
    for (int64_t e = 0; e < E; ++e) {
        int ci[3] = {0, 0, 0};
        for (int i = 0; i < d; ++i) {
            double c = 0.0;
            for (int a = 0; a < nn; ++a) c += mesh->xyz[(int64_t)conn[e * nn + a] * d + i];
            c /= nn;
            const int k = (int)std::floor((c - lo[i]) / hg[i]);
            ci[i] = std::min(std::max(k, 0), ctx->ng[i] - 1);
        }
        cell_of[e] = ci[0] + ctx->ng[0] * (ci[1] + ctx->ng[1] * ci[2]);
    }
    const int64_t ncell = (int64_t)ctx->ng[0] * ctx->ng[1] * ctx->ng[2];
    ctx->h_min = 1e300;
    for (int i = 0; i < d; ++i) ctx->h_min = std::min(ctx->h_min, (hi[i] - lo[i]) / mesh->grid[i]);
    // the most nodes per element over the grid cells: a band of cells holds
    // at most this many nodes per band element (sizes the band storage)
    {
        std::vector<int64_t> ecount(ncell, 0), ncount(ncell, 0);
        constexpr int SL = 8;
        std::vector<int32_t> slot((size_t)N * SL, -1);
        bool over = false;
        for (int64_t e = 0; e < E; ++e) {
            const int32_t c = cell_of[e];
            ecount[c] += 1;
            for (int a = 0; a < nn && !over; ++a) {
                int32_t *sl = &slot[(size_t)conn[e * nn + a] * SL];
                int k = 0;
                while (k < SL && sl[k] >= 0 && sl[k] != c) ++k;
                if (k == SL) over = true;
                else if (sl[k] < 0) {
                    sl[k] = c;
                    ncount[c] += 1;
                }
            }
        }
        double r = 0.0;
        for (int64_t c = 0; c < ncell; ++c)
            if (ecount[c] > 0) r = std::max(r, (double)ncount[c] / (double)ecount[c]);
        ctx->band_node_ratio = over ? (double)nn : std::max(r, 1e-3);
    }
    // device copies
    EFT_TRY(upload(ctx, &ctx->xyz, mesh->xyz, N * d));
    EFT_TRY(upload(ctx, &ctx->conn, conn, E * nn));
    EFT_TRY(upload(ctx, &ctx->epos, epos.data(), E * nn * nn));
    EFT_TRY(upload(ctx, &ctx->iptr, iptr.data(), N + 1));
    EFT_TRY(upload(ctx, &ctx->ient, ient.data(), E * nn));
    EFT_TRY(upload(ctx, &ctx->islot, islot.data(), E * nn));
    {
        std::vector<int32_t> wnptr, wnode;
        std::vector<uint32_t> iloc;
        if (eft_ns_stage_build(N, nn, conn, iptr, ient, ctx->rpb_ns, wnptr, wnode, iloc, ctx->maxnl, ctx->maxpw)) {
            EFT_TRY(upload(ctx, &ctx->wnptr, wnptr.data(), (int64_t)wnptr.size()));
            EFT_TRY(upload(ctx, &ctx->wnode, wnode.data(), (int64_t)wnode.size()));
            EFT_TRY(upload(ctx, &ctx->iloc, iloc.data(), (int64_t)iloc.size()));
        }
    }
    EFT_TRY(upload(ctx, &ctx->cell_of, cell_of.data(), E));
    ctx->n_dir = mesh->n_dir;
    if (mesh->n_dir > 0) {
        for (int64_t t = 0; t < mesh->n_dir; ++t)
            if (mesh->dir_node[t] < 0 || mesh->dir_node[t] >= N) {
                ctx->err = "Dirichlet node out of range";
                return EFT_EINVAL;
            }
        EFT_TRY(upload(ctx, &ctx->dir_node, mesh->dir_node, mesh->n_dir));
        EFT_TRY(upload(ctx, &ctx->dir_mask, mesh->dir_mask, mesh->n_dir));
        EFT_TRY(upload(ctx, &ctx->dir_val, mesh->dir_val, mesh->n_dir * bs));
    }
    EFT_TRY(upload(ctx, &ctx->phase_tab, tab.data(), (int64_t)tab.size()));
    EFT_TRY(upload(ctx, &ctx->ind_of_phase, iop.data(), (int64_t)iop.size()));
    ctx->J.bs = bs;
    ctx->J.n = N;
    ctx->J.nnzb = nnzb;
    EFT_TRY(upload(ctx, &ctx->J.rowptr, rowptr.data(), N + 1));
    EFT_TRY(upload(ctx, &ctx->J.col, col.data(), nnzb));
    {
        // the multigrid's narrow-value sweeps read the pattern in stencil
        // form when it has one (one offset per lane of a row's segment)
        std::vector<int32_t> soff;
        std::vector<uint16_t> sm;
        if (eft_stencil_form(N, rowptr, col, bs == 4 ? 16 : 8, soff, sm)) {
            EFT_TRY(upload(ctx, &ctx->J.stn_mask, sm.data(), N));
            EFT_TRY(upload(ctx, &ctx->J.stn_off, soff.data(), (int64_t)soff.size()));
        }
    }
    EFT_TRY(upload(ctx, &ctx->J.diag, diag.data(), N));
    EFT_TRY(alloc_jacobian_values(ctx));
    // Dirichlet bits of every node, and the free bits the assembly writes
    // unit rows by
    std::vector<uint8_t> dm(N, 0), fm(N);
    for (int64_t t = 0; t < mesh->n_dir; ++t) dm[mesh->dir_node[t]] |= mesh->dir_mask[t];
    for (int64_t p = 0; p < N; ++p) fm[p] = (uint8_t)(~dm[p] & ((1 << bs) - 1));
    EFT_TRY(upload(ctx, &ctx->fmask0, fm.data(), N));
    // geometric multigrid needs the structured Kuhn layout of a box
    ctx->structured = structured_kuhn(d, mesh->grid, N, E, mesh->xyz, conn);
    if (ctx->structured) {
        EFT_TRY(eft_mg_create(ctx, mesh->grid, dm));
        EFT_TRY(eft_mg_reserve(ctx));
        EFT_TRY(eft_ilu_reserve(ctx));
    }
    const int mx = std::max(bs, nv);
    EFT_TRY(dalloc(ctx, &ctx->va, N * d));
    EFT_TRY(dalloc(ctx, &ctx->acc, N * d));
    EFT_TRY(dalloc(ctx, &ctx->rho, N));
    EFT_TRY(dalloc(ctx, &ctx->mu, N));
    EFT_TRY(dalloc(ctx, &ctx->smask, N));
    {
        std::vector<int32_t> si(std::max(ctx->n_s, 1), 0);
        for (int s = 0; s < ctx->n_s; ++s) si[s] = ctx->solid_ind[s];
        EFT_TRY(upload(ctx, &ctx->solid_ind_d, si.data(), (int64_t)si.size()));
    }
    EFT_TRY(dalloc(ctx, &ctx->R, N * mx));
    EFT_TRY(dalloc(ctx, &ctx->dx, N * mx));
    EFT_TRY(dalloc(ctx, &ctx->l_vp, N * bs));
    EFT_TRY(dalloc(ctx, &ctx->l_vdot, N * d));
    EFT_TRY(dalloc(ctx, &ctx->l_phi, N * std::max(ctx->n_ind, 1)));
    EFT_TRY(dalloc(ctx, &ctx->l_phidot, N * std::max(ctx->n_ind, 1)));
    EFT_TRY(dalloc(ctx, &ctx->l_B, N * nv * std::max(ctx->n_s, 1)));
    EFT_TRY(dalloc(ctx, &ctx->l_Bdot, N * nv * std::max(ctx->n_s, 1)));
    EFT_TRY(dalloc(ctx, &ctx->seed, ncell));
    EFT_TRY(dalloc(ctx, &ctx->active, ncell));
    EFT_TRY(dalloc(ctx, &ctx->nin, N));
    EFT_TRY(dalloc(ctx, &ctx->nout, N));
    EFT_TRY(dalloc(ctx, &ctx->ein, E));
    EFT_TRY(dalloc(ctx, &ctx->g2b, N));
    EFT_TRY(dalloc(ctx, &ctx->gpos2b, nnzb));
    ctx->nred = (int32_t)(2 * ((N + 255) / 256) + 2 * ((E + 255) / 256) + 4096);
    EFT_TRY(dalloc(ctx, &ctx->red, ctx->nred));
    EFT_TRY(dalloc(ctx, &ctx->dscal, 64));
    EFT_TRY(dalloc(ctx, &ctx->tsc, 1024));
    if (hipHostMalloc((void **)&ctx->htsc, sizeof(double) * 1024, hipHostMallocDefault) != hipSuccess) {
        ctx->err = "out of pinned host memory";
        return EFT_ENOMEM;
    }
    if (hipHostMalloc((void **)&ctx->hscal, sizeof(double) * 64, hipHostMallocDefault) != hipSuccess) {
        ctx->err = "pinned host allocation failed";
        return EFT_ENOMEM;
    }
    // Krylov workspace for the largest system: momentum block or a full-size band
    EFT_TRY(eft_krylov_reserve(ctx, N, mx, par->restart));
    EFT_TRY(eft_scratch_attach(ctx));
    EFT_TRY(eft_band_reserve(ctx));
    EFT_HIP(hipDeviceSynchronize());
    return EFT_OK;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// --------------------------------------------------------------- the ABI --

// ------------------------------------------------------- kernel timing ----

int64_t eft_kt_begin(eft_ctx *ctx, int role)
{
    KTimer &T = ctx->kt;
    if (!((T.mask >> role) & 1u)) return -1;
    const size_t need = 2 * (size_t)(T.pend + 1);
    while (T.ev.size() < need) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        T.ev.push_back(e);
    }
    if (hipEventRecord(T.ev[2 * T.pend], ctx->stream) != hipSuccess) return -1;
    return T.pend;
}

void eft_kt_end(eft_ctx *ctx, int64_t slot, double bytes, int role)
{
    KTimer &T = ctx->kt;
    if (slot < 0 || slot != T.pend) return;
    if (hipEventRecord(T.ev[2 * slot + 1], ctx->stream) != hipSuccess) return;
    T.pbytes.resize(T.pend + 1);
    T.ptag.resize(T.pend + 1);
    T.prole.resize(T.pend + 1);
    T.pbytes[slot] = bytes;
    T.ptag[slot] = T.tag;
    T.prole[slot] = role;
    T.pend += 1;
}

void eft_kt_void_from(eft_ctx *ctx, int tag0)
{
    KTimer &T = ctx->kt;
    for (int64_t i = 0; i < T.pend; ++i)
        if (T.ptag[i] >= tag0) T.pbytes[i] = -1.0;
}

eft_status eft_kt_harvest(eft_ctx *ctx)
{
    KTimer &T = ctx->kt;
    if (T.pend == 0) return EFT_OK;
    EFT_HIP(hipEventSynchronize(T.ev[2 * T.pend - 1]));
    for (int64_t i = 0; i < T.pend; ++i) {
        float ms = 0.0f;
        EFT_HIP(hipEventElapsedTime(&ms, T.ev[2 * i], T.ev[2 * i + 1]));
        const int r = T.prole[i];
        T.seconds[r] += 1e-3 * ms;
        T.launches[r] += 1;
        if (T.pbytes[i] >= 0.0) {
            T.active[r] += 1;
            T.bytes[r] += T.pbytes[i];
        }
    }
    T.pend = 0;
    return EFT_OK;
}

extern "C" {

eft_status eft_create(const eft_mesh *mesh, const eft_materials *mat, const eft_params *par, void *hip_stream,
                      eft_ctx **out)
{
    if (!out || !mesh || !mat || !par) return EFT_EINVAL;
    *out = nullptr;
    eft_ctx *ctx = new (std::nothrow) eft_ctx();
    if (!ctx) return EFT_ENOMEM;
    ctx->stream = (hipStream_t)hip_stream;
    eft_status st = create_impl(ctx, mesh, mat, par);
    if (st != EFT_OK) {
        // keep the message: a context that failed is returned for eft_last_error
        free_all(ctx);
        eft_ctx *dead = new (std::nothrow) eft_ctx();
        if (dead) dead->err = ctx->err;
        delete ctx;
        *out = dead;
        return st;
    }
    *out = ctx;
    return EFT_OK;
}

eft_status eft_destroy(eft_ctx *ctx)
{
    if (!ctx) return EFT_EINVAL;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    free_all(ctx);
    delete ctx;
    return EFT_OK;
}

const char *eft_last_error(const eft_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : "null context";
}

eft_status eft_set_params(eft_ctx *ctx, const eft_params *par)
{
    if (!ctx || !par) return EFT_EINVAL;
    EFT_TRY(check_params(ctx, par));
    const bool prec = par->precision != ctx->par.precision;
    const bool grid = par->band_cell != ctx->par.band_cell;
    if (grid) {
        ctx->err = "band_cell is fixed at creation";
        return EFT_EINVAL;
    }
    if (par->restart > ctx->kw.cap_m) EFT_TRY(eft_krylov_reserve(ctx, ctx->N, std::max(ctx->bs, ctx->nv), par->restart));
    const bool rebands = par->band_reserve != ctx->par.band_reserve || ((par->band_flat < 0.0) != (ctx->par.band_flat < 0.0));
    ctx->par = *par;
    if (prec) {
        EFT_TRY(alloc_jacobian_values(ctx));
        ctx->mg_valid = false;
    }
    EFT_TRY(eft_mg_reserve(ctx));
    EFT_TRY(eft_ilu_reserve(ctx));
    if (rebands) EFT_TRY(eft_band_reserve(ctx));
    else if (par->restart > ctx->kw.cap_m) EFT_TRY(eft_krylov_reserve(ctx, ctx->bp.cap_n, ctx->nv, par->restart));
    ctx->bands_valid = false;
    return EFT_OK;
}

eft_status eft_ns_matrix(eft_ctx *ctx, eft_matrix **out)
{
    if (!ctx || !out) return EFT_EINVAL;
    *out = &ctx->J;
    return EFT_OK;
}

eft_status eft_matrix_shape(const eft_matrix *A, int64_t *n_rows, int64_t *nnzb, int32_t *bs)
{
    if (!A) return EFT_EINVAL;
    if (n_rows) *n_rows = A->n;
    if (nnzb) *nnzb = A->nnzb;
    if (bs) *bs = A->bs;
    return EFT_OK;
}

eft_status eft_matrix_export(eft_ctx *ctx, const eft_matrix *A, int32_t *rowptr, int32_t *col, double *val)
{
    if (!ctx || !A) return EFT_EINVAL;
    if (rowptr) EFT_HIP(hipMemcpyAsync(rowptr, A->rowptr, sizeof(int32_t) * (A->n + 1), hipMemcpyDeviceToDevice, ctx->stream));
    if (col) EFT_HIP(hipMemcpyAsync(col, A->col, sizeof(int32_t) * A->nnzb, hipMemcpyDeviceToDevice, ctx->stream));
    const int64_t nv = A->nnzb * A->bs * A->bs;
    if (val) {
        if (A->fp32) {
            hipLaunchKernelGGL(k_widen, dim3(sgrid(nv)), dim3(256), 0, ctx->stream, A->val32, val, nv);
            EFT_HIP(hipGetLastError());
        } else {
            EFT_HIP(hipMemcpyAsync(val, A->val, sizeof(double) * nv, hipMemcpyDeviceToDevice, ctx->stream));
        }
    }
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    return EFT_OK;
}

__global__ void k_narrow(const double *a, float *b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

eft_status eft_matrix_import(eft_ctx *ctx, eft_matrix *A, const double *val)
{
    if (!ctx || !A || !val) return EFT_EINVAL;
    if (A != &ctx->J) {
        ctx->err = "only the context's momentum matrix can be imported";
        return EFT_EINVAL;
    }
    const int64_t nv = A->nnzb * A->bs * A->bs;
    if (A->fp32) {
        hipLaunchKernelGGL(k_narrow, dim3(sgrid(nv)), dim3(256), 0, ctx->stream, val, A->val32, nv);
        EFT_HIP(hipGetLastError());
    } else {
        EFT_HIP(hipMemcpyAsync(A->val, val, sizeof(double) * nv, hipMemcpyDeviceToDevice, ctx->stream));
    }
    ctx->mg_f32_fresh = false;   // the multigrid hierarchy belongs to the assembled Jacobian
    ctx->mg_valid = false;
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    return EFT_OK;
}

eft_status eft_assemble(eft_ctx *ctx, const eft_state *lvl, const eft_iterate *it, double *R, eft_matrix *J)
{
    if (!ctx || !lvl || !it || !R || !lvl->vp || !lvl->vdot || !it->vp) return EFT_EINVAL;
    if ((ctx->n_ind > 0 && (!lvl->phi || !it->phi)) || (ctx->n_s > 0 && (!lvl->B || !it->B))) return EFT_EINVAL;
    if (J && J != &ctx->J) {
        ctx->err = "J must be the context's momentum matrix";
        return EFT_EINVAL;
    }
    EFT_TRY(eft_props(ctx, lvl, it));
    return eft_ns_kernels(ctx, it, R, J);
}

eft_status eft_spmv(eft_ctx *ctx, const eft_matrix *A, const double *x, double *y)
{
    if (!ctx || !A || !x || !y) return EFT_EINVAL;
    return eft_spmv_dev(ctx, A, x, y);
}

eft_status eft_fgmres(eft_ctx *ctx, const eft_matrix *A, const double *b, double *x, eft_solve_info *info)
{
    if (!ctx || !A || !b || !x) return EFT_EINVAL;
    return eft_fgmres_dev(ctx, A, b, x, info);
}

eft_status eft_bands_build(eft_ctx *ctx, const eft_state *lvl)
{
    if (!ctx || !lvl) return EFT_EINVAL;
    if (ctx->n_ind == 0) {
        ctx->bands_valid = true;
        return EFT_OK;
    }
    if (!lvl->phi) return EFT_EINVAL;
    return eft_bands_build_dev(ctx, lvl->phi);
}

eft_status eft_band_export(eft_ctx *ctx, int32_t k, uint8_t *band_elem, uint8_t *free_node)
{
    if (!ctx || k < 0 || k >= ctx->n_ind || !ctx->bands_valid) return EFT_EINVAL;
    const Band &B = ctx->band[k];
    if (band_elem) {
        EFT_TRY(eft_fill_u8(ctx, band_elem, ctx->E));
        if (B.ne > 0) hipLaunchKernelGGL(k_scatter_one, dim3(eft_grid(B.ne, 256)), dim3(256), 0, ctx->stream, B.ne, B.elem, band_elem);
    }
    if (free_node) {
        EFT_TRY(eft_fill_u8(ctx, free_node, ctx->N));
        if (B.n > 0)
            hipLaunchKernelGGL(k_scatter_u8, dim3(eft_grid(B.n, 256)), dim3(256), 0, ctx->stream, B.n, B.node, B.fre,
                               free_node);
    }
    EFT_HIP(hipGetLastError());
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    return EFT_OK;
}

eft_status eft_band_system(eft_ctx *ctx, const eft_state *lvl, const eft_iterate *it, int32_t kind, int32_t index,
                           int64_t *n, int64_t *nnz, int32_t *node, int32_t *rowptr, int32_t *col, double *R,
                           double *J, double *gamma_beta)
{
    if (!ctx || !lvl || !it) return EFT_EINVAL;
    if (ctx->n_ind == 0 || !lvl->phi || !lvl->phidot || !it->phi || (kind == 1 && (!lvl->B || !lvl->Bdot || !it->B)))
        return EFT_EINVAL;
    return eft_band_system_dev(ctx, lvl, it, kind, index, n, nnz, node, rowptr, col, R, J, gamma_beta);
}

eft_status eft_transport_solids(eft_ctx *ctx, const eft_state *lvl, eft_iterate *it, eft_transport_info *info)
{
    if (!ctx || !lvl || !it) return EFT_EINVAL;
    if (ctx->n_ind == 0) {
        if (info) *info = eft_transport_info{};
        return EFT_OK;
    }
    if (!lvl->phi || !lvl->phidot || !it->phi || (ctx->n_s > 0 && (!lvl->B || !lvl->Bdot || !it->B))) return EFT_EINVAL;
    eft_status st = eft_transport_dev(ctx, lvl, it, info);
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    return st;
}

eft_status eft_time_kernel(eft_ctx *ctx, int32_t role_mask)
{
    if (!ctx) return EFT_EINVAL;
    const uint32_t ok = (1u << EFT_KT_SMOOTH) | (1u << EFT_KT_SPMV) | (1u << EFT_KT_ASSEMBLE);
    if ((uint32_t)role_mask & ~ok) {
        ctx->err = "eft_time_kernel: role_mask may only set bits 1 (smoother), 2 (SpMV), 3 (assembly)";
        return EFT_EINVAL;
    }
    EFT_TRY(eft_kt_harvest(ctx));
    KTimer &T = ctx->kt;
    T.mask = (uint32_t)role_mask;
    T.tag = -1;
    for (int r = 0; r < EFT_KT_NROLE; ++r) {
        T.launches[r] = T.active[r] = 0;
        T.seconds[r] = T.bytes[r] = 0.0;
    }
    return EFT_OK;
}

eft_status eft_kernel_time_read(eft_ctx *ctx, int32_t role, eft_kernel_time *out)
{
    if (!ctx || !out) return EFT_EINVAL;
    if (role < 1 || role >= EFT_KT_NROLE) {
        ctx->err = "eft_kernel_time_read: role must be 1, 2 or 3";
        return EFT_EINVAL;
    }
    EFT_TRY(eft_kt_harvest(ctx));
    out->launches = ctx->kt.launches[role];
    out->active = ctx->kt.active[role];
    out->seconds = ctx->kt.seconds[role];
    out->bytes = ctx->kt.bytes[role];
    return EFT_OK;
}

eft_status eft_step(eft_ctx *ctx, eft_state *st, double dt, eft_step_info *info)
{
    if (!ctx || !st || !st->vp || !st->vdot) return EFT_EINVAL;
    if ((ctx->n_ind > 0 && (!st->phi || !st->phidot)) || (ctx->n_s > 0 && (!st->B || !st->Bdot))) return EFT_EINVAL;
    if (dt > 0.0) ctx->par.dt = dt;
    // the nonlinear iteration counter reads 0 again however the step ends
    struct NlReset {
        eft_ctx *c;
        ~NlReset() { c->nl_k = 0; }
    } nl_reset{ctx};
    const int64_t N = ctx->N;
    const int d = ctx->dim, bs = ctx->bs, nv = ctx->nv;
    const int64_t nvp = N * bs, nphi = N * ctx->n_ind, nB = N * nv * ctx->n_s;
    GA ga = ga_of(ctx->par.rho_inf, ctx->par.dt);
    eft_step_info inf{};
    inf.n_blocks = 1 + ctx->n_ind + ctx->n_s;
    double t0 = now_s();
    // level-n snapshot; the caller's arrays hold the iterate from here on
    EFT_HIP(hipMemcpyAsync(ctx->l_vp, st->vp, sizeof(double) * nvp, hipMemcpyDeviceToDevice, ctx->stream));
    EFT_HIP(hipMemcpyAsync(ctx->l_vdot, st->vdot, sizeof(double) * N * d, hipMemcpyDeviceToDevice, ctx->stream));
    if (nphi) {
        EFT_HIP(hipMemcpyAsync(ctx->l_phi, st->phi, sizeof(double) * nphi, hipMemcpyDeviceToDevice, ctx->stream));
        EFT_HIP(hipMemcpyAsync(ctx->l_phidot, st->phidot, sizeof(double) * nphi, hipMemcpyDeviceToDevice, ctx->stream));
    }
    if (nB) {
        EFT_HIP(hipMemcpyAsync(ctx->l_B, st->B, sizeof(double) * nB, hipMemcpyDeviceToDevice, ctx->stream));
        EFT_HIP(hipMemcpyAsync(ctx->l_Bdot, st->Bdot, sizeof(double) * nB, hipMemcpyDeviceToDevice, ctx->stream));
    }
    eft_state lvl{ctx->l_vp, ctx->l_vdot, ctx->l_phi, ctx->l_phidot, ctx->l_B, ctx->l_Bdot, st->t, st->step};
    eft_iterate it{st->vp, st->phi, st->B};
    // bands of phi^n (within the storage reserved at creation; the state is
    // untouched if they do not fit)
    if (ctx->n_ind > 0) EFT_TRY(eft_bands_build_dev(ctx, ctx->l_phi));
    // predictor: same values (rates follow from the update formula), boundary data
    if (ctx->n_dir > 0) {
        hipLaunchKernelGGL(k_apply_dirichlet, dim3(eft_grid(ctx->n_dir, 128)), dim3(128), 0, ctx->stream, ctx->n_dir,
                           ctx->dir_node, ctx->dir_mask, ctx->dir_val, bs, st->vp);
        EFT_HIP(hipGetLastError());
    }
    auto restore = [&]() {
        (void)hipMemcpyAsync(st->vp, ctx->l_vp, sizeof(double) * nvp, hipMemcpyDeviceToDevice, ctx->stream);
        if (nphi) (void)hipMemcpyAsync(st->phi, ctx->l_phi, sizeof(double) * nphi, hipMemcpyDeviceToDevice, ctx->stream);
        if (nB) (void)hipMemcpyAsync(st->B, ctx->l_B, sizeof(double) * nB, hipMemcpyDeviceToDevice, ctx->stream);
        (void)hipStreamSynchronize(ctx->stream);
    };
    const int nl_lim = ctx->par.nl_fixed > 0 ? ctx->par.nl_fixed : ctx->par.nl_max;
    int k = 0;
    bool conv = false;
    for (k = 1; k <= nl_lim; ++k) {
        double ta = now_s();
        ctx->nl_k = k;
        EFT_TRY(eft_props(ctx, &lvl, &it));
        EFT_TRY(eft_ns_kernels(ctx, &it, ctx->R, &ctx->J));
        hipLaunchKernelGGL(k_neg, dim3(sgrid(nvp)), dim3(256), 0, ctx->stream, ctx->R, nvp);
        EFT_HIP(hipGetLastError());
        EFT_HIP(hipStreamSynchronize(ctx->stream));
        double tb = now_s();
        inf.t_assemble += tb - ta;
        eft_solve_info si{};
        eft_status ls = eft_fgmres_dev(ctx, &ctx->J, ctx->R, ctx->dx, &si);
        inf.lin_iters_total += si.iters;
        inf.lin_iters_block[0] += si.iters;
        if (ls == EFT_ENAN || ls == EFT_EDEVICE || ls == EFT_ENOMEM || ls == EFT_EBREAKDOWN || ls == EFT_EINVAL) {
            restore();
            return ls;
        }
        hipLaunchKernelGGL(k_add, dim3(sgrid(nvp)), dim3(256), 0, ctx->stream, st->vp, ctx->dx, nvp);
        EFT_HIP(hipGetLastError());
        double dn, xn;
        EFT_TRY(eft_norm2(ctx, ctx->dx, nvp, &dn));
        EFT_TRY(eft_norm2(ctx, st->vp, nvp, &xn));
        inf.block_ratio[0] = dn / std::max(xn, 1e-300);
        double tc = now_s();
        inf.t_solve += tc - tb;
        if (!std::isfinite(inf.block_ratio[0])) {
            restore();
            ctx->err = "NaN in the momentum/mass update";
            return EFT_ENAN;
        }
        if (ctx->n_ind > 0) {
            eft_transport_info ti{};
            eft_status ts = eft_transport_dev(ctx, &lvl, &it, &ti);
            if (ts != EFT_OK && ts != EFT_ENOTCONV) {
                restore();
                return ts;
            }
            inf.lin_iters_total += ti.ac_iters + ti.b_iters;
            for (int b = 0; b < ctx->n_ind + ctx->n_s; ++b) {
                inf.block_ratio[1 + b] = ti.ratio[b];
                inf.lin_iters_block[1 + b] += ti.lin_iters[b];
                if (!std::isfinite(ti.ratio[b])) {
                    restore();
                    ctx->err = "NaN in the transport update";
                    return EFT_ENAN;
                }
            }
        }
        inf.t_transport += now_s() - tc;
        if (ctx->par.nl_fixed <= 0) {
            bool ok = true;
            for (int b = 0; b < inf.n_blocks; ++b) ok &= inf.block_ratio[b] < ctx->par.nl_rtol;
            if (ok) {
                conv = true;
                break;
            }
        }
    }
    if (ctx->par.nl_fixed > 0) {
        conv = true;
        k = ctx->par.nl_fixed;
    } else if (!conv) {
        k = ctx->par.nl_max;
    }
    // corrector: rates at n+1
    hipLaunchKernelGGL(k_rates, dim3(eft_grid(N * d, 256)), dim3(256), 0, ctx->stream, N, d, bs, d, ctx->l_vp,
                       ctx->l_vdot, st->vp, st->vdot, ga.dt, ga.vs);
    if (nphi)
        hipLaunchKernelGGL(k_rates, dim3(eft_grid(nphi, 256)), dim3(256), 0, ctx->stream, nphi, 1, 1, 1, ctx->l_phi,
                           ctx->l_phidot, st->phi, st->phidot, ga.dt, ga.vs);
    if (nB)
        hipLaunchKernelGGL(k_rates, dim3(eft_grid(nB, 256)), dim3(256), 0, ctx->stream, nB, 1, 1, 1, ctx->l_B,
                           ctx->l_Bdot, st->B, st->Bdot, ga.dt, ga.vs);
    EFT_HIP(hipGetLastError());
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    st->t += ctx->par.dt;
    st->step += 1;
    inf.nl_iters = k;
    inf.converged = conv ? 1 : 0;
    (void)t0;
    if (info) *info = inf;
    return EFT_OK;
}

}  // extern "C"
