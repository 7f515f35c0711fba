// Element assembly of the unified momentum/mass system, eq. (PG_NS).
//
// Three kernels:
//   k_props       per node: generalized-alpha level values (Sec. 2.1.2) and
//                 phase-interpolated rho, mu (Sec. 2.1.1), solid fractions and
//                 B at n+alpha;
//   k_ns_fluid    per element: Galerkin + SUPG/PSPG/LSIC residual and tangent
//                 of the Newtonian part (tau_m, tau_c formula), scattered with
//                 hardware FP64 atomics into the residual and the BSR Jacobian;
//   k_ns_elastic  per element touched by a solid: the left-Cauchy-Green stress
//                 mu_L (B - I) in the residual and its tangent through
//                 dB/dv of eq. (Bext) / Appendix B.
// The tangent is factored: per element the quadrature sums that multiply each
// node-pair block are formed once (about 10 scalars per pair), so a 4x4 block
// costs a few dozen flops instead of a loop over quadrature points.
#include "dev_common.h"
#include "eft_internal.h"

// ------------------------------------------------------------------ props --

struct PropsArgs {
    int64_t N;
    int n_phase, n_ind, n_s;
    double alpha, alpha_m, vs, dt;
    const double *tab;          // [5][EFT_MAX_PHASE]
    const int32_t *ind_of_phase;
    const int32_t *solid_ind;   // [n_s] indicator of each solid
    const double *l_vp, *l_vdot, *it_vp;
    const double *l_phi, *it_phi;
    const double *l_B, *it_B;
    double *va, *acc, *rho, *mu, *as, *Ba;
};

template <int D>
__global__ __launch_bounds__(256) void k_props(PropsArgs a)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.N) return;
    constexpr int BS = D + 1, NVv = NV<D>::v;
    for (int i = 0; i < D; ++i) {
        double xn = a.l_vp[p * BS + i], xd = a.l_vdot[p * D + i], x1 = a.it_vp[p * BS + i];
        double xd1 = xd + (x1 - xn - a.dt * xd) / (a.vs * a.dt);
        a.acc[p * D + i] = xd + a.alpha_m * (xd1 - xd);
        a.va[p * D + i] = xn + a.alpha * (x1 - xn);
    }
    const double *kind = a.tab, *tr = a.tab + EFT_MAX_PHASE, *rh = a.tab + 2 * EFT_MAX_PHASE,
                 *vi = a.tab + 3 * EFT_MAX_PHASE;
    (void)kind;
    double sum = 0.0, r = 0.0, m = 0.0;
    int bg = -1;
    for (int ph = 0; ph < a.n_phase; ++ph) {
        if (tr[ph] == 0.0) {
            bg = ph;
            continue;
        }
        const int k = a.ind_of_phase[ph];
        const double fn = a.l_phi[(int64_t)k * a.N + p], f1 = a.it_phi[(int64_t)k * a.N + p];
        const double fa = fn + a.alpha * (f1 - fn);
        const double al = fmin(fmax(0.5 * (1.0 + fa), 0.0), 1.0);
        sum += al;
        r += al * rh[ph];
        m += al * vi[ph];
    }
    if (bg >= 0) {
        const double al = sum < 1.0 ? 1.0 - sum : 0.0;
        r += al * rh[bg];
        m += al * vi[bg];
    }
    a.rho[p] = r;
    a.mu[p] = m;
    for (int s = 0; s < a.n_s; ++s) {
        const int k = a.solid_ind[s];
        const double fn = a.l_phi[(int64_t)k * a.N + p], f1 = a.it_phi[(int64_t)k * a.N + p];
        const double fa = fn + a.alpha * (f1 - fn);
        a.as[(int64_t)s * a.N + p] = fmin(fmax(0.5 * (1.0 + fa), 0.0), 1.0);
        for (int c = 0; c < NVv; ++c) {
            const int64_t o = ((int64_t)s * a.N + p) * NVv + c;
            a.Ba[o] = a.l_B[o] + a.alpha * (a.it_B[o] - a.l_B[o]);
        }
    }
}

// ------------------------------------------------------------ fluid part --

struct NSArgs {
    int64_t E;
    const int32_t *conn, *epos;
    const double *xyz, *va, *acc, *vp, *rho, *mu;
    double ct, alpha, dt, C_I, g0, g1, g2;
    double *R;
};

template <typename T> __device__ __forceinline__ void atomic_add(T *p, double v);
template <> __device__ __forceinline__ void atomic_add<double>(double *p, double v) { unsafeAtomicAdd(p, v); }
template <> __device__ __forceinline__ void atomic_add<float>(float *p, double v) { unsafeAtomicAdd(p, (float)v); }

template <int D, typename TJ>
__global__ __launch_bounds__(128) void k_ns_fluid(NSArgs a, TJ *__restrict__ Jv)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.E) return;
    constexpr int NN = D + 1, BS = D + 1, NQ = Rule<D>::NQ;
    const double gv[3] = {a.g0, a.g1, a.g2};
    int nd[NN];
    double X[NN][D], v[NN][D], ac[NN][D], p[NN], rh[NN], mu[NN];
#pragma unroll
    for (int b = 0; b < NN; ++b) {
        nd[b] = a.conn[e * NN + b];
        const int64_t n = nd[b];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            X[b][i] = a.xyz[n * D + i];
            v[b][i] = a.va[n * D + i];
            ac[b][i] = a.acc[n * D + i];
        }
        p[b] = a.vp[n * BS + D];
        rh[b] = a.rho[n];
        mu[b] = a.mu[n];
    }
    double dN[NN][D], G[D][D];
    const double vol = simplex_geom<D>(X, dN, G);
    double GG = 0.0, trG = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        trG += G[i][i];
#pragma unroll
        for (int j = 0; j < D; ++j) GG += G[i][j] * G[i][j];
    }
    double L[D][D], gp[D], divv = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            double s = 0.0;
#pragma unroll
            for (int b = 0; b < NN; ++b) s += v[b][i] * dN[b][j];
            L[i][j] = s;
        }
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < NN; ++b) s += p[b] * dN[b][i];
        gp[i] = s;
    }
#pragma unroll
    for (int i = 0; i < D; ++i) divv += L[i][i];

    const double w = vol * Rule<D>::WF;
    const double inv4dt2 = 4.0 / (a.dt * a.dt);
    double rl[NN][BS];
#pragma unroll
    for (int b = 0; b < NN; ++b)
#pragma unroll
        for (int i = 0; i < BS; ++i) rl[b][i] = 0.0;
    double W[NN][NQ], U[NN][NQ], TM[NQ];
    double muI = 0.0, Tc = 0.0, Tp = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double rq = 0.0, mq = 0.0, pq = 0.0, vq[D], aq[D];
#pragma unroll
        for (int i = 0; i < D; ++i) vq[i] = aq[i] = 0.0;
#pragma unroll
        for (int b = 0; b < NN; ++b) {
            const double Nb = shape_at<D>(q, b);
            rq += Nb * rh[b];
            mq += Nb * mu[b];
            pq += Nb * p[b];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                vq[i] += Nb * v[b][i];
                aq[i] += Nb * ac[b][i];
            }
        }
        double Lv[D], vGv = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double s = 0.0, t = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                s += L[i][j] * vq[j];
                t += G[i][j] * vq[j];
            }
            Lv[i] = s;
            vGv += vq[i] * t;
        }
        double Rm[D], body[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            body[i] = aq[i] + Lv[i] - gv[i];
            Rm[i] = rq * body[i] + gp[i];
        }
        const double nu = mq / rq;
        const double tau_m = 1.0 / sqrt(inv4dt2 + vGv + a.C_I * nu * nu * GG);
        const double tau_c = 1.0 / (trG * tau_m);
        double u[NN];
#pragma unroll
        for (int b = 0; b < NN; ++b) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) s += vq[j] * dN[b][j];
            u[b] = s;
        }
#pragma unroll
        for (int b = 0; b < NN; ++b) {
            const double Nb = shape_at<D>(q, b);
            double gR = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                double sd = -pq * dN[b][i];
#pragma unroll
                for (int j = 0; j < D; ++j) sd += mq * (L[i][j] + L[j][i]) * dN[b][j];
                rl[b][i] += w * (Nb * rq * body[i] + sd + tau_m * u[b] * Rm[i] + tau_c * rq * dN[b][i] * divv);
                gR += dN[b][i] * Rm[i];
            }
            rl[b][D] += w * (Nb * divv + (tau_m / rq) * gR);
            W[b][q] = w * rq * (Nb + tau_m * u[b]);
            U[b][q] = u[b];
        }
        TM[q] = w * tau_m;
        muI += w * mq;
        Tc += w * tau_c * rq;
        Tp += w * tau_m / rq;
    }
#pragma unroll
    for (int b = 0; b < NN; ++b)
#pragma unroll
        for (int i = 0; i < BS; ++i) unsafeAtomicAdd(a.R + (int64_t)nd[b] * BS + i, rl[b][i]);
    if (Jv == nullptr) return;

    const double al = a.alpha, ct = a.ct;
    // integral of one shape function with the rule: w * (QA + (NQ-1) QB)
    const double NI = w * (Rule<D>::QA + (NQ - 1) * Rule<D>::QB);
    const int32_t *ep = a.epos + e * NN * NN;
#pragma unroll
    for (int ia = 0; ia < NN; ++ia) {
        double Pa = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) Pa += TM[q] * U[ia][q];
        double aL[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) s += dN[ia][j] * L[j][k];
            aL[k] = s;
        }
#pragma unroll
        for (int ib = 0; ib < NN; ++ib) {
            double A = 0.0, C = 0.0, Q1 = 0.0, Q2 = 0.0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const double Nb = shape_at<D>(q, ib);
                const double lin = ct * Nb + al * U[ib][q];
                A += W[ia][q] * lin;
                C += W[ia][q] * Nb;
                Q1 += TM[q] * lin;
                Q2 += TM[q] * Nb;
            }
            C *= al;
            double gab = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) gab += dN[ia][j] * dN[ib][j];
            TJ *blk = Jv + (int64_t)ep[ia * NN + ib] * (BS * BS);
#pragma unroll
            for (int i = 0; i < D; ++i) {
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    double val = C * L[i][k] + al * muI * dN[ia][k] * dN[ib][i] + al * Tc * dN[ia][i] * dN[ib][k];
                    if (i == k) val += A + al * muI * gab;
                    atomic_add<TJ>(blk + i * BS + k, val);
                }
                atomic_add<TJ>(blk + i * BS + D, -dN[ia][i] * NI + Pa * dN[ib][i]);
            }
#pragma unroll
            for (int k = 0; k < D; ++k) atomic_add<TJ>(blk + D * BS + k, al * dN[ib][k] * NI + dN[ia][k] * Q1 + al * aL[k] * Q2);
            atomic_add<TJ>(blk + D * BS + D, Tp * gab);
        }
    }
}

// ---------------------------------------------------------- elastic part --

struct ElArgs {
    int64_t E, N;
    int n_s;
    const int32_t *conn, *epos;
    const double *xyz, *as, *Ba, *muL;   // muL [n_s] (device)
    double alpha, kappa;
    double *R;
};

template <int D, typename TJ>
__global__ __launch_bounds__(128) void k_ns_elastic(ElArgs a, TJ *__restrict__ Jv)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.E) return;
    constexpr int NN = D + 1, BS = D + 1, NQ = Rule<D>::NQ, NVv = NV<D>::v;
    int nd[NN];
#pragma unroll
    for (int b = 0; b < NN; ++b) nd[b] = a.conn[e * NN + b];
    bool geo = false;
    double dN[NN][D], G[D][D], vol = 0.0;
    for (int s = 0; s < a.n_s; ++s) {
        double asn[NN];
        bool any = false;
#pragma unroll
        for (int b = 0; b < NN; ++b) {
            asn[b] = a.as[(int64_t)s * a.N + nd[b]];
            any |= asn[b] != 0.0;
        }
        if (!any) continue;
        if (!geo) {
            double X[NN][D];
#pragma unroll
            for (int b = 0; b < NN; ++b)
#pragma unroll
                for (int i = 0; i < D; ++i) X[b][i] = a.xyz[(int64_t)nd[b] * D + i];
            vol = simplex_geom<D>(X, dN, G);
            geo = true;
        }
        const double muL = a.muL[s];
        double Bn[NN][NVv];
#pragma unroll
        for (int b = 0; b < NN; ++b)
#pragma unroll
            for (int c = 0; c < NVv; ++c) Bn[b][c] = a.Ba[((int64_t)s * a.N + nd[b]) * NVv + c];
        const double w = vol * Rule<D>::WF;
        double rl[NN][D], M2[D][D], Wb[NN];
#pragma unroll
        for (int b = 0; b < NN; ++b) {
            Wb[b] = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) rl[b][i] = 0.0;
        }
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) M2[i][j] = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double aq = 0.0, bq[NVv];
#pragma unroll
            for (int c = 0; c < NVv; ++c) bq[c] = 0.0;
#pragma unroll
            for (int b = 0; b < NN; ++b) {
                const double Nb = shape_at<D>(q, b);
                aq += Nb * asn[b];
#pragma unroll
                for (int c = 0; c < NVv; ++c) bq[c] += Nb * Bn[b][c];
            }
            double Bq[D][D];
            vfull<D>(bq, Bq);
            const double f = aq * muL;
#pragma unroll
            for (int b = 0; b < NN; ++b) {
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    double s2 = 0.0;
#pragma unroll
                    for (int j = 0; j < D; ++j) s2 += (Bq[i][j] - (i == j ? 1.0 : 0.0)) * dN[b][j];
                    rl[b][i] += w * f * s2;
                }
                Wb[b] += w * shape_at<D>(q, b) * f;
            }
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) M2[i][j] += w * f * Bq[i][j];
        }
#pragma unroll
        for (int b = 0; b < NN; ++b)
#pragma unroll
            for (int i = 0; i < D; ++i) unsafeAtomicAdd(a.R + (int64_t)nd[b] * BS + i, rl[b][i]);
        if (Jv == nullptr) continue;
        // gradient of B (constant on the element), full symmetric matrices
        double gB[D][D][D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double gk[NVv];
#pragma unroll
            for (int c = 0; c < NVv; ++c) {
                double s2 = 0.0;
#pragma unroll
                for (int b = 0; b < NN; ++b) s2 += dN[b][k] * Bn[b][c];
                gk[c] = s2;
            }
            vfull<D>(gk, gB[k]);
        }
        const double ak = a.alpha * a.kappa;
        const int32_t *ep = a.epos + e * NN * NN;
#pragma unroll
        for (int ia = 0; ia < NN; ++ia) {
            double Dk[D][D];  // Dk[i][k] = (dB/dx_k grad N_a)_i
#pragma unroll
            for (int k = 0; k < D; ++k)
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    double s2 = 0.0;
#pragma unroll
                    for (int j = 0; j < D; ++j) s2 += gB[k][i][j] * dN[ia][j];
                    Dk[i][k] = s2;
                }
#pragma unroll
            for (int ib = 0; ib < NN; ++ib) {
                double Mb[D], aMb = 0.0;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    double s2 = 0.0;
#pragma unroll
                    for (int l = 0; l < D; ++l) s2 += M2[i][l] * dN[ib][l];
                    Mb[i] = s2;
                    aMb += dN[ia][i] * s2;
                }
                TJ *blk = Jv + (int64_t)ep[ia * NN + ib] * (BS * BS);
#pragma unroll
                for (int i = 0; i < D; ++i)
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        double val = -Wb[ib] * Dk[i][k] + dN[ia][k] * Mb[i];
                        if (i == k) val += aMb;
                        atomic_add<TJ>(blk + i * BS + k, ak * val);
                    }
            }
        }
    }
}

// ------------------------------------------------------ boundary rows ----

template <typename TJ>
__global__ void k_bc_rows(int64_t n_dir, const int32_t *dir_node, const uint8_t *dir_mask, const int32_t *rowptr,
                          const int32_t *col, int BS, double *R, TJ *Jv)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_dir) return;
    const int n = dir_node[t];
    const int m = dir_mask[t];
    for (int i = 0; i < BS; ++i) {
        if (!((m >> i) & 1)) continue;
        if (R) R[(int64_t)n * BS + i] = 0.0;
        if (!Jv) continue;
        for (int k = rowptr[n]; k < rowptr[n + 1]; ++k)
            for (int j = 0; j < BS; ++j) Jv[((int64_t)k * BS + i) * BS + j] = (col[k] == n && j == i) ? TJ(1) : TJ(0);
    }
}

// ---------------------------------------------------------------- fills --

template <typename T> __global__ void k_fill(T *p, int64_t n, T v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static int fill_grid(int64_t n) { return (int)std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256)); }

eft_status eft_fill(eft_ctx *ctx, double *p, int64_t n, double v)
{
    if (n <= 0) return EFT_OK;
    hipLaunchKernelGGL(k_fill<double>, dim3(fill_grid(n)), dim3(256), 0, ctx->stream, p, n, v);
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}

eft_status eft_fill32(eft_ctx *ctx, float *p, int64_t n, float v)
{
    if (n <= 0) return EFT_OK;
    hipLaunchKernelGGL(k_fill<float>, dim3(fill_grid(n)), dim3(256), 0, ctx->stream, p, n, v);
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}

eft_status eft_fill_u8(eft_ctx *ctx, uint8_t *p, int64_t n)
{
    if (n <= 0) return EFT_OK;
    hipLaunchKernelGGL(k_fill<uint8_t>, dim3(fill_grid(n)), dim3(256), 0, ctx->stream, p, n, (uint8_t)0);
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}

// ------------------------------------------------------------- launchers --

eft_status eft_props(eft_ctx *ctx, const eft_state *lvl, const eft_iterate *it)
{
    GA ga = ga_of(ctx->par.rho_inf, ctx->par.dt);
    PropsArgs a;
    a.N = ctx->N;
    a.n_phase = ctx->n_phase;
    a.n_ind = ctx->n_ind;
    a.n_s = ctx->n_s;
    a.alpha = ga.alpha;
    a.alpha_m = ga.alpha_m;
    a.vs = ga.vs;
    a.dt = ga.dt;
    a.tab = ctx->phase_tab;
    a.ind_of_phase = ctx->ind_of_phase;
    a.solid_ind = ctx->ind_of_phase + EFT_MAX_PHASE;
    a.l_vp = lvl->vp;
    a.l_vdot = lvl->vdot;
    a.it_vp = it->vp;
    a.l_phi = lvl->phi;
    a.it_phi = it->phi;
    a.l_B = lvl->B;
    a.it_B = it->B;
    a.va = ctx->va;
    a.acc = ctx->acc;
    a.rho = ctx->rho;
    a.mu = ctx->mu;
    a.as = ctx->as;
    a.Ba = ctx->Ba;
    const int nb = eft_grid(ctx->N, 256);
    if (ctx->dim == 2)
        hipLaunchKernelGGL(k_props<2>, dim3(nb), dim3(256), 0, ctx->stream, a);
    else
        hipLaunchKernelGGL(k_props<3>, dim3(nb), dim3(256), 0, ctx->stream, a);
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}


// Residual and Jacobian of the momentum/mass block at the iterate (the
// node fields va, acc, rho, mu, as, Ba must be current, see eft_props).
// Residual and Jacobian of the momentum/mass block on one mesh level (the
// node fields of the view must be current).
eft_status eft_ns_level(eft_ctx *ctx, const MeshView &M, const double *vp, double *R, eft_matrix *J)
{
    GA ga = ga_of(ctx->par.rho_inf, ctx->par.dt);
    const int BS = ctx->bs;
    EFT_TRY(eft_fill(ctx, R, M.N * BS, 0.0));
    if (J) {
        if (J->fp32)
            EFT_TRY(eft_fill32(ctx, J->val32, J->nnzb * BS * BS, 0.0f));
        else
            EFT_TRY(eft_fill(ctx, J->val, J->nnzb * BS * BS, 0.0));
    }
    NSArgs a;
    a.E = M.E;
    a.conn = M.conn;
    a.epos = M.epos;
    a.xyz = M.xyz;
    a.va = M.va;
    a.acc = M.acc;
    a.vp = vp;
    a.rho = M.rho;
    a.mu = M.mu;
    a.ct = ga.ct;
    a.alpha = ga.alpha;
    a.dt = ga.dt;
    a.C_I = ctx->par.C_I;
    a.g0 = ctx->g[0];
    a.g1 = ctx->g[1];
    a.g2 = ctx->g[2];
    a.R = R;
    ElArgs el;
    el.E = M.E;
    el.N = M.N;
    el.n_s = ctx->n_s;
    el.conn = M.conn;
    el.epos = M.epos;
    el.xyz = M.xyz;
    el.as = M.as;
    el.Ba = M.Ba;
    el.muL = ctx->phase_tab + 5 * EFT_MAX_PHASE;  // mu_L of each solid
    el.alpha = ga.alpha;
    el.kappa = ga.kappa;
    el.R = R;
    const int nb = eft_grid(M.E, 128);
    if (ctx->dim == 2) {
        if (J && J->fp32) {
            hipLaunchKernelGGL((k_ns_fluid<2, float>), dim3(nb), dim3(128), 0, ctx->stream, a, J->val32);
            if (ctx->n_s > 0) hipLaunchKernelGGL((k_ns_elastic<2, float>), dim3(nb), dim3(128), 0, ctx->stream, el, J->val32);
        } else {
            double *Jv = J ? J->val : nullptr;
            hipLaunchKernelGGL((k_ns_fluid<2, double>), dim3(nb), dim3(128), 0, ctx->stream, a, Jv);
            if (ctx->n_s > 0) hipLaunchKernelGGL((k_ns_elastic<2, double>), dim3(nb), dim3(128), 0, ctx->stream, el, Jv);
        }
    } else {
        if (J && J->fp32) {
            hipLaunchKernelGGL((k_ns_fluid<3, float>), dim3(nb), dim3(128), 0, ctx->stream, a, J->val32);
            if (ctx->n_s > 0) hipLaunchKernelGGL((k_ns_elastic<3, float>), dim3(nb), dim3(128), 0, ctx->stream, el, J->val32);
        } else {
            double *Jv = J ? J->val : nullptr;
            hipLaunchKernelGGL((k_ns_fluid<3, double>), dim3(nb), dim3(128), 0, ctx->stream, a, Jv);
            if (ctx->n_s > 0) hipLaunchKernelGGL((k_ns_elastic<3, double>), dim3(nb), dim3(128), 0, ctx->stream, el, Jv);
        }
    }
    EFT_HIP(hipGetLastError());
    if (M.n_dir > 0) {
        const int nbd = eft_grid(M.n_dir, 128);
        if (J && J->fp32)
            hipLaunchKernelGGL(k_bc_rows<float>, dim3(nbd), dim3(128), 0, ctx->stream, M.n_dir, M.dir_node, M.dir_mask,
                               J->rowptr, J->col, BS, R, J->val32);
        else
            hipLaunchKernelGGL(k_bc_rows<double>, dim3(nbd), dim3(128), 0, ctx->stream, M.n_dir, M.dir_node,
                               M.dir_mask, J ? J->rowptr : nullptr, J ? J->col : nullptr, BS, R,
                               J ? J->val : (double *)nullptr);
        EFT_HIP(hipGetLastError());
    }
    return EFT_OK;
}

// Residual and Jacobian of the momentum/mass block at the iterate (the node
// fields va, acc, rho, mu, as, Ba must be current, see eft_props); with a
// Jacobian, the multigrid levels are refreshed too.
eft_status eft_ns_kernels(eft_ctx *ctx, const eft_iterate *it, double *R, eft_matrix *J)
{
    MeshView M;
    M.N = ctx->N;
    M.E = ctx->E;
    M.conn = ctx->conn;
    M.epos = ctx->epos;
    M.xyz = ctx->xyz;
    M.va = ctx->va;
    M.acc = ctx->acc;
    M.rho = ctx->rho;
    M.mu = ctx->mu;
    M.as = ctx->as;
    M.Ba = ctx->Ba;
    M.n_dir = ctx->n_dir;
    M.dir_node = ctx->dir_node;
    M.dir_mask = ctx->dir_mask;
    EFT_TRY(eft_ns_level(ctx, M, it->vp, R, J));
    if (J && eft_mg_active(ctx, J)) EFT_TRY(eft_mg_setup(ctx, it->vp));
    return EFT_OK;
}
