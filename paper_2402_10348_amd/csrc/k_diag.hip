// Diagnostics of the immersed solids (monitoring hooks outside the step):
//   centre of mass of the region of an order parameter (Sec. 3, the
//   rotating disk case: x_c = int x alpha^s dOmega / int alpha^s dOmega);
//   particle tracking (Appendix, parallel implementation of particle
//   tracking): every element is searched in parallel, the particle's element
//   is the one whose P1 shape functions at the particle all lie in [0, 1],
//   and the particle moves with the interpolated velocity.
#include <climits>

#include "dev_common.h"
#include "eft_internal.h"

namespace {

constexpr int DB = 256;
constexpr int MAX_PARTICLES = 4096;

__device__ __forceinline__ double frac_of(double phi)
{
    const double a = 0.5 * (1.0 + phi);
    return a < 0.0 ? 0.0 : (a > 1.0 ? 1.0 : a);
}

// Per-block partial sums of int alpha and int x alpha over the elements
// (degree-2 rule, exact for the linear-times-linear integrand).
template <int D>
__global__ __launch_bounds__(DB) void k_com_part(int64_t E, const int32_t *__restrict__ conn,
                                                 const double *__restrict__ xyz, const double *__restrict__ phi,
                                                 double *__restrict__ part)
{
    __shared__ double lds[DB / 64];
    constexpr int NN = D + 1, NQ = Rule<D>::NQ;
    double acc[1 + D];
#pragma unroll
    for (int c = 0; c <= D; ++c) acc[c] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * DB + threadIdx.x; e < E; e += (int64_t)gridDim.x * DB) {
        double X[NN][D], al[NN];
#pragma unroll
        for (int a = 0; a < NN; ++a) {
            const int64_t n = conn[e * NN + a];
#pragma unroll
            for (int i = 0; i < D; ++i) X[a][i] = xyz[n * D + i];
            al[a] = frac_of(phi[n]);
        }
        double dN[NN][D], G[D][D];
        const double w = simplex_geom<D>(X, dN, G) * Rule<D>::WF;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double aq = 0.0, xq[D];
#pragma unroll
            for (int i = 0; i < D; ++i) xq[i] = 0.0;
#pragma unroll
            for (int a = 0; a < NN; ++a) {
                const double Na = shape_at<D>(q, a);
                aq += Na * al[a];
#pragma unroll
                for (int i = 0; i < D; ++i) xq[i] += Na * X[a][i];
            }
            acc[0] += w * aq;
#pragma unroll
            for (int i = 0; i < D; ++i) acc[1 + i] += w * aq * xq[i];
        }
    }
#pragma unroll
    for (int c = 0; c <= D; ++c) {
        const double s = block_sum<DB>(acc[c], lds);
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * 4 + c] = s;
    }
}

// out[4 k + c] = sum over blocks of part[b][c] (fixed order), one block
__global__ __launch_bounds__(DB) void k_com_sum(const double *__restrict__ part, int nblk, int ncomp,
                                                double *__restrict__ out)
{
    __shared__ double lds[DB / 64];
    for (int c = 0; c < ncomp; ++c) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblk; b += DB) s += part[(int64_t)b * 4 + c];
        s = block_sum<DB>(s, lds);
        if (threadIdx.x == 0) out[c] = s;
    }
}

// P1 shape functions of element e at x.  They are the rows of the inverse of
// the matrix [x_a 1] of the vertex coordinates; equivalently (the form used
// here) N_a(x) = delta_a0 + grad N_a . (x - x_0) with the gradients of the
// affine map.
template <int D>
__device__ __forceinline__ void shape_at_point(const double (&X)[D + 1][D], const double (&dN)[D + 1][D],
                                               const double *x, double (&N)[D + 1])
{
#pragma unroll
    for (int a = 0; a <= D; ++a) {
        double s = a == 0 ? 1.0 : 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) s += dN[a][i] * (x[i] - X[0][i]);
        N[a] = s;
    }
}

template <int D>
__device__ __forceinline__ void element_geometry(int64_t e, const int32_t *conn, const double *xyz,
                                                 int64_t (&nodes)[D + 1], double (&X)[D + 1][D],
                                                 double (&dN)[D + 1][D])
{
#pragma unroll
    for (int a = 0; a <= D; ++a) {
        nodes[a] = conn[e * (D + 1) + a];
#pragma unroll
        for (int i = 0; i < D; ++i) X[a][i] = xyz[nodes[a] * D + i];
    }
    double G[D][D];
    (void)simplex_geom<D>(X, dN, G);
}

// found[p] = lowest element containing particle p (within tol), else INT_MAX
template <int D>
__global__ __launch_bounds__(DB) void k_locate(int64_t E, const int32_t *__restrict__ conn,
                                               const double *__restrict__ xyz, int np, const double *__restrict__ xp,
                                               double tol, int32_t *found)
{
    const int64_t e = (int64_t)blockIdx.x * DB + threadIdx.x;
    if (e >= E) return;
    int64_t nodes[D + 1];
    double X[D + 1][D], dN[D + 1][D];
    element_geometry<D>(e, conn, xyz, nodes, X, dN);
    for (int p = 0; p < np; ++p) {
        double N[D + 1];
        shape_at_point<D>(X, dN, xp + (int64_t)p * D, N);
        bool in = true;
#pragma unroll
        for (int a = 0; a <= D; ++a) in = in && N[a] >= -tol && N[a] <= 1.0 + tol;
        if (in) atomicMin(found + p, (int32_t)e);
    }
}

// x_p += dt sum_a N_a v_a in the element found; found[p] = -1 when none
template <int D>
__global__ void k_move(int np, const int32_t *__restrict__ conn, const double *__restrict__ xyz,
                       const double *__restrict__ vp, double dt, double *xp, int32_t *found)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int32_t e = found[p];
    if (e == INT_MAX) {
        found[p] = -1;
        return;
    }
    int64_t nodes[D + 1];
    double X[D + 1][D], dN[D + 1][D], N[D + 1];
    element_geometry<D>(e, conn, xyz, nodes, X, dN);
    double *x = xp + (int64_t)p * D;
    shape_at_point<D>(X, dN, x, N);
    double v[D];
#pragma unroll
    for (int i = 0; i < D; ++i) v[i] = 0.0;
#pragma unroll
    for (int a = 0; a <= D; ++a)
#pragma unroll
        for (int i = 0; i < D; ++i) v[i] += N[a] * vp[nodes[a] * (D + 1) + i];
#pragma unroll
    for (int i = 0; i < D; ++i) x[i] += dt * v[i];
}

__global__ void k_fill_i32(int32_t *p, int n, int32_t v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

eft_status diag_reserve(eft_ctx *ctx, int64_t doubles)
{
    if (doubles <= ctx->dg_cap) return EFT_OK;
    if (ctx->dg) (void)hipFree(ctx->dg);
    ctx->dg = nullptr;
    ctx->dg_cap = 0;
    if (hipMalloc(&ctx->dg, sizeof(double) * doubles) != hipSuccess) {
        ctx->err = "out of device memory (diagnostics)";
        return EFT_ENOMEM;
    }
    ctx->dg_cap = doubles;
    return EFT_OK;
}

}  // namespace

eft_status eft_center_of_mass(eft_ctx *ctx, const double *phi, double *xc, double *mass)
{
    if (!ctx || (ctx->n_ind > 0 && (!phi || !xc || !mass))) return EFT_EINVAL;
    const int D = ctx->dim, K = ctx->n_ind;
    const int nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (ctx->E + DB - 1) / DB));
    EFT_TRY(diag_reserve(ctx, (int64_t)nblk * 4 + 4 * (int64_t)K));
    double *part = ctx->dg, *out = ctx->dg + (int64_t)nblk * 4;
    for (int k = 0; k < K; ++k) {
        const double *ph = phi + (int64_t)k * ctx->N;
        if (D == 2)
            hipLaunchKernelGGL(k_com_part<2>, dim3(nblk), dim3(DB), 0, ctx->stream, ctx->E, ctx->conn, ctx->xyz, ph,
                               part);
        else
            hipLaunchKernelGGL(k_com_part<3>, dim3(nblk), dim3(DB), 0, ctx->stream, ctx->E, ctx->conn, ctx->xyz, ph,
                               part);
        hipLaunchKernelGGL(k_com_sum, dim3(1), dim3(DB), 0, ctx->stream, part, nblk, D + 1, out + 4 * k);
    }
    EFT_HIP(hipGetLastError());
    std::vector<double> h(4 * (size_t)K);
    if (K > 0) EFT_HIP(hipMemcpyAsync(h.data(), out, sizeof(double) * 4 * K, hipMemcpyDeviceToHost, ctx->stream));
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < K; ++k) {
        const double m = h[4 * k];
        mass[k] = m;
        for (int i = 0; i < 3; ++i) xc[3 * k + i] = (i < D && m > 0.0) ? h[4 * k + 1 + i] / m : 0.0;
    }
    return EFT_OK;
}

eft_status eft_track_particles(eft_ctx *ctx, const double *vp, int32_t n_p, double dt, double tol, double *x,
                               int32_t *elem)
{
    if (!ctx || n_p < 0 || (n_p > 0 && (!vp || !x || !elem))) return EFT_EINVAL;
    if (n_p > MAX_PARTICLES) {
        ctx->err = "at most 4096 particles per call";
        return EFT_EINVAL;
    }
    if (!(tol >= 0.0)) {
        ctx->err = "tol must be >= 0";
        return EFT_EINVAL;
    }
    if (n_p == 0) return EFT_OK;
    const int D = ctx->dim;
    // particles [n_p][D] then the found indices (int32, packed in doubles)
    EFT_TRY(diag_reserve(ctx, (int64_t)n_p * D + (n_p + 1) / 2 + 1));
    double *xp = ctx->dg;
    int32_t *found = reinterpret_cast<int32_t *>(ctx->dg + (int64_t)n_p * D);
    EFT_HIP(hipMemcpyAsync(xp, x, sizeof(double) * n_p * D, hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(k_fill_i32, dim3((n_p + 255) / 256), dim3(256), 0, ctx->stream, found, n_p, (int32_t)INT_MAX);
    const dim3 ge((unsigned)((ctx->E + DB - 1) / DB));
    if (D == 2) {
        hipLaunchKernelGGL(k_locate<2>, ge, dim3(DB), 0, ctx->stream, ctx->E, ctx->conn, ctx->xyz, n_p, xp, tol, found);
        hipLaunchKernelGGL(k_move<2>, dim3((n_p + 63) / 64), dim3(64), 0, ctx->stream, n_p, ctx->conn, ctx->xyz, vp, dt,
                           xp, found);
    } else {
        hipLaunchKernelGGL(k_locate<3>, ge, dim3(DB), 0, ctx->stream, ctx->E, ctx->conn, ctx->xyz, n_p, xp, tol, found);
        hipLaunchKernelGGL(k_move<3>, dim3((n_p + 63) / 64), dim3(64), 0, ctx->stream, n_p, ctx->conn, ctx->xyz, vp, dt,
                           xp, found);
    }
    EFT_HIP(hipGetLastError());
    EFT_HIP(hipMemcpyAsync(x, xp, sizeof(double) * n_p * D, hipMemcpyDeviceToHost, ctx->stream));
    EFT_HIP(hipMemcpyAsync(elem, found, sizeof(int32_t) * n_p, hipMemcpyDeviceToHost, ctx->stream));
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    return EFT_OK;
}
