// Block ILU(0) preconditioner of the momentum/mass system: the unit
// block-lower L and block-upper U keep the matrix pattern and L U equals A on
// it (natural row order; Saad, Iterative Methods for Sparse Linear Systems,
// Sec. 10.3).  A plain preconditioner beside point-block Jacobi and the
// multigrid V-cycle for the right-preconditioned FGMRES of eq. (LS_NS).
//
// Level schedule.  Row i of the factorization and of the forward solve needs
// the rows k < i of its pattern, the backward solve the rows j > i; the host
// groups the rows by the length of the longest such chain (computed once per
// pattern), and one launch per level treats its rows in parallel, one thread
// per block row.  On a structured Kuhn mesh in lexicographic order a node's
// level is about i + j + k, so there are about nx + ny + nz levels.
//
// Factorization of row i, in the oracle's order: for the k < i of the row in
// increasing order, L_ik = A_ik U_kk^-1, then A_ij -= L_ik U_kj for the j > k
// of row i that row k holds (a merge of the two sorted column lists); then
// dinv[i] = U_ii^-1 (Gauss-Jordan with partial pivoting).
#include <vector>

#include "dev_common.h"
#include "eft_internal.h"

namespace {

template <int BS, typename TV>
__global__ __launch_bounds__(256) void k_ilu_copy(int64_t nv, const TV *__restrict__ val, double *__restrict__ lu)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x)
        lu[i] = (double)val[i];
}

template <int BS>
__device__ __forceinline__ void blk_mul(const double *__restrict__ A, const double *__restrict__ B, double (&C)[BS][BS])
{
#pragma unroll
    for (int i = 0; i < BS; ++i)
#pragma unroll
        for (int j = 0; j < BS; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < BS; ++k) s += A[i * BS + k] * B[k * BS + j];
            C[i][j] = s;
        }
}

// inverse of one block by Gauss-Jordan with partial pivoting; false if singular
template <int BS> __device__ __forceinline__ bool blk_inverse(const double *__restrict__ blk, double *__restrict__ out)
{
    double A[BS][BS], I[BS][BS];
#pragma unroll
    for (int i = 0; i < BS; ++i)
#pragma unroll
        for (int j = 0; j < BS; ++j) {
            A[i][j] = blk[i * BS + j];
            I[i][j] = i == j ? 1.0 : 0.0;
        }
    bool ok = true;
#pragma unroll
    for (int k = 0; k < BS; ++k) {
        int pr = k;
        double best = fabs(A[k][k]);
#pragma unroll
        for (int i = k + 1; i < BS; ++i)
            if (fabs(A[i][k]) > best) {
                best = fabs(A[i][k]);
                pr = i;
            }
        ok = ok && best != 0.0;
#pragma unroll
        for (int i = k + 1; i < BS; ++i)
            if (i == pr)
#pragma unroll
                for (int j = 0; j < BS; ++j) {
                    double t = A[k][j];
                    A[k][j] = A[i][j];
                    A[i][j] = t;
                    t = I[k][j];
                    I[k][j] = I[i][j];
                    I[i][j] = t;
                }
        const double inv = best != 0.0 ? 1.0 / A[k][k] : 0.0;
#pragma unroll
        for (int j = 0; j < BS; ++j) {
            A[k][j] *= inv;
            I[k][j] *= inv;
        }
#pragma unroll
        for (int i = 0; i < BS; ++i) {
            if (i == k) continue;
            const double f = A[i][k];
#pragma unroll
            for (int j = 0; j < BS; ++j) {
                A[i][j] -= f * A[k][j];
                I[i][j] -= f * I[k][j];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < BS; ++i)
#pragma unroll
        for (int j = 0; j < BS; ++j) out[i * BS + j] = ok ? I[i][j] : (i == j ? 1.0 : 0.0);
    return ok;
}

// one level of the factorization (rows of the level, one thread each)
template <int BS>
__global__ __launch_bounds__(256) void k_ilu_factor(int nr, const int32_t *__restrict__ rows,
                                                    const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                                    const int32_t *__restrict__ diag, double *__restrict__ lu,
                                                    double *__restrict__ dinv, int32_t *sing)
{
    constexpr int B2 = BS * BS;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nr) return;
    const int i = rows[t];
    const int pe = rowptr[i + 1], pd = diag[i];
    for (int p = rowptr[i]; p < pd; ++p) {
        const int k = col[p];
        double L[BS][BS];
        blk_mul<BS>(lu + (int64_t)p * B2, dinv + (int64_t)k * B2, L);
#pragma unroll
        for (int a = 0; a < BS; ++a)
#pragma unroll
            for (int b = 0; b < BS; ++b) lu[(int64_t)p * B2 + a * BS + b] = L[a][b];
        int qk = diag[k] + 1;
        const int ke = rowptr[k + 1];
        for (int q = p + 1; q < pe && qk < ke; ++q) {
            const int j = col[q];
            while (qk < ke && col[qk] < j) ++qk;
            if (qk < ke && col[qk] == j) {
                const double *Ukj = lu + (int64_t)qk * B2;
                double *Aij = lu + (int64_t)q * B2;
#pragma unroll
                for (int a = 0; a < BS; ++a)
#pragma unroll
                    for (int b = 0; b < BS; ++b) {
                        double s = 0.0;
#pragma unroll
                        for (int c = 0; c < BS; ++c) s += L[a][c] * Ukj[c * BS + b];
                        Aij[a * BS + b] -= s;
                    }
            }
        }
    }
    if (!blk_inverse<BS>(lu + (int64_t)pd * B2, dinv + (int64_t)i * B2) && sing) *sing = 1;
}

// one level of L y = r (unit diagonal), y written to z
template <int BS>
__global__ __launch_bounds__(256) void k_ilu_lower(int nr, const int32_t *__restrict__ rows,
                                                   const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                                   const int32_t *__restrict__ diag, const double *__restrict__ lu,
                                                   const double *__restrict__ r, double *__restrict__ z,
                                                   const int32_t *flag)
{
    constexpr int B2 = BS * BS;
    if (flag && flag[0] == 0) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nr) return;
    const int i = rows[t];
    double y[BS];
#pragma unroll
    for (int a = 0; a < BS; ++a) y[a] = r[(int64_t)i * BS + a];
    for (int p = rowptr[i]; p < diag[i]; ++p) {
        const double *Lp = lu + (int64_t)p * B2, *zk = z + (int64_t)col[p] * BS;
#pragma unroll
        for (int a = 0; a < BS; ++a)
#pragma unroll
            for (int c = 0; c < BS; ++c) y[a] -= Lp[a * BS + c] * zk[c];
    }
#pragma unroll
    for (int a = 0; a < BS; ++a) z[(int64_t)i * BS + a] = y[a];
}

// one level of U z = y (in place in z)
template <int BS>
__global__ __launch_bounds__(256) void k_ilu_upper(int nr, const int32_t *__restrict__ rows,
                                                   const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                                   const int32_t *__restrict__ diag, const double *__restrict__ lu,
                                                   const double *__restrict__ dinv, double *__restrict__ z,
                                                   const int32_t *flag)
{
    constexpr int B2 = BS * BS;
    if (flag && flag[0] == 0) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nr) return;
    const int i = rows[t];
    double y[BS];
#pragma unroll
    for (int a = 0; a < BS; ++a) y[a] = z[(int64_t)i * BS + a];
    for (int p = diag[i] + 1; p < rowptr[i + 1]; ++p) {
        const double *Up = lu + (int64_t)p * B2, *zj = z + (int64_t)col[p] * BS;
#pragma unroll
        for (int a = 0; a < BS; ++a)
#pragma unroll
            for (int c = 0; c < BS; ++c) y[a] -= Up[a * BS + c] * zj[c];
    }
    const double *D = dinv + (int64_t)i * B2;
#pragma unroll
    for (int a = 0; a < BS; ++a) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < BS; ++c) s += D[a * BS + c] * y[c];
        z[(int64_t)i * BS + a] = s;
    }
}

// rows grouped by level: lower (k < i) when up is false, upper (j > i) else
void levels(int64_t n, const std::vector<int32_t> &rowptr, const std::vector<int32_t> &col, bool up,
            std::vector<int32_t> &off, std::vector<int32_t> &rows)
{
    std::vector<int32_t> lev(n, 0);
    int32_t nlev = 0;
    for (int64_t s = 0; s < n; ++s) {
        const int64_t i = up ? n - 1 - s : s;
        int32_t l = 0;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            const int64_t k = col[p];
            if (up ? k > i : k < i) l = std::max(l, lev[k] + 1);
        }
        lev[i] = l;
        nlev = std::max(nlev, l + 1);
    }
    off.assign(nlev + 1, 0);
    for (int64_t i = 0; i < n; ++i) off[lev[i] + 1]++;
    for (int32_t l = 0; l < nlev; ++l) off[l + 1] += off[l];
    rows.assign(n, 0);
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (int64_t i = 0; i < n; ++i) rows[fill[lev[i]]++] = (int32_t)i;
}

}  // namespace

// Storage and level schedule of the factors, reserved when the momentum
// solves use ILU(0) (at creation and when the parameters change), so that a
// time step allocates nothing.
eft_status eft_ilu_reserve(eft_ctx *ctx)
{
    IluState &S = ctx->ilu;
    if (ctx->par.precond != 3 || S.lu) return EFT_OK;
    const eft_matrix &J = ctx->J;
    const int b2 = J.bs * J.bs;
    std::vector<int32_t> rowptr(J.n + 1), col(J.nnzb);
    EFT_HIP(hipMemcpy(rowptr.data(), J.rowptr, sizeof(int32_t) * (J.n + 1), hipMemcpyDeviceToHost));
    EFT_HIP(hipMemcpy(col.data(), J.col, sizeof(int32_t) * J.nnzb, hipMemcpyDeviceToHost));
    std::vector<int32_t> lrows, urows;
    levels(J.n, rowptr, col, false, S.loff, lrows);
    levels(J.n, rowptr, col, true, S.uoff, urows);
    if (hipMalloc(&S.lu, sizeof(double) * J.nnzb * b2) != hipSuccess ||
        hipMalloc(&S.dinv, sizeof(double) * J.n * b2) != hipSuccess ||
        hipMalloc(&S.lrows, sizeof(int32_t) * J.n) != hipSuccess ||
        hipMalloc(&S.urows, sizeof(int32_t) * J.n) != hipSuccess) {
        ctx->err = "out of device memory for the ILU(0) factors";
        return EFT_ENOMEM;
    }
    EFT_HIP(hipMemcpy(S.lrows, lrows.data(), sizeof(int32_t) * J.n, hipMemcpyHostToDevice));
    EFT_HIP(hipMemcpy(S.urows, urows.data(), sizeof(int32_t) * J.n, hipMemcpyHostToDevice));
    return EFT_OK;
}

void eft_ilu_free(eft_ctx *ctx)
{
    IluState &S = ctx->ilu;
    for (void *p : {(void *)S.lu, (void *)S.dinv, (void *)S.lrows, (void *)S.urows})
        if (p) (void)hipFree(p);
    S = IluState{};
}

// Factor the context's momentum matrix (sing set to 1 on a singular U_ii).
eft_status eft_ilu_setup(eft_ctx *ctx, const eft_matrix *A, int32_t *sing)
{
    IluState &S = ctx->ilu;
    if (A != &ctx->J || !S.lu) {
        ctx->err = "ILU(0) factors are reserved for the momentum/mass matrix with precond = 3";
        return EFT_EINVAL;
    }
    const int bs = A->bs;
    const int64_t nv = A->nnzb * bs * bs;
    const int g = (int)std::min<int64_t>(8192, (nv + 255) / 256);
    if (bs == 4) {
        if (A->fp32) hipLaunchKernelGGL((k_ilu_copy<4, float>), dim3(g), dim3(256), 0, ctx->stream, nv, A->val32, S.lu);
        else hipLaunchKernelGGL((k_ilu_copy<4, double>), dim3(g), dim3(256), 0, ctx->stream, nv, A->val, S.lu);
    } else {
        if (A->fp32) hipLaunchKernelGGL((k_ilu_copy<3, float>), dim3(g), dim3(256), 0, ctx->stream, nv, A->val32, S.lu);
        else hipLaunchKernelGGL((k_ilu_copy<3, double>), dim3(g), dim3(256), 0, ctx->stream, nv, A->val, S.lu);
    }
    for (size_t l = 0; l + 1 < S.loff.size(); ++l) {
        const int nr = S.loff[l + 1] - S.loff[l];
        const dim3 gr((nr + 255) / 256), tb(256);
        if (bs == 4)
            hipLaunchKernelGGL(k_ilu_factor<4>, gr, tb, 0, ctx->stream, nr, S.lrows + S.loff[l], A->rowptr, A->col,
                               A->diag, S.lu, S.dinv, sing);
        else
            hipLaunchKernelGGL(k_ilu_factor<3>, gr, tb, 0, ctx->stream, nr, S.lrows + S.loff[l], A->rowptr, A->col,
                               A->diag, S.lu, S.dinv, sing);
    }
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}

// z = (L U)^-1 r with the current factors (gated by flag[0] when flag is set).
eft_status eft_ilu_apply(eft_ctx *ctx, const double *r, double *z, const int32_t *flag)
{
    const IluState &S = ctx->ilu;
    const eft_matrix &A = ctx->J;
    const int bs = A.bs;
    for (size_t l = 0; l + 1 < S.loff.size(); ++l) {
        const int nr = S.loff[l + 1] - S.loff[l];
        const dim3 gr((nr + 255) / 256), tb(256);
        if (bs == 4)
            hipLaunchKernelGGL(k_ilu_lower<4>, gr, tb, 0, ctx->stream, nr, S.lrows + S.loff[l], A.rowptr, A.col,
                               A.diag, S.lu, r, z, flag);
        else
            hipLaunchKernelGGL(k_ilu_lower<3>, gr, tb, 0, ctx->stream, nr, S.lrows + S.loff[l], A.rowptr, A.col,
                               A.diag, S.lu, r, z, flag);
    }
    for (size_t l = 0; l + 1 < S.uoff.size(); ++l) {
        const int nr = S.uoff[l + 1] - S.uoff[l];
        const dim3 gr((nr + 255) / 256), tb(256);
        if (bs == 4)
            hipLaunchKernelGGL(k_ilu_upper<4>, gr, tb, 0, ctx->stream, nr, S.urows + S.uoff[l], A.rowptr, A.col,
                               A.diag, S.lu, S.dinv, z, flag);
        else
            hipLaunchKernelGGL(k_ilu_upper<3>, gr, tb, 0, ctx->stream, nr, S.urows + S.uoff[l], A.rowptr, A.col,
                               A.diag, S.lu, S.dinv, z, flag);
    }
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}

// Test hook: the factors of the current momentum matrix (device arrays of
// the caller: lu [nnzb][bs*bs], dinv [n][bs*bs]).
extern "C" eft_status eft_ilu_export(eft_ctx *ctx, double *lu, double *dinv)
{
    if (!ctx) return EFT_EINVAL;
    if (ctx->par.precond != 3 || !ctx->ilu.lu) {
        ctx->err = "eft_ilu_export needs precond = 3";
        return EFT_EINVAL;
    }
    int32_t *sing = nullptr;
    EFT_HIP(hipMalloc(&sing, sizeof(int32_t)));
    EFT_HIP(hipMemsetAsync(sing, 0, sizeof(int32_t), ctx->stream));
    eft_status st = eft_ilu_setup(ctx, &ctx->J, sing);
    int32_t hs = 0;
    if (st == EFT_OK) {
        const eft_matrix &A = ctx->J;
        const int b2 = A.bs * A.bs;
        if (lu) EFT_HIP(hipMemcpyAsync(lu, ctx->ilu.lu, sizeof(double) * A.nnzb * b2, hipMemcpyDeviceToDevice, ctx->stream));
        if (dinv) EFT_HIP(hipMemcpyAsync(dinv, ctx->ilu.dinv, sizeof(double) * A.n * b2, hipMemcpyDeviceToDevice, ctx->stream));
        EFT_HIP(hipMemcpyAsync(&hs, sing, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
        EFT_HIP(hipStreamSynchronize(ctx->stream));
    }
    (void)hipFree(sing);
    if (st == EFT_OK && hs) {
        ctx->err = "ILU(0): singular diagonal block";
        return EFT_EBREAKDOWN;
    }
    return st;
}
