// Sparse kernels of the Krylov solve (eq. LS_NS and the band systems):
// BSR sparse matrix-vector product and point-block Jacobi.
//
// SpMV layout for bs = 3, 4, 6 (the momentum/mass system in 2D and 3D and
// the 3D B system): one wavefront per block row, one lane per scalar row of
// a block (bsr_rows.h); FP32 values of bs 3 and 4 take one block per lane.
// Other bs: one value per lane, LDS reduction.  bs = 1 uses 16 lanes per row.
#include <type_traits>

#include "bsr_rows.h"
#include "dev_common.h"
#include "eft_internal.h"

template <typename TV> __device__ __forceinline__ double ld(const TV *p) { return (double)*p; }

// bs in {3, 4, 6}: SPMV_R block rows per wavefront, cached value loads
// (measured fastest on the 64^3 momentum matrix).  GATED instances (inside
// the Krylov loop) return at once when the solve has converged; the plain
// instances always do the product.
constexpr int SPMV_R = 2;

template <int BS, typename TV, bool GATED>
__global__ __launch_bounds__(256) void k_spmv_rows(int64_t n, const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ col, const TV *__restrict__ val,
                                                   const double *__restrict__ x, double *__restrict__ y,
                                                   const int32_t *active)
{
    const int64_t w = (int64_t)blockIdx.x * 4 + wave_id();
    int64_t row[SPMV_R];
#pragma unroll
    for (int q = 0; q < SPMV_R; ++q) row[q] = w * SPMV_R + q;
    int k0[SPMV_R], k1[SPMV_R];
    row_extents<SPMV_R>(row, n, rowptr, k0, k1);
    if ((GATED && *active == 0) || row[0] >= n) return;
    const int lane = threadIdx.x & 63;
    double acc[SPMV_R];
    bsr_rows_dot<BS, TV, SPMV_R, false>(k0, k1, col, val, x, lane, acc);
#pragma unroll
    for (int q = 0; q < SPMV_R; ++q)
        if (lane < BS && row[q] < n) y[row[q] * BS + lane] = acc[q];
}

// The same product for a pattern in stencil form (FP64 values, bs 3 or 4):
// the row masks are wave-uniform (scalar loads) and no column index is read.
template <int BS, bool GATED>
__global__ __launch_bounds__(256) void k_spmv_stn(int64_t n, const int32_t *__restrict__ rowptr,
                                                  const uint16_t *__restrict__ smask, const int32_t *__restrict__ soff,
                                                  const double *__restrict__ val, const double *__restrict__ x,
                                                  double *__restrict__ y, const int32_t *active)
{
    constexpr int MAXS = BS == 4 ? 16 : 8;
    const int64_t w = (int64_t)blockIdx.x * 4 + wave_id();
    int64_t row[SPMV_R];
#pragma unroll
    for (int q = 0; q < SPMV_R; ++q) row[q] = w * SPMV_R + q;
    int k0[SPMV_R], k1[SPMV_R];
    row_extents<SPMV_R>(row, n, rowptr, k0, k1);
    uint32_t m[SPMV_R];
#pragma unroll
    for (int q = 0; q < SPMV_R; ++q) m[q] = row[q] < n ? smask[row[q]] : 0u;
    if ((GATED && *active == 0) || row[0] >= n) return;
    const int lane = threadIdx.x & 63, j = lane / BS;
    const int oj = j < MAXS ? soff[j] : 0;
    double acc[SPMV_R];
    bsr_rows_stencil_dot<BS, double, SPMV_R, MAXS>(k0, m, row, oj, val, x, lane, acc);
#pragma unroll
    for (int q = 0; q < SPMV_R; ++q)
        if (lane < BS && row[q] < n) y[row[q] * BS + lane] = acc[q];
}

// The same product with one block per lane (narrow values, bs 3 or 4),
// with the pattern's column indices or (STN) its stencil form.
template <int BS, typename TV, bool GATED, bool STN>
__global__ __launch_bounds__(256) void k_spmv_blk(int64_t n, const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col, const uint16_t *__restrict__ smask,
                                                  const int32_t *__restrict__ soff, const TV *__restrict__ val,
                                                  const double *__restrict__ x, double *__restrict__ y,
                                                  const int32_t *active)
{
    constexpr int SEG = BlockSeg<BS>::SEG, RPW = BlockSeg<BS>::RPW;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave_id()) * RPW;
    if ((GATED && *active == 0) || row0 >= n) return;
    const int lane = threadIdx.x & 63, q = lane / SEG, j = lane - q * SEG;
    const int64_t row = row0 + q;
    uint32_t m = 0;
    int oj = 0;
    if constexpr (STN) {
        m = row < n ? smask[row] : 0u;
        oj = soff[j];
    }
    int k0, k1;
    seg_extents<RPW>(row0, n, rowptr, q, k0, k1);
    double acc[BS];
    if constexpr (STN) bsr_stencil_dot<BS, TV, SEG>(k0, m, row < n ? row : row0, oj, val, x, j, acc);
    else bsr_block_dot<BS, TV, SEG>(k0, k1, col, val, x, j, acc);
#pragma unroll
    for (int c = 0; c < BS; ++c)
        if (j == c && row < n) y[row * BS + c] = acc[c];
}

// general bs in 2..8: LDS reduction per wavefront.
template <typename TV>
__global__ __launch_bounds__(256) void k_spmvb(int64_t n, int bs, const int32_t *__restrict__ rowptr,
                                               const int32_t *__restrict__ col, const TV *__restrict__ val,
                                               const double *__restrict__ x, double *__restrict__ y,
                                               const int32_t *active)
{
    __shared__ double lds[256];
    if (active && *active == 0) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int b2 = bs * bs, slots = 64 / b2;
    const int slot = lane / b2, e = lane - slot * b2, c = e % bs;
    double acc = 0.0;
    if (row < n && slot < slots) {
        const int k0 = rowptr[row], k1 = rowptr[row + 1];
        for (int k = k0 + slot; k < k1; k += slots) acc += ld(val + (int64_t)k * b2 + e) * x[(int64_t)col[k] * bs + c];
    }
    lds[threadIdx.x] = acc;
    __syncthreads();
    if (row < n && lane < bs) {
        double s = 0.0;
        for (int sl = 0; sl < slots; ++sl)
            for (int cc = 0; cc < bs; ++cc) s += lds[wv * 64 + sl * b2 + lane * bs + cc];
        y[row * bs + lane] = s;
    }
}

// bs = 1: 16 lanes per row.
template <typename TV>
__global__ __launch_bounds__(256) void k_spmv1(int64_t n, const int32_t *__restrict__ rowptr,
                                               const int32_t *__restrict__ col, const TV *__restrict__ val,
                                               const double *__restrict__ x, double *__restrict__ y,
                                               const int32_t *active)
{
    if (active && *active == 0) return;
    const int sub = threadIdx.x & 15;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    double acc = 0.0;
    if (row < n) {
        const int k0 = rowptr[row], k1 = rowptr[row + 1];
        for (int k = k0 + sub; k < k1; k += 16) acc += ld(val + k) * x[col[k]];
    }
    acc += __shfl_xor(acc, 1, 16);
    acc += __shfl_xor(acc, 2, 16);
    acc += __shfl_xor(acc, 4, 16);
    acc += __shfl_xor(acc, 8, 16);
    if (row < n && sub == 0) y[row] = acc;
}

template <int BS, typename TV>
static void spmv_rows_launch(eft_ctx *ctx, int64_t n, const int32_t *rowptr, const int32_t *col, const TV *val,
                             const double *x, double *y, const int32_t *active, const uint16_t *smask = nullptr,
                             const int32_t *soff = nullptr)
{
    if constexpr (sizeof(TV) < 8 && BS <= 4) {
        const dim3 g(eft_grid(n, 4 * BlockSeg<BS>::RPW));
#define EFT_SPMV_BLK(G_, S_) \
    hipLaunchKernelGGL((k_spmv_blk<BS, TV, G_, S_>), g, dim3(256), 0, ctx->stream, n, rowptr, col, smask, soff, val, x, y, active)
        if (smask) {
            if (active) EFT_SPMV_BLK(true, true);
            else EFT_SPMV_BLK(false, true);
        } else {
            if (active) EFT_SPMV_BLK(true, false);
            else EFT_SPMV_BLK(false, false);
        }
#undef EFT_SPMV_BLK
    } else if (active)
        hipLaunchKernelGGL((k_spmv_rows<BS, TV, true>), dim3(eft_grid(n, 4 * SPMV_R)), dim3(256), 0, ctx->stream, n,
                           rowptr, col, val, x, y, active);
    else
        hipLaunchKernelGGL((k_spmv_rows<BS, TV, false>), dim3(eft_grid(n, 4 * SPMV_R)), dim3(256), 0, ctx->stream, n,
                           rowptr, col, val, x, y, active);
}

template <typename TV>
static void spmv_launch(eft_ctx *ctx, int64_t n, int bs, const int32_t *rowptr, const int32_t *col, const TV *val,
                        const double *x, double *y, const int32_t *active)
{
    if (bs == 1)
        hipLaunchKernelGGL(k_spmv1<TV>, dim3(eft_grid(n, 16)), dim3(256), 0, ctx->stream, n, rowptr, col, val, x, y,
                           active);
    else if (bs == 3)
        spmv_rows_launch<3, TV>(ctx, n, rowptr, col, val, x, y, active);
    else if (bs == 4)
        spmv_rows_launch<4, TV>(ctx, n, rowptr, col, val, x, y, active);
    else if (bs == 6)
        spmv_rows_launch<6, TV>(ctx, n, rowptr, col, val, x, y, active);
    else
        hipLaunchKernelGGL(k_spmvb<TV>, dim3(eft_grid(n, 4)), dim3(256), 0, ctx->stream, n, bs, rowptr, col, val, x,
                           y, active);
}

eft_status eft_spmv_flag(eft_ctx *ctx, const eft_matrix *A, const double *x, double *y, const int32_t *active)
{
    if (A->n == 0) return EFT_OK;
    if (A->bcmp) return eft_bcmp_spmv(ctx, A, x, y, active);
    if (A->stn_mask && !A->fp32 && (A->bs == 3 || A->bs == 4)) {
#define EFT_SPMV_STN(B_, G_)                                                                                       \
    hipLaunchKernelGGL((k_spmv_stn<B_, G_>), dim3(eft_grid(A->n, 4 * SPMV_R)), dim3(256), 0, ctx->stream, A->n, \
                       A->rowptr, A->stn_mask, A->stn_off, A->val, x, y, active)
        if (A->bs == 3) {
            if (active) EFT_SPMV_STN(3, true);
            else EFT_SPMV_STN(3, false);
        } else {
            if (active) EFT_SPMV_STN(4, true);
            else EFT_SPMV_STN(4, false);
        }
#undef EFT_SPMV_STN
    } else if (A->fp32 && A->stn_mask && (A->bs == 3 || A->bs == 4)) {
        if (A->bs == 3)
            spmv_rows_launch<3, float>(ctx, A->n, A->rowptr, A->col, A->val32, x, y, active, A->stn_mask, A->stn_off);
        else
            spmv_rows_launch<4, float>(ctx, A->n, A->rowptr, A->col, A->val32, x, y, active, A->stn_mask, A->stn_off);
    } else if (A->fp32) {
        spmv_launch<float>(ctx, A->n, A->bs, A->rowptr, A->col, A->val32, x, y, active);
    } else {
        spmv_launch<double>(ctx, A->n, A->bs, A->rowptr, A->col, A->val, x, y, active);
    }
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}

eft_status eft_spmv_dev(eft_ctx *ctx, const eft_matrix *A, const double *x, double *y)
{
    return eft_spmv_flag(ctx, A, x, y, nullptr);
}

// -------------------------------------------------- point-block Jacobi ----

// Inverse of each diagonal block by Gauss-Jordan elimination with partial
// pivoting.  A block with a zero pivot gets the identity (no scaling).
template <typename TV, typename TD>
__global__ __launch_bounds__(256) void k_bj_setup(int64_t n, int bs, const int32_t *__restrict__ diag,
                                                  const TV *__restrict__ val, TD *__restrict__ Dinv, int32_t *sing)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double A[8][8], I[8][8];
    const int b2 = bs * bs;
    const TV *blk = val + (int64_t)diag[r] * b2;
    for (int i = 0; i < bs; ++i)
        for (int j = 0; j < bs; ++j) {
            A[i][j] = (double)blk[i * bs + j];
            I[i][j] = (i == j) ? 1.0 : 0.0;
        }
    bool ok = true;
    for (int k = 0; k < bs && ok; ++k) {
        int pr = k;
        for (int i = k + 1; i < bs; ++i)
            if (fabs(A[i][k]) > fabs(A[pr][k])) pr = i;
        if (A[pr][k] == 0.0) {
            ok = false;
            break;
        }
        if (pr != k)
            for (int j = 0; j < bs; ++j) {
                double t = A[k][j]; A[k][j] = A[pr][j]; A[pr][j] = t;
                t = I[k][j]; I[k][j] = I[pr][j]; I[pr][j] = t;
            }
        const double inv = 1.0 / A[k][k];
        for (int j = 0; j < bs; ++j) {
            A[k][j] *= inv;
            I[k][j] *= inv;
        }
        for (int i = 0; i < bs; ++i) {
            if (i == k) continue;
            const double f = A[i][k];
            if (f == 0.0) continue;
            for (int j = 0; j < bs; ++j) {
                A[i][j] -= f * A[k][j];
                I[i][j] -= f * I[k][j];
            }
        }
    }
    TD *out = Dinv + r * b2;
    for (int i = 0; i < bs; ++i)
        for (int j = 0; j < bs; ++j) out[i * bs + j] = (TD)(ok ? I[i][j] : (i == j ? 1.0 : 0.0));
    if (!ok && sing) *sing = 1;
}

// The same elimination with the block size fixed at compile time: every
// loop unrolls and the row exchange of the pivot search is a predicated swap
// at static indices, so the block stays in registers (with a run-time size
// the arrays above live in scratch memory).
template <int BS, typename TV, typename TD>
__global__ __launch_bounds__(256) void k_bj_setup_t(int64_t n, const int32_t *__restrict__ diag,
                                                    const TV *__restrict__ val, TD *__restrict__ Dinv, int32_t *sing)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double A[BS][BS], I[BS][BS];
    const TV *blk = val + (int64_t)diag[r] * BS * BS;
#pragma unroll
    for (int i = 0; i < BS; ++i)
#pragma unroll
        for (int j = 0; j < BS; ++j) {
            A[i][j] = (double)blk[i * BS + j];
            I[i][j] = (i == j) ? 1.0 : 0.0;
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
    TD *out = Dinv + r * BS * BS;
#pragma unroll
    for (int i = 0; i < BS; ++i)
#pragma unroll
        for (int j = 0; j < BS; ++j) out[i * BS + j] = (TD)(ok ? I[i][j] : (i == j ? 1.0 : 0.0));
    if (!ok && sing) *sing = 1;
}

template <typename TD>
__global__ __launch_bounds__(256) void k_bj_apply(int64_t nd, int bs, const TD *__restrict__ Dinv, double omega,
                                                  const double *__restrict__ x, double *__restrict__ z,
                                                  const int32_t *active)
{
    if (active && *active == 0) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nd) return;
    const int64_t r = t / bs;
    const int i = (int)(t - r * bs);
    const TD *D = Dinv + r * bs * bs + i * bs;
    const double *xr = x + r * bs;
    double s = 0.0;
    for (int c = 0; c < bs; ++c) s += (double)D[c] * xr[c];
    z[t] = omega * s;
}

// One damped point-block Jacobi sweep zo = z + omega D^-1 (v - A z), the
// arithmetic and vectors FP64, values and inverses FP64 or FP32 copies.
// bs = 1: 16 lanes per row as the scalar product.
template <typename TV>
__global__ __launch_bounds__(256) void k_jsweep1(int64_t n, const int32_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ col, const TV *__restrict__ val,
                                                 const TV *__restrict__ Dinv, double omega,
                                                 const double *__restrict__ v, const double *__restrict__ z,
                                                 double *__restrict__ zo, const int32_t *active)
{
    if (*active == 0) return;
    const int sub = threadIdx.x & 15;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    double acc = 0.0;
    if (row < n) {
        const int k0 = rowptr[row], k1 = rowptr[row + 1];
        for (int k = k0 + sub; k < k1; k += 16) acc += (double)val[k] * z[col[k]];
    }
    acc += __shfl_xor(acc, 1, 16);
    acc += __shfl_xor(acc, 2, 16);
    acc += __shfl_xor(acc, 4, 16);
    acc += __shfl_xor(acc, 8, 16);
    if (row < n && sub == 0) zo[row] = z[row] + omega * (double)Dinv[row] * (v[row] - acc);
}

// bs in {3, 6}: SPMV_R block rows per wavefront (bsr_rows.h), lanes 0..bs-1
// finish the rows.  Values FP64 or a BF16 copy (the arithmetic FP64).
template <int BS, typename TV>
__global__ __launch_bounds__(256) void k_jsweep_rows(int64_t n, const int32_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ col, const TV *__restrict__ val,
                                                     const double *__restrict__ Dinv, double omega,
                                                     const double *__restrict__ v, const double *__restrict__ z,
                                                     double *__restrict__ zo, const int32_t *active)
{
    const int64_t w = (int64_t)blockIdx.x * 4 + wave_id();
    int64_t row[SPMV_R];
#pragma unroll
    for (int q = 0; q < SPMV_R; ++q) row[q] = w * SPMV_R + q;
    int k0[SPMV_R], k1[SPMV_R];
    row_extents<SPMV_R>(row, n, rowptr, k0, k1);
    if (*active == 0 || row[0] >= n) return;
    const int lane = threadIdx.x & 63;
    const int rl = lane < BS ? lane : 0;
    double vr[SPMV_R], zr[SPMV_R], d[SPMV_R][BS], az[SPMV_R];
#pragma unroll
    for (int q = 0; q < SPMV_R; ++q) {
        const int64_t rr = row[q] < n ? row[q] : row[0];
        vr[q] = v[rr * BS + rl];
        zr[q] = z[rr * BS + rl];
        RowLoad<BS, double, false>::get(Dinv + (rr * BS + rl) * BS, d[q]);
    }
    bsr_rows_dot<BS, TV, SPMV_R, false>(k0, k1, col, val, z, lane, az);
#pragma unroll
    for (int q = 0; q < SPMV_R; ++q) {
        const double res = vr[q] - az[q];
        double u = 0.0;
#pragma unroll
        for (int c = 0; c < BS; ++c) u += d[q][c] * __shfl(res, c, 64);
        if (lane < BS && row[q] < n) zo[row[q] * BS + lane] = zr[q] + omega * u;
    }
}

// ------------------------------------------- compact B-system blocks ----

// A block of a B (left Cauchy-Green) band system is s1 I - LE(M): the
// scalar s1 and the D x D matrix M (1 + D*D numbers, the assembly's
// accumulators) define all NV x NV entries, and (LE(M) x)_c = (M X + X M^T)_ij
// for the Voigt pair (i, j) of c, X the symmetric tensor of x (Voigt order
// 11, 22, 33, 12, 23, 13 / 11, 22, 12).  The products read this compact form
// (80 instead of 288 bytes per 6x6 block) and expand it on the fly, in FP64.
template <int D> struct BCmp {
    static constexpr int NV = D == 3 ? 6 : 3, NC = 1 + D * D;
};

template <int D>
__device__ __forceinline__ void bcmp_block_apply(const double (&cm)[BCmp<D>::NC], const double (&xv)[BCmp<D>::NV],
                                                 double (&acc)[BCmp<D>::NV])
{
    constexpr int NV = BCmp<D>::NV;
    double X[D][D];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        int i, j;
        vpair<D>(c, i, j);
        X[i][j] = xv[c];
        X[j][i] = xv[c];
    }
    double MX[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) t += cm[1 + i * D + k] * X[k][j];
            MX[i][j] = t;
        }
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        int i, j;
        vpair<D>(c, i, j);
        acc[c] += cm[0] * xv[c] - (MX[i][j] + MX[j][i]);
    }
}

// (A z) of the segment's block row, one compact block per lane, reduced
// over the segment (every lane of it holds the row's sums)
template <int D, int SEG, typename TC = double>
__device__ __forceinline__ void bcmp_row_dot(int k0, int k1, const int32_t *__restrict__ col,
                                             const TC *__restrict__ cmp, const double *__restrict__ z, int j,
                                             double (&acc)[BCmp<D>::NV])
{
    constexpr int NV = BCmp<D>::NV, NC = BCmp<D>::NC;
#pragma unroll
    for (int c = 0; c < NV; ++c) acc[c] = 0.0;
    for (int k = k0 + j; k < k1; k += SEG) {
        double cm[NC], xv[NV];
        RowLoad<NC, TC, false>::get(cmp + (int64_t)k * NC, cm);
        x_get<NV>(z, col[k], xv);
        bcmp_block_apply<D>(cm, xv, acc);
    }
#pragma unroll
    for (int s = SEG / 2; s > 0; s >>= 1)
#pragma unroll
        for (int c = 0; c < NV; ++c) acc[c] += __shfl_xor(acc[c], s, 64);
}

template <int D>
__global__ __launch_bounds__(256) void k_spmv_bcmp(int64_t n, const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ col, const double *__restrict__ cmp,
                                                   const double *__restrict__ x, double *__restrict__ y,
                                                   const int32_t *active)
{
    constexpr int NV = BCmp<D>::NV, SEG = BlockSeg<NV>::SEG, RPW = BlockSeg<NV>::RPW;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave_id()) * RPW;
    if ((active && *active == 0) || row0 >= n) return;
    const int lane = threadIdx.x & 63, q = lane / SEG, j = lane - q * SEG;
    int k0, k1;
    seg_extents<RPW>(row0, n, rowptr, q, k0, k1);
    double acc[NV];
    bcmp_row_dot<D, SEG>(k0, k1, col, cmp, x, j, acc);
    const int64_t row = row0 + q;
#pragma unroll
    for (int c = 0; c < NV; ++c)
        if (j == c && row < n) y[row * NV + c] = acc[c];
}

// damped block-Jacobi sweep zo = z + omega D^-1 (v - A z), lane j < NV of a
// row's segment finishes component j (compact blocks and inverses FP64 or
// FP32 copies, the arithmetic FP64)
template <int D, typename TC>
__global__ __launch_bounds__(256) void k_jsweep_bcmp(int64_t n, const int32_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ col, const TC *__restrict__ cmp,
                                                     const TC *__restrict__ Dinv, double omega,
                                                     const double *__restrict__ v, const double *__restrict__ z,
                                                     double *__restrict__ zo, const int32_t *active)
{
    constexpr int NV = BCmp<D>::NV, SEG = BlockSeg<NV>::SEG, RPW = BlockSeg<NV>::RPW;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave_id()) * RPW;
    if (*active == 0 || row0 >= n) return;
    const int lane = threadIdx.x & 63, q = lane / SEG, j = lane - q * SEG;
    const int64_t row = row0 + q, rr = row < n ? row : row0;   // rr: in bounds, unused past n
    const int jj = j < NV ? j : 0;
    double vv[NV], d[NV];
    x_get<NV>(v, rr, vv);
    RowLoad<NV, TC, false>::get(Dinv + (rr * NV + jj) * NV, d);
    const double zr = z[rr * NV + jj];
    int k0, k1;
    seg_extents<RPW>(row0, n, rowptr, q, k0, k1);
    double az[NV];
    bcmp_row_dot<D, SEG, TC>(k0, k1, col, cmp, z, j, az);
    double u = 0.0;
#pragma unroll
    for (int c = 0; c < NV; ++c) u += d[c] * (vv[c] - az[c]);
    if (j < NV && row < n) zo[row * NV + j] = zr + omega * u;
}

template <typename TD> static eft_status bj_setup(eft_ctx *ctx, const eft_matrix *A, TD *Dinv, int32_t *sing)
{
    if (A->n == 0) return EFT_OK;
    if (A->bs > 8) {
        ctx->err = "block size above 8";
        return EFT_EINVAL;
    }
    const dim3 g(eft_grid(A->n, 256)), t(256);
    auto fixed = [&](auto bsc) {
        constexpr int BS = decltype(bsc)::value;
        if (A->fp32)
            hipLaunchKernelGGL((k_bj_setup_t<BS, float, TD>), g, t, 0, ctx->stream, A->n, A->diag, A->val32, Dinv,
                               sing);
        else
            hipLaunchKernelGGL((k_bj_setup_t<BS, double, TD>), g, t, 0, ctx->stream, A->n, A->diag, A->val, Dinv,
                               sing);
    };
    if (A->bs == 3) fixed(std::integral_constant<int, 3>{});
    else if (A->bs == 4) fixed(std::integral_constant<int, 4>{});
    else if (A->bs == 6) fixed(std::integral_constant<int, 6>{});
    else if (A->fp32)
        hipLaunchKernelGGL((k_bj_setup<float, TD>), g, t, 0, ctx->stream, A->n, A->bs, A->diag, A->val32, Dinv,
                           sing);
    else
        hipLaunchKernelGGL((k_bj_setup<double, TD>), g, t, 0, ctx->stream, A->n, A->bs, A->diag, A->val, Dinv,
                           sing);
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}

eft_status eft_bj_setup(eft_ctx *ctx, const eft_matrix *A, double *Dinv, int32_t *sing)
{
    return bj_setup<double>(ctx, A, Dinv, sing);
}

eft_status eft_bj_setup32(eft_ctx *ctx, const eft_matrix *A, float *Dinv, int32_t *sing)
{
    return bj_setup<float>(ctx, A, Dinv, sing);
}

eft_status eft_bj_apply(eft_ctx *ctx, int bs, int64_t n, const double *Dinv, const double *x, double *z,
                        const int32_t *active)
{
    const int64_t nd = n * bs;
    if (nd == 0) return EFT_OK;
    hipLaunchKernelGGL(k_bj_apply<double>, dim3(eft_grid(nd, 256)), dim3(256), 0, ctx->stream, nd, bs, Dinv, 1.0, x,
                       z, active);
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}

eft_status eft_jacobi_apply(eft_ctx *ctx, const eft_matrix *A, const double *Dinv, const double *v, double *z,
                            double *tmp, int sweeps, double omega, const int32_t *active)
{
    const int bs = A->bs;
    const int64_t n = A->n, nd = n * bs;
    if (nd == 0) return EFT_OK;
    const bool sweepable = !A->fp32 && (bs == 1 || bs == 3 || bs == 6);
    if (sweeps < 1 || (sweeps > 1 && !sweepable)) {
        ctx->err = "Jacobi sweeps need FP64 values and bs 1, 3 or 6";
        return EFT_EINVAL;
    }
    // FP32 copies of the values (or compact blocks) and block inverses
    const bool narrow = eft_jacobi_narrow(A);
    // sweep s writes z when (sweeps - 1 - s) is even, tmp otherwise, so the
    // last one ends in z
    double *buf[2] = {z, tmp};
    double *cur = buf[(sweeps - 1) & 1];
    if (narrow)
        hipLaunchKernelGGL(k_bj_apply<float>, dim3(eft_grid(nd, 256)), dim3(256), 0, ctx->stream, nd, bs, A->dinv32,
                           omega, v, cur, active);
    else
        hipLaunchKernelGGL(k_bj_apply<double>, dim3(eft_grid(nd, 256)), dim3(256), 0, ctx->stream, nd, bs, Dinv,
                           omega, v, cur, active);
    for (int s = 1; s < sweeps; ++s) {
        double *nxt = buf[(sweeps - 1 - s) & 1];
        if (A->bcmp)
            EFT_TRY(eft_bcmp_sweep(ctx, A, Dinv, omega, v, cur, nxt, active));
        else if (bs == 1 && narrow)
            hipLaunchKernelGGL(k_jsweep1<float>, dim3(eft_grid(n, 16)), dim3(256), 0, ctx->stream, n, A->rowptr,
                               A->col, A->pc32, A->dinv32, omega, v, cur, nxt, active);
        else if (bs == 1)
            hipLaunchKernelGGL(k_jsweep1<double>, dim3(eft_grid(n, 16)), dim3(256), 0, ctx->stream, n, A->rowptr,
                               A->col, A->val, Dinv, omega, v, cur, nxt, active);
        else if (bs == 3)
            hipLaunchKernelGGL((k_jsweep_rows<3, double>), dim3(eft_grid(n, 4 * SPMV_R)), dim3(256), 0, ctx->stream,
                               n, A->rowptr, A->col, A->val, Dinv, omega, v, cur, nxt, active);
        else
            hipLaunchKernelGGL((k_jsweep_rows<6, double>), dim3(eft_grid(n, 4 * SPMV_R)), dim3(256), 0, ctx->stream,
                               n, A->rowptr, A->col, A->val, Dinv, omega, v, cur, nxt, active);
        cur = nxt;
    }
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}

eft_status eft_bcmp_spmv(eft_ctx *ctx, const eft_matrix *A, const double *x, double *y, const int32_t *active)
{
    const int64_t n = A->n;
    if (n == 0) return EFT_OK;
    if (A->bs == 6)
        hipLaunchKernelGGL(k_spmv_bcmp<3>, dim3(eft_grid(n, 4 * BlockSeg<6>::RPW)), dim3(256), 0, ctx->stream, n,
                           A->rowptr, A->col, A->bcmp, x, y, active);
    else if (A->bs == 3)
        hipLaunchKernelGGL(k_spmv_bcmp<2>, dim3(eft_grid(n, 4 * BlockSeg<3>::RPW)), dim3(256), 0, ctx->stream, n,
                           A->rowptr, A->col, A->bcmp, x, y, active);
    else {
        ctx->err = "compact B blocks need bs 3 or 6";
        return EFT_EINVAL;
    }
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}

eft_status eft_bcmp_sweep(eft_ctx *ctx, const eft_matrix *A, const double *Dinv, double omega, const double *v,
                          const double *z, double *zo, const int32_t *active)
{
    const int64_t n = A->n;
    if (n == 0) return EFT_OK;
    const bool narrow = eft_jacobi_narrow(A);
    auto go = [&](auto dc, auto tc, const auto *cmp, const auto *dinv) {
        constexpr int D = decltype(dc)::value, NV = BCmp<D>::NV;
        using TC = decltype(tc);
        hipLaunchKernelGGL((k_jsweep_bcmp<D, TC>), dim3(eft_grid(n, 4 * BlockSeg<NV>::RPW)), dim3(256), 0,
                           ctx->stream, n, A->rowptr, A->col, cmp, dinv, omega, v, z, zo, active);
    };
    if (A->bs == 6 && narrow)
        go(std::integral_constant<int, 3>{}, 0.0f, A->pc32, A->dinv32);
    else if (A->bs == 6)
        go(std::integral_constant<int, 3>{}, 0.0, A->bcmp, Dinv);
    else if (A->bs == 3 && narrow)
        go(std::integral_constant<int, 2>{}, 0.0f, A->pc32, A->dinv32);
    else if (A->bs == 3)
        go(std::integral_constant<int, 2>{}, 0.0, A->bcmp, Dinv);
    else {
        ctx->err = "compact B blocks need bs 3 or 6";
        return EFT_EINVAL;
    }
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}
