// Right-preconditioned FGMRES(m) with classical Gram-Schmidt and a second,
// conditional orthogonalization pass ("twice is enough": the pass runs only
// when the first one removed more than half of ||w||^2), FP64 throughout.
//
// Every kernel of an iteration reads a device flag and returns at once after
// convergence, so the host enqueues iterations in chunks and reads the status
// once per chunk; the Hessenberg column, Givens rotations and the triangular
// solve run in single-workgroup kernels (the column's bookkeeping is fused
// with the last reduction of its pass).  With at most 32 basis vectors the
// first pass's update also yields the second pass's dots, the first pass's
// closing kernel completes the column (with the second pass, ||w''||^2 is
// ||w'||^2 - ||h2||^2: the basis is orthonormal to working precision and the
// second pass removes little), and the second pass's update runs fused with
// the normalization of v_{j+1}.  Dot products reduce
// deterministically: each block writes a partial, a second kernel sums the
// partials in a fixed order.
#include <cstring>
#include <mutex>
#include <string>

#include "dev_common.h"
#include "eft_internal.h"

namespace {

constexpr int RB = 256;   // reduction block size
constexpr int KC = 8;     // vectors per multi-dot block
constexpr int MAXBLK = 4 * RB;   // most partials of one reduction (blocks of a reduction grid)

// This thread's share of the sum of p[0..nblk) (nblk <= MAXBLK): four
// unguarded loads at clamped indices, masked by a product, all in flight
// together.
__device__ __forceinline__ double part_share(const double *__restrict__ p, int nblk)
{
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < MAXBLK / RB; ++u) {
        const int b = threadIdx.x + u * RB;
        s += p[b < nblk ? b : nblk - 1] * (b < nblk ? 1.0 : 0.0);
    }
    return s;
}

// layout of KrylovWs::small (doubles) for restart m
struct Small {
    int m;
    __host__ __device__ int64_t H() const { return 0; }                        // [(m+1)][m]
    __host__ __device__ int64_t cs() const { return (int64_t)(m + 1) * m; }    // [m]
    __host__ __device__ int64_t sn() const { return cs() + m; }                // [m]
    __host__ __device__ int64_t g() const { return sn() + m; }                 // [m+1]
    __host__ __device__ int64_t y() const { return g() + m + 1; }              // [m]
    __host__ __device__ int64_t h() const { return y() + m; }                  // [m+2] dots, then ||w||^2
    __host__ __device__ int64_t h2() const { return h() + m + 2; }             // [m+2]
    __host__ __device__ int64_t sc() const { return h2() + m + 2; }            // [8] scalars
    __host__ __device__ int64_t size() const { return sc() + 8; }
};
// scalars: sc+0 ||w'||^2 (after pass 1), sc+1 ||w''||^2, sc+2 tol_abs, sc+3 beta,
// sc+4 H[j+1][j] before the rotation, sc+5 |g[j+1]| (residual estimate)
// flags: 0 active, 1 columns done in this cycle, 2 breakdown, 3 second-pass gate

// dots of w with V[0..nvec-1] (and w.w as index nvec when with_ww): partials
__global__ __launch_bounds__(RB) void k_mdot(const double *__restrict__ V, int64_t nd, int nvec, int with_ww,
                                             const double *__restrict__ w, double *__restrict__ part, int nblk,
                                             const int32_t *flag, int gated)
{
    __shared__ double lds[RB / 64];
    if (flag[0] == 0 || (gated && flag[3] == 0)) return;
    const int k0 = blockIdx.y * KC;
    const int ntot = nvec + with_ww;
    // every slot loads a basis vector (clamped index) and is masked by a
    // product, so that the KC loads of an element are in flight together
    // rather than each behind its own branch
    const double *vk[KC];
    double mv[KC], mw[KC], acc[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const int k = k0 + kk;
        vk[kk] = V + (int64_t)(k < nvec ? k : nvec - 1) * nd;
        mv[kk] = k < nvec ? 1.0 : 0.0;
        mw[kk] = (k == nvec && with_ww) ? 1.0 : 0.0;
        acc[kk] = 0.0;
    }
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < nd; i += (int64_t)nblk * RB) {
        const double wi = w[i];
        double v[KC];
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) v[kk] = vk[kk][i];
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) acc[kk] += (v[kk] * mv[kk] + wi * mw[kk]) * wi;
    }
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const double s = block_sum<RB>(acc[kk], lds);
        const int k = k0 + kk;
        if (threadIdx.x == 0 && k < ntot) part[(int64_t)k * nblk + blockIdx.x] = s;
    }
}

// out[k] = sum of part[k][*], grid = number of sums
__global__ __launch_bounds__(RB) void k_sum_parts(const double *__restrict__ part, int nblk, double *__restrict__ out,
                                                  const int32_t *flag, int gated)
{
    __shared__ double lds[RB / 64];
    if (flag && (flag[0] == 0 || (gated && flag[3] == 0))) return;
    double s = part_share(part + (int64_t)blockIdx.x * nblk, nblk);
    s = block_sum<RB>(s, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// w -= sum_k c[k] V[k] (sign = -1) or x += sum_k c[k] V[k] (sign = +1);
// partial sums of the squared result when part != nullptr
__global__ __launch_bounds__(RB) void k_maxpy(const double *__restrict__ V, int64_t nd, int nvec,
                                              const double *__restrict__ c, double sign, double *__restrict__ w,
                                              double *__restrict__ part, int nblk, const int32_t *flag, int gated)
{
    __shared__ double cl[EFT_MAX_RESTART + 2];
    __shared__ double lds[RB / 64];
    if (flag && (flag[0] == 0 || (gated && flag[3] == 0))) return;
    for (int k = threadIdx.x; k < nvec; k += RB) cl[k] = sign * c[k];
    __syncthreads();
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < nd; i += (int64_t)nblk * RB) {
        double s = w[i];
        for (int k = 0; k < nvec; ++k) s += cl[k] * V[(int64_t)k * nd + i];
        w[i] = s;
        acc += s * s;
    }
    if (part) {
        const double t = block_sum<RB>(acc, lds);
        if (threadIdx.x == 0) part[blockIdx.x] = t;
    }
}

// The first pass's update w' = w - sum_k c[k] V[k] fused with the second
// pass's dots V[k].w' and ||w'||^2: each lane keeps its entries of the nvec
// (<= NV) basis vectors in registers, so V is read once for both.  Partials:
// part[b] = ||w'||^2 of block b, part[(1 + k) nblk + b] = its V[k].w'.
template <int NV>
__global__ __launch_bounds__(RB) void k_maxpy_mdot(const double *__restrict__ V, int64_t nd, int nvec,
                                                   const double *__restrict__ c, double *__restrict__ w,
                                                   double *__restrict__ part, int nblk, const int32_t *flag)
{
    __shared__ double cl[NV];
    __shared__ double red[RB / 64][NV + 1];
    if (flag[0] == 0) return;
    for (int k = threadIdx.x; k < NV; k += RB) cl[k] = k < nvec ? -c[k] : 0.0;
    __syncthreads();
    double acc[NV + 1];
#pragma unroll
    for (int k = 0; k <= NV; ++k) acc[k] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < nd; i += (int64_t)nblk * RB) {
        double v[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = k < nvec ? V[(int64_t)k * nd + i] : 0.0;
        double s = w[i];
#pragma unroll
        for (int k = 0; k < NV; ++k)
            if (k < nvec) s += cl[k] * v[k];
        w[i] = s;
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] += v[k] * s;
        acc[NV] += s * s;
    }
    const int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
#pragma unroll
    for (int k = 0; k <= NV; ++k) {
        const double t = wave_sum(acc[k]);
        if (ln == 0) red[wv][k] = t;
    }
    __syncthreads();
    const int k = threadIdx.x;
    if (k < nvec || k == NV) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < RB / 64; ++q) t += red[q][k];
        part[(k == NV ? 0 : (int64_t)(1 + k) * nblk) + blockIdx.x] = t;
    }
}

// Givens update of column j (col[0..j+1], in LDS), residual estimate,
// convergence and breakdown flags; one thread.  cs, sn are the earlier
// rotations (LDS copies); the new rotation, g and the column go to small.
__device__ void givens_column(double *small, int m, int j, double *col, const double *csl, const double *snl,
                              int32_t *flag)
{
    Small L{m};
    double *H = small + L.H(), *cs = small + L.cs(), *sn = small + L.sn(), *g = small + L.g();
    for (int i = 0; i < j; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = csl[i] * a + snl[i] * b;
        col[i + 1] = -snl[i] * a + csl[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double hn = b;
    small[L.sc() + 4] = hn;   // ||w||, kept for the normalization of v_{j+1}
    const double den = sqrt(a * a + b * b);
    const double c = den == 0.0 ? 1.0 : a / den, sv = den == 0.0 ? 0.0 : b / den;
    cs[j] = c;
    sn[j] = sv;
    col[j] = c * a + sv * b;
    col[j + 1] = 0.0;
    for (int i = 0; i <= j + 1; ++i) H[(int64_t)i * m + j] = col[i];
    const double gj = g[j];
    g[j + 1] = -sv * gj;
    g[j] = c * gj;
    small[L.sc() + 5] = fabs(g[j + 1]);   // residual estimate after column j
    flag[1] = j + 1;
    const double tol = small[L.sc() + 2];
    if (!(fabs(g[j + 1]) > tol)) flag[0] = 0;  // converged (or NaN)
    if (hn == 0.0) {
        flag[0] = 0;
        flag[2] = 1;
    }
    if (j + 1 >= m) flag[0] = 0;
}

// End of an orthogonalization pass of column j (one workgroup): ||w||^2
// from the update's partials, then pass 1 stores the dots as the column and
// decides on pass 2 (taken when pass 1 removed more than half of ||w||^2);
// the pass that completes the column sets H[j+1][j] = ||w|| and applies the
// Givens rotations.  The column and the earlier rotations are staged in LDS
// by the whole workgroup, so the serial rotation loop reads no global memory.
// With ndots > 0 (pass 1 fused with the second pass's dots) it also sums the
// ndots dot partials that follow the norm partials into h2, one wavefront
// per dot.
__global__ __launch_bounds__(RB) void k_close_pass(const double *__restrict__ part, int nblk, int ndots, double *small,
                                                   int m, int j, int pass, int32_t *flag)
{
    __shared__ double lds[RB / 64];
    __shared__ double col[EFT_MAX_RESTART + 2], csl[EFT_MAX_RESTART], snl[EFT_MAX_RESTART];
    if (flag[0] == 0 || (pass == 2 && flag[3] == 0)) return;
    __shared__ double red[RB / 64][32];
    Small L{m};
    if (ndots > 0) {
        // (ndots <= 32) eight dots at a time, their loads issued together
        const int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
        for (int k0 = 0; k0 < ndots; k0 += 8) {
            double t[8];
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                // unguarded loads at clamped indices, masked by a product
                // (dots past ndots are summed and never read), so that the
                // 32 loads are in flight together
                const int k = k0 + kk;
                t[kk] = part_share(part + (int64_t)(1 + (k < ndots ? k : ndots - 1)) * nblk, nblk);
            }
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                const double v = wave_sum(t[kk]);
                if (ln == 0) red[wv][k0 + kk] = v;   // (k0 + kk < 32)
            }
        }
    }
    double *H = small + L.H();
    const double *h = small + L.h(), *h2 = small + L.h2();
    for (int i = threadIdx.x; i <= j; i += RB) {
        col[i] = pass == 1 ? h[i] : H[(int64_t)i * m + j] + h2[i];
        if (i < j) {
            csl[i] = small[L.cs() + i];
            snl[i] = small[L.sn() + i];
        }
    }
    double s = part_share(part, nblk);
    s = block_sum<RB>(s, lds);   // (its barriers also publish col, csl, snl, red)
    __shared__ double hh2[32];
    if (ndots > 0) {
        if ((int)threadIdx.x < ndots) {
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < RB / 64; ++q) v += red[q][threadIdx.x];
            small[L.h2() + threadIdx.x] = v;
            hh2[threadIdx.x] = v;
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    if (pass == 1 && ndots > 0) {
        // the second pass's dots are known, so this pass completes the
        // column either way: with the second pass, the column gains its
        // dots and ||w''||^2 = ||w'||^2 - ||h2||^2 (the basis is orthonormal
        // and the second pass removes little), and the second pass's update
        // runs fused with the normalization
        small[L.sc() + 0] = s;
        flag[3] = (s < 0.5 * h[j + 1]) ? 1 : 0;
        if (flag[3]) {
            double q = 0.0;
            for (int i = 0; i <= j; ++i) {
                col[i] += hh2[i];
                q += hh2[i] * hh2[i];
            }
            // ||w''||^2 by subtraction keeps its digits while s - q is not
            // far below s; below 1e-8 s it would be mostly rounding, and
            // w'' is then within 1e-4 of the span of the basis: the column
            // ends the cycle as a breakdown (H[j+1][j] = 0), and the restart
            // from the true residual takes over
            s = (s - q > 1e-8 * s) ? s - q : 0.0;
            small[L.sc() + 1] = s;
        }
    } else if (pass == 1) {
        small[L.sc() + 0] = s;
        flag[3] = (s < 0.5 * h[j + 1]) ? 1 : 0;
        if (flag[3]) {   // pass 2 completes the column: store the dots
            for (int i = 0; i <= j; ++i) H[(int64_t)i * m + j] = col[i];
            return;
        }
    } else {
        small[L.sc() + 1] = s;
    }
    col[j + 1] = sqrt(s);
    givens_column(small, m, j, col, csl, snl, flag);
}

// v_{j+1} = (w - sum_k h2[k] V[k]) / H[j+1][j], the update only when the
// second pass was taken (nvec <= 32)
__global__ __launch_bounds__(RB) void k_update_normalize(const double *__restrict__ V, int64_t nd, int nvec,
                                                         const double *__restrict__ w, double *__restrict__ v,
                                                         const double *small, int m, const int32_t *flag)
{
    __shared__ double cl[32];
    if (flag[0] == 0) return;
    Small L{m};
    const double inv = 1.0 / small[L.sc() + 4];
    const int nv = flag[3] ? nvec : 0;
    for (int k = threadIdx.x; k < nv; k += RB) cl[k] = -small[L.h2() + k];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < nd; i += (int64_t)gridDim.x * RB) {
        double s = w[i];
        for (int k = 0; k < nv; ++k) s += cl[k] * V[(int64_t)k * nd + i];
        v[i] = s * inv;
    }
}

// v_{j+1} = w / H[j+1][j]
__global__ __launch_bounds__(RB) void k_normalize(const double *__restrict__ w, double *__restrict__ v, int64_t nd,
                                                  const double *small, int m, int j, const int32_t *flag)
{
    if (flag[0] == 0) return;
    Small L{m};
    const double inv = 1.0 / small[L.sc() + 4];
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < nd; i += (int64_t)gridDim.x * RB) v[i] = w[i] * inv;
}

// y = H^-1 g (upper triangular, jj columns)
// Back substitution H[0..jj)[0..jj) y = g on one wavefront: row by row from
// the last, the lanes share the dot product of row i with the known part of
// y (a shuffle tree), y kept in LDS.
__global__ __launch_bounds__(64) void k_trisolve(double *small, int m, const int32_t *flag)
{
    __shared__ double ys[EFT_MAX_RESTART];
    Small L{m};
    const int jj = flag[1];
    const double *H = small + L.H(), *g = small + L.g();
    double *y = small + L.y();
    const int l = threadIdx.x;
    for (int i = jj - 1; i >= 0; --i) {
        double s = 0.0;
        for (int k = i + 1 + l; k < jj; k += 64) s += H[(int64_t)i * m + k] * ys[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (l == 0) ys[i] = (g[i] - s) / H[(int64_t)i * m + i];
        __syncthreads();
    }
    for (int i = l; i < jj; i += 64) y[i] = ys[i];
}

// flags of a solve, before its first cycle
__global__ void k_clear_flags(int32_t *flag)
{
    if (threadIdx.x < 8) flag[threadIdx.x] = 0;
}

// start of a cycle: v0 = r / beta, g = (beta, 0, ...), flags
__global__ __launch_bounds__(RB) void k_start_cycle(const double *__restrict__ r, double *__restrict__ v0, int64_t nd,
                                                    double *small, int m, double beta, double tol, int32_t *flag)
{
    Small L{m};
    const double inv = 1.0 / beta;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < nd; i += (int64_t)gridDim.x * RB) v0[i] = r[i] * inv;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double *g = small + L.g();
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        small[L.sc() + 2] = tol;
        flag[0] = 1;
        flag[1] = 0;
        flag[2] = 0;
        flag[3] = 0;
    }
}

// r = b - r
__global__ __launch_bounds__(RB) void k_bmr(const double *__restrict__ b, double *__restrict__ r, int64_t nd)
{
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < nd; i += (int64_t)gridDim.x * RB) r[i] = b[i] - r[i];
}

__global__ __launch_bounds__(RB) void k_norm_part(const double *__restrict__ x, int64_t nd, double *part, int nblk)
{
    __shared__ double lds[RB / 64];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < nd; i += (int64_t)nblk * RB) acc += x[i] * x[i];
    acc = block_sum<RB>(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

int nblk_for(int64_t nd) { return (int)std::max<int64_t>(1, std::min<int64_t>(MAXBLK, (nd + RB - 1) / RB)); }
int stream_grid(int64_t nd) { return (int)std::max<int64_t>(1, std::min<int64_t>(8192, (nd + RB - 1) / RB)); }

}  // namespace

eft_status eft_krylov_reserve(eft_ctx *ctx, int64_t n, int bs, int m)
{
    KrylovWs &K = ctx->kw;
    const int64_t nd = n * bs;
    if (m > EFT_MAX_RESTART) {
        ctx->err = "restart above 512";
        return EFT_EINVAL;
    }
    if (nd <= K.cap_nd && m <= K.cap_m && n <= K.cap_n && bs * bs * n <= K.cap_bs * K.cap_bs * K.cap_n) return EFT_OK;
    if (ctx->no_alloc) {
        ctx->err = "the Krylov workspace would have to grow inside an allocation-free call";
        return EFT_ENOMEM;
    }
    const int64_t cnd = std::max(nd, K.cap_nd);
    const int cm = std::max(m, K.cap_m);
    const int64_t cn = std::max(n, K.cap_n);
    const int cbs = std::max(bs, K.cap_bs);
    auto fr = [](void *p) {
        if (p) (void)hipFree(p);
    };
    fr(K.V); fr(K.Z); fr(K.w); fr(K.r); fr(K.Dinv); fr(K.part); fr(K.small); fr(K.flag);
    K = KrylovWs{};
    Small L{cm};
    const int nblk = nblk_for(cnd);
    if (hipMalloc(&K.V, sizeof(double) * cnd * (cm + 1)) != hipSuccess ||
        hipMalloc(&K.Z, sizeof(double) * cnd * cm) != hipSuccess || hipMalloc(&K.w, sizeof(double) * cnd) != hipSuccess ||
        hipMalloc(&K.r, sizeof(double) * cnd) != hipSuccess ||
        hipMalloc(&K.Dinv, sizeof(double) * cn * cbs * cbs) != hipSuccess ||
        hipMalloc(&K.part, sizeof(double) * (int64_t)nblk * (cm + 2)) != hipSuccess ||
        hipMalloc(&K.small, sizeof(double) * L.size()) != hipSuccess ||
        hipMalloc(&K.flag, sizeof(int32_t) * 8) != hipSuccess) {
        ctx->err = "out of device memory for the Krylov workspace";
        return EFT_ENOMEM;
    }
    K.cap_nd = cnd;
    K.cap_m = cm;
    K.cap_n = cn;
    K.cap_bs = cbs;
    K.nblk = nblk;
    return EFT_OK;
}

static eft_status sum_to_host(eft_ctx *ctx, const double *part, int nblk, int count, double *host)
{
    hipLaunchKernelGGL(k_sum_parts, dim3(count), dim3(RB), 0, ctx->stream, part, nblk, ctx->dscal,
                       (const int32_t *)nullptr, 0);
    EFT_HIP(hipGetLastError());
    EFT_HIP(hipMemcpyAsync(ctx->hscal, ctx->dscal, sizeof(double) * count, hipMemcpyDeviceToHost, ctx->stream));
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < count; ++i) host[i] = ctx->hscal[i];
    return EFT_OK;
}

eft_status eft_norm2(eft_ctx *ctx, const double *x, int64_t n, double *out_host)
{
    if (n == 0) {
        *out_host = 0.0;
        return EFT_OK;
    }
    const int nblk = nblk_for(n);
    hipLaunchKernelGGL(k_norm_part, dim3(nblk), dim3(RB), 0, ctx->stream, x, n, ctx->red, nblk);
    EFT_HIP(hipGetLastError());
    double s;
    EFT_TRY(sum_to_host(ctx, ctx->red, nblk, 1, &s));
    *out_host = sqrt(s);
    return EFT_OK;
}

// Solve A x = b (x0 = 0).  The preconditioner is the point-block Jacobi of A.
// Algorithmic bytes of one SpMV: values, column indices, row pointers, x
// read and y written once.
static double spmv_bytes(const eft_matrix *A)
{
    // (in stencil form the row masks replace the column indices)
    const double vb = A->fp32 ? 4.0 : 8.0, b2 = (double)A->bs * A->bs;
    const bool stn = A->stn_mask && (A->bs == 3 || A->bs == 4);
    const double cols = stn ? (double)A->n * 2.0 : (double)A->nnzb * 4.0;
    return (double)A->nnzb * b2 * vb + cols + (double)(A->n + 1) * 4.0 + 2.0 * A->n * A->bs * 8.0;
}

// Enqueue column j of a momentum solve as a HIP graph: captured from the
// column's launches the first time, replayed afterwards.  The cache holds one
// graph per column index and belongs to the parameters, the Krylov workspace
// and the matrix arrays it was captured on; any change drops it.
template <typename F>
static eft_status column_graph(eft_ctx *ctx, const eft_matrix *A, int j, int m, int64_t nd, F &column)
{
    auto &G = ctx->colg;
    const KrylovWs &K = ctx->kw;
    const MGLevel &F0 = ctx->mg[0];
    const std::vector<const void *> key = {K.V, K.Z, K.w, K.part, K.small, K.flag, A->val, A->val32,
                                           F0.A.val16, F0.A.val32, (const void *)(intptr_t)nd,
                                           (const void *)(intptr_t)m};
    if (G.key != key || std::memcmp(&G.par, &ctx->par, sizeof(eft_params)) != 0 || (int)G.exec.size() != m) {
        for (hipGraphExec_t g : G.exec)
            if (g) EFT_HIP(hipGraphExecDestroy(g));
        G.exec.assign(m, nullptr);
        G.key = key;
        G.par = ctx->par;
    }
    if (!G.exec[j]) {
        // recorded on the context's own capture stream (the null stream
        // cannot be captured): the column enqueues on ctx->stream, which
        // points there while recording; nothing executes until the launch
        if (!G.cap) EFT_HIP(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        const hipStream_t s0 = ctx->stream;
        const hipError_t be = hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal);
        if (be != hipSuccess) EFT_HIP(be);
        ctx->stream = G.cap;
        const eft_status st = column(j);
        const hipError_t e = hipStreamEndCapture(G.cap, &g);
        ctx->stream = s0;
        if (st != EFT_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        EFT_HIP(e);
        hipGraphExec_t x = nullptr;
        const hipError_t ie = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        EFT_HIP(ie);
        G.exec[j] = x;
    }
    EFT_HIP(hipGraphLaunch(G.exec[j], ctx->stream));
    return EFT_OK;
}

eft_status eft_fgmres_dev(eft_ctx *ctx, const eft_matrix *A, const double *b, double *x, eft_solve_info *info,
                          double rtol)
{
    const int bs = A->bs;
    const int64_t n = A->n, nd = n * bs;
    const int m = std::max(1, std::min(ctx->par.restart, EFT_MAX_RESTART));
    eft_solve_info inf{};
    inf.rel_res0 = 1.0;
    EFT_TRY(eft_krylov_reserve(ctx, n, bs, m));
    KrylovWs &K = ctx->kw;
    Small L{m};
    const int nblk = nblk_for(nd), sg = stream_grid(nd);
    EFT_TRY(eft_fill(ctx, x, nd, 0.0));
    double bnorm;
    EFT_TRY(eft_norm2(ctx, b, nd, &bnorm));
    if (!std::isfinite(bnorm)) {
        ctx->err = "non-finite right-hand side";
        return EFT_ENAN;
    }
    if (bnorm == 0.0) {
        inf.converged = 1;
        inf.rel_res = 0.0;
        if (info) *info = inf;
        return EFT_OK;
    }
    // the multigrid V-cycle (hierarchy refreshed by the assembly): the
    // preconditioner with precond = 1, the learned one's base with nn_base = 1
    const bool mg = eft_mg_active(ctx, A);
    inf.fallback_used = (ctx->par.precond == 1 && A == &ctx->J && !mg) ? 1 : 0;
    // learned preconditioner on the momentum system (block Jacobi elsewhere)
    bool learned = ctx->par.precond == 2 && A == &ctx->J;
    const bool nn_mg = learned && ctx->par.nn_base == 1;
    if (learned && !ctx->net.ready) {
        ctx->err = "precond = 2 needs eft_nn_init (learned preconditioner parameters)";
        return EFT_EINVAL;
    }
    if (nn_mg && !mg) {
        ctx->err = "nn_base = 1 needs the multigrid hierarchy (a structured Kuhn mesh, assembled)";
        return EFT_EINVAL;
    }
    const int maxit = std::max(1, ctx->par.lin_maxit);
    // past this many iterations a learned-preconditioned solve continues with
    // its base (block Jacobi or the V-cycle), its fallback (FGMRES admits the
    // change between columns)
    const int nn_budget = ctx->par.nn_maxit > 0 ? ctx->par.nn_maxit : std::max(1, maxit / 2);
    // training pairs (base of A z_j, z_j) from the momentum solves
    NNState &NS = ctx->net;
    const bool harvest = NS.cap_pairs > 0 && A == &ctx->J;
    if (harvest && ctx->par.nn_base == 1 && !mg) {
        ctx->err = "harvesting for nn_base = 1 needs the multigrid hierarchy";
        return EFT_EINVAL;
    }
    hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, ctx->stream, K.flag);
    // block ILU(0) on the momentum system (point-block Jacobi elsewhere)
    const bool ilu = ctx->par.precond == 3 && A == &ctx->J;
    if (ilu) EFT_TRY(eft_ilu_setup(ctx, A, K.flag + 6));
    if (eft_jacobi_narrow(A))
        EFT_TRY(eft_bj_setup32(ctx, A, A->dinv32, K.flag + 6));
    else if ((!mg && !ilu) || (harvest && ctx->par.nn_base == 0))
        EFT_TRY(eft_bj_setup(ctx, A, K.Dinv, K.flag + 6));
    const double tol = (rtol > 0.0 ? rtol : ctx->par.lin_rtol) * bnorm;
    int chunk = 8;   // columns enqueued between two reads of the solver state
    int total = 0;
    double *small = K.small;
    eft_status st = EFT_ENOTCONV;
    // first residual: r = b
    EFT_HIP(hipMemcpyAsync(K.r, b, sizeof(double) * nd, hipMemcpyDeviceToDevice, ctx->stream));
    double beta = bnorm;
    // one column j of the Arnoldi process: preconditioner, product and
    // orthogonalization (every kernel gated by the device flags)
    auto column = [&](int j) -> eft_status {
        double *vj = K.V + (int64_t)j * nd, *zj = K.Z + (int64_t)j * nd;
        ctx->kt.tag = j;
        if (learned)
            EFT_TRY(eft_nn_precond(ctx, K.Dinv, vj, zj, K.flag));
        else if (mg)
            EFT_TRY(eft_mg_vcycle(ctx, vj, zj, K.flag));
        else if (ilu)
            EFT_TRY(eft_ilu_apply(ctx, vj, zj, K.flag));
        else if (A == &ctx->J)
            EFT_TRY(eft_bj_apply(ctx, bs, n, K.Dinv, vj, zj, K.flag));
        else   // band systems (w is free until the product below)
            EFT_TRY(eft_jacobi_apply(ctx, A, K.Dinv, vj, zj, K.w, ctx->par.band_sweeps, ctx->par.band_omega,
                                     K.flag));
        const int64_t slot = A == &ctx->J ? eft_kt_begin(ctx, EFT_KT_SPMV) : -1;
        EFT_TRY(eft_spmv_flag(ctx, A, zj, K.w, K.flag));
        eft_kt_end(ctx, slot, spmv_bytes(A), EFT_KT_SPMV);
        if (harvest) EFT_TRY(eft_nn_store_pair(ctx, K.Dinv, K.w, zj, (NS.next + j) % NS.cap_pairs, K.flag));
        // pass 1: dots with V[0..j] and ||w||^2
        dim3 g1(nblk, (j + 2 + KC - 1) / KC);
        hipLaunchKernelGGL(k_mdot, g1, dim3(RB), 0, ctx->stream, K.V, nd, j + 1, 1, K.w, K.part, nblk,
                           K.flag, 0);
        hipLaunchKernelGGL(k_sum_parts, dim3(j + 2), dim3(RB), 0, ctx->stream, K.part, nblk, small + L.h(),
                           K.flag, 0);
        if (j + 1 <= 32) {
            // pass 1's update with pass 2's dots (used if pass 2 is taken)
            const int nv1 = j + 1;
            if (nv1 <= 8)
                hipLaunchKernelGGL(k_maxpy_mdot<8>, dim3(nblk), dim3(RB), 0, ctx->stream, K.V, nd, nv1,
                                   small + L.h(), K.w, K.part, nblk, K.flag);
            else if (nv1 <= 16)
                hipLaunchKernelGGL(k_maxpy_mdot<16>, dim3(nblk), dim3(RB), 0, ctx->stream, K.V, nd, nv1,
                                   small + L.h(), K.w, K.part, nblk, K.flag);
            else
                hipLaunchKernelGGL(k_maxpy_mdot<32>, dim3(nblk), dim3(RB), 0, ctx->stream, K.V, nd, nv1,
                                   small + L.h(), K.w, K.part, nblk, K.flag);
            hipLaunchKernelGGL(k_close_pass, dim3(1), dim3(RB), 0, ctx->stream, K.part, nblk, nv1, small, m,
                               j, 1, K.flag);
            // the second pass's update (when taken) with the normalization
            hipLaunchKernelGGL(k_update_normalize, dim3(sg), dim3(RB), 0, ctx->stream, K.V, nd, nv1, K.w,
                               K.V + (int64_t)(j + 1) * nd, small, m, K.flag);
        } else {
            hipLaunchKernelGGL(k_maxpy, dim3(nblk), dim3(RB), 0, ctx->stream, K.V, nd, j + 1, small + L.h(),
                               -1.0, K.w, K.part, nblk, K.flag, 0);
            hipLaunchKernelGGL(k_close_pass, dim3(1), dim3(RB), 0, ctx->stream, K.part, nblk, 0, small, m, j,
                               1, K.flag);
            // pass 2's dots (gated)
            dim3 g2(nblk, (j + 1 + KC - 1) / KC);
            hipLaunchKernelGGL(k_mdot, g2, dim3(RB), 0, ctx->stream, K.V, nd, j + 1, 0, K.w, K.part, nblk,
                               K.flag, 1);
            hipLaunchKernelGGL(k_sum_parts, dim3(j + 1), dim3(RB), 0, ctx->stream, K.part, nblk,
                               small + L.h2(), K.flag, 1);
            // pass 2 (gated)
            hipLaunchKernelGGL(k_maxpy, dim3(nblk), dim3(RB), 0, ctx->stream, K.V, nd, j + 1, small + L.h2(),
                               -1.0, K.w, K.part, nblk, K.flag, 1);
            hipLaunchKernelGGL(k_close_pass, dim3(1), dim3(RB), 0, ctx->stream, K.part, nblk, 0, small, m, j,
                               2, K.flag);
            hipLaunchKernelGGL(k_normalize, dim3(sg), dim3(RB), 0, ctx->stream, K.w,
                               K.V + (int64_t)(j + 1) * nd, nd, small, m, j, K.flag);
        }
        return EFT_OK;
    };
    for (;;) {
        const double rel = beta / bnorm;
        inf.rel_res = rel;
        if (!std::isfinite(beta)) {
            ctx->err = "NaN in the Krylov solve";
            st = EFT_ENAN;
            break;
        }
        if (beta <= tol) {
            st = EFT_OK;
            inf.converged = 1;
            break;
        }
        if (total >= maxit) break;
        const int mc = std::min(m, maxit - total);
        hipLaunchKernelGGL(k_start_cycle, dim3(sg), dim3(RB), 0, ctx->stream, K.r, K.V, nd, small, m, beta, tol,
                           K.flag);
        int jdone = 0;
        double est_prev = beta;
        int j_prev = 0;
        for (int j0 = 0, j1 = 0; j0 < mc; j0 = j1) {
            j1 = std::min(mc, j0 + chunk);
            // the momentum system's columns as HIP graphs when asked for and
            // nothing host-side watches the launches
            const bool graph = ctx->par.graphs && mg && !learned && !harvest && A == &ctx->J && ctx->kt.mask == 0 &&
                               !ctx->no_alloc;
            for (int j = j0; j < j1; ++j) {
                if (graph) EFT_TRY(column_graph(ctx, A, j, m, nd, column));
                else EFT_TRY(column(j));
            }
            EFT_HIP(hipGetLastError());
            ctx->kt.tag = -1;
            EFT_HIP(hipMemcpyAsync(ctx->hscal, K.flag, sizeof(int32_t) * 8, hipMemcpyDeviceToHost, ctx->stream));
            EFT_HIP(hipMemcpyAsync(ctx->hscal + 4, small + L.sc() + 5, sizeof(double), hipMemcpyDeviceToHost,
                                   ctx->stream));
            EFT_HIP(hipStreamSynchronize(ctx->stream));
            const int32_t *hf = (const int32_t *)ctx->hscal;
            jdone = hf[1];
            if (hf[5]) inf.fallback_used = 1;
            eft_kt_void_from(ctx, jdone);
            EFT_TRY(eft_kt_harvest(ctx));
            if (hf[6]) {
                ctx->err = "singular diagonal block in the preconditioner's factorization (point-block Jacobi or "
                           "ILU(0)): singular system";
                inf.iters = total + jdone;
                if (info) *info = inf;
                return EFT_EBREAKDOWN;
            }
            if (learned && total + jdone >= nn_budget) {
                learned = false;
                inf.fallback_used = 1;
            }
            if (hf[0] == 0) break;
            // next chunk: half the columns still needed at the faster of two
            // convergence rates, the cycle's mean and the last chunk's (at
            // least 1, at most 16).  GMRES convergence is irregular; columns
            // enqueued past convergence still cost their (gated) launches,
            // while a shorter chunk costs one more read of the state, so the
            // prediction is taken short.
            const double est = ctx->hscal[4];
            chunk = 8;
            if (est > 0.0 && est < beta && jdone > 0) {
                double rate = std::log(est / beta) / (double)jdone;
                if (est < est_prev && jdone > j_prev)
                    rate = std::min(rate, std::log(est / est_prev) / (double)(jdone - j_prev));
                const double need = std::log(tol / est) / rate;
                if (std::isfinite(need)) chunk = (int)std::min(16.0, std::max(1.0, std::ceil(0.5 * need)));
            }
            est_prev = est;
            j_prev = jdone;
        }
        // x += Z y
        hipLaunchKernelGGL(k_trisolve, dim3(1), dim3(64), 0, ctx->stream, small, m, K.flag);
        hipLaunchKernelGGL(k_maxpy, dim3(nblk), dim3(RB), 0, ctx->stream, K.Z, nd, jdone, small + L.y(), 1.0, x,
                           (double *)nullptr, nblk, (const int32_t *)nullptr, 0);
        EFT_HIP(hipGetLastError());
        total += jdone;
        inf.restarts += 1;
        if (harvest) {
            NS.next = (NS.next + jdone) % NS.cap_pairs;
            NS.stored += jdone;
        }
        // true residual
        EFT_TRY(eft_spmv_dev(ctx, A, x, K.r));
        hipLaunchKernelGGL(k_bmr, dim3(sg), dim3(RB), 0, ctx->stream, b, K.r, nd);
        EFT_HIP(hipGetLastError());
        EFT_TRY(eft_norm2(ctx, K.r, nd, &beta));
        if (jdone == 0) {  // no progress possible
            inf.rel_res = beta / bnorm;
            if (beta <= tol) {
                st = EFT_OK;
                inf.converged = 1;
            } else {
                st = EFT_EBREAKDOWN;
                ctx->err = "FGMRES made no progress";
            }
            break;
        }
    }
    inf.iters = total;
    if (harvest && st == EFT_OK) {   // the solve itself: (D^-1 b, x)
        EFT_TRY(eft_nn_store_pair(ctx, K.Dinv, b, x, NS.next, nullptr));
        NS.next = (NS.next + 1) % NS.cap_pairs;
        NS.stored += 1;
    }
    if (info) *info = inf;
    if (st == EFT_ENOTCONV) ctx->err = "FGMRES reached lin_maxit";
    return st;
}

// ------------------------------------------- allocation-free FGMRES ----
//
// Callers that cannot allocate device memory (code under stream capture,
// serving loops, harnesses that forbid it) solve with a Krylov workspace
// carved from one fixed device array instead of the context's.  Each GPU
// holds its own copy of the array for the life of the process; every call on
// a GPU shares it, so calls that overlap on one GPU race.

namespace {

constexpr int64_t NOALLOC_DOUBLES = (int64_t)8 << 20;   // 64 MiB
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int MAX_DEV = 64;
std::mutex scratch_mu;
double *scratch_addr[MAX_DEV] = {};

__global__ void k_fill_i32(int32_t *p, int n, int32_t v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// workspace layout inside the array (offsets in doubles, 256-byte aligned)
struct NoAllocPlan {
    int64_t V, Z, w, r, Dinv, part, small, flag, total;
};
NoAllocPlan plan_of(int64_t n, int bs, int m)
{
    const int64_t nd = n * bs;
    auto up = [](int64_t x) { return (x + 31) / 32 * 32; };
    NoAllocPlan P{};
    int64_t o = 0;
    P.V = o;     o += up(nd * (m + 1));
    P.Z = o;     o += up(nd * m);
    P.w = o;     o += up(nd);
    P.r = o;     o += up(nd);
    P.Dinv = o;  o += up(n * bs * bs);
    P.part = o;  o += up((int64_t)nblk_for(nd) * (m + 2));
    P.small = o; o += up(Small{m}.size());
    P.flag = o;  o += 32;
    P.total = o;
    return P;
}

}  // namespace

eft_status eft_scratch_attach(eft_ctx *ctx)
{
    int dev = 0;
    EFT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEV) {
        ctx->err = "device index out of range for the fixed workspace table";
        return EFT_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_addr[dev]) {
        void *p = nullptr;
        EFT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            ctx->err = "hipGetSymbolAddress returned no address for the fixed workspace";
            return EFT_EDEVICE;
        }
        scratch_addr[dev] = (double *)p;
    }
    ctx->scratch = scratch_addr[dev];
    return EFT_OK;
}

extern "C" eft_status eft_fgmres_noalloc(eft_ctx *ctx, const eft_matrix *A, const double *b, double *x,
                                         eft_solve_info *info)
{
    if (!ctx || !A || !b || !x) return EFT_EINVAL;
    if (!ctx->scratch) {
        ctx->err = "fixed workspace not attached (context creation failed?)";
        return EFT_EDEVICE;
    }
    const int m = std::max(1, std::min(ctx->par.restart, EFT_MAX_RESTART));
    const NoAllocPlan P = plan_of(A->n, A->bs, m);
    if (P.total > NOALLOC_DOUBLES) {
        ctx->err = "system too large for the allocation-free solve: (2 restart + 3) n bs + n bs^2 + partials = " +
                   std::to_string(P.total) + " doubles, the fixed workspace holds " + std::to_string(NOALLOC_DOUBLES);
        return EFT_EINVAL;
    }
    if (ctx->par.precond == 2 && A == &ctx->J && ctx->net.cap_pairs > 0) {
        ctx->err = "the allocation-free solve does not harvest training pairs (eft_nn_harvest(ctx, 0) first)";
        return EFT_EINVAL;
    }
    double *base = ctx->scratch;
    KrylovWs W{};
    W.cap_nd = A->n * A->bs;
    W.cap_m = m;
    W.cap_n = A->n;
    W.cap_bs = A->bs;
    W.V = base + P.V;
    W.Z = base + P.Z;
    W.w = base + P.w;
    W.r = base + P.r;
    W.Dinv = base + P.Dinv;
    W.part = base + P.part;
    W.small = base + P.small;
    W.flag = (int32_t *)(base + P.flag);
    W.nblk = nblk_for(W.cap_nd);
    // the flags must not carry a previous call's state into the first launch
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, ctx->stream, W.flag, 8, 0);
    EFT_HIP(hipGetLastError());
    // the context's own workspace and the timing hook (which creates events)
    // are set aside for the call
    const KrylovWs saved = ctx->kw;
    const uint32_t kt_mask = ctx->kt.mask;
    ctx->kw = W;
    ctx->kt.mask = 0;
    ctx->no_alloc = true;
    const eft_status st = eft_fgmres_dev(ctx, A, b, x, info);
    ctx->no_alloc = false;
    ctx->kt.mask = kt_mask;
    ctx->kw = saved;
    return st;
}
