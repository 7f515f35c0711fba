// Learned right preconditioner for the FGMRES solve of the momentum/mass
// system (eq. LS_NS).  The paper does not have it: FGMRES admits any variable
// right preconditioner, so the network changes only the iteration count,
// never the converged answer.
//
//   u = D^-1 r                 node-block Jacobi (nn_base = 0), or the
//                              multigrid V-cycle applied to r (nn_base = 1)
//   s = sqrt(mean(u^2))        global scale (1 when u = 0)
//   f_i = [u_i / s, m_i]       m = 1 on free dofs, 0 on Dirichlet dofs
//   h0 = relu(f W_in + b_in)
//   l = 1..L:  g_i = mean of h_j over the matrix-graph neighbours j of i
//              (i itself included);   h = relu([h, g] W_l + b_l)
//   z = u + s (m * (h W_out))
//
// With W_out = 0 (its initial value) the map is exactly its base (block
// Jacobi or the V-cycle).  The
// dense layers are GEMMs [nodes x K] x [K x H] on the matrix cores (gfx950
// MFMA 32x32x16 BF16 operands, FP32 accumulation); activations and parameters are
// FP32, the input and output vectors FP64.  Training (one pair per
// gradient, Adam) runs on the device by the backward kernels below.
//
// Parameter layout (one FP32 vector): W_in [F][H], b_in [H], then per layer
// W_l [2H][H], b_l [H], then W_out [H][bs]; F = 2 bs.
#include "dev_common.h"
#include "eft_internal.h"

typedef __bf16 eft_bf8 __attribute__((ext_vector_type(8)));
typedef float eft_f16v __attribute__((ext_vector_type(16)));

namespace {

constexpr int NB = 256;   // threads of the elementwise and reduction kernels

struct Offs {
    int64_t Win, bin, W[9], b[9], Wout, n;
};

Offs offs_of(const NNState &S)
{
    Offs o{};
    const int64_t H = S.H, F = S.F;
    o.Win = 0;
    o.bin = F * H;
    int64_t p = o.bin + H;
    for (int l = 1; l <= S.L; ++l) {
        o.W[l] = p;
        o.b[l] = p + 2 * H * H;
        p = o.b[l] + H;
    }
    o.Wout = p;
    o.n = p + H * S.bs;
    return o;
}

__device__ __forceinline__ bool gated_off(const int32_t *flag) { return flag != nullptr && flag[0] == 0; }

// ------------------------------------------------------------- GEMM ----

// C[z][m][n] = sum over k in split z of A(m, k) B(k, n) (+ bias[n]), with
// A(m, k) = A1[m a1m + k a1k] for k < K1 and A2[m a2m + (k - K1) a2k]
// otherwise; B(k, n) = B[k bk + n bn].  A wavefront computes a 32 x 64 tile
// with two 32x32x16 BF16 MFMA accumulators (gfx950); a workgroup stacks 4
// wavefronts along m and shares the B tile: 64 rows of k at a time, staged
// in LDS as BF16 (rounded once, to nearest even), padded against bank
// conflicts.  Lane l supplies A(row l%32, k0 + 8(l/32) + t) and
// B(k0 + 8(l/32) + t, col l%32), t < 8, and receives C(8(t/4) + 4(l/32) + t%4,
// l%32) in accumulator slot t.  Rows of A with unit k stride are read as
// two 16-byte vectors per 8 values.
struct GemmArgs {
    int64_t M, N, K, K1;
    const float *A1, *A2;
    int64_t a1m, a1k, a2m, a2k;
    const float *B;
    int64_t bk, bn;
    const float *bias;
    float *C, *Crelu;
    int64_t cm, csplit;
    int64_t kchunk;
    const int32_t *flag;
};

constexpr int GKT = 64;   // k rows of the B tile per LDS stage

// 8 consecutive values of A's row am from k (within one source, unit stride
// and 16-byte alignment when vec)
__device__ __forceinline__ void a_row8(const GemmArgs &g, int64_t am, int64_t k, int64_t kend, bool vec,
                                       eft_bf8 &a)
{
    if (am < g.M && vec && k + 8 <= kend && (k + 8 <= g.K1 || k >= g.K1)) {
        const float *p = k < g.K1 ? g.A1 + am * g.a1m + k : g.A2 + am * g.a2m + (k - g.K1);
        const float4 x0 = reinterpret_cast<const float4 *>(p)[0], x1 = reinterpret_cast<const float4 *>(p)[1];
        a[0] = (__bf16)x0.x;
        a[1] = (__bf16)x0.y;
        a[2] = (__bf16)x0.z;
        a[3] = (__bf16)x0.w;
        a[4] = (__bf16)x1.x;
        a[5] = (__bf16)x1.y;
        a[6] = (__bf16)x1.z;
        a[7] = (__bf16)x1.w;
        return;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int64_t kk = k + t;
        float v = 0.0f;
        if (am < g.M && kk < kend) v = kk < g.K1 ? g.A1[am * g.a1m + kk * g.a1k] : g.A2[am * g.a2m + (kk - g.K1) * g.a2k];
        a[t] = (__bf16)v;
    }
}

__global__ __launch_bounds__(256) void k_gemm(GemmArgs g)
{
    if (gated_off(g.flag)) return;
    __shared__ __bf16 Bs[GKT][64 + 8];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t m0 = ((int64_t)blockIdx.x * 4 + w) * 32, n0 = (int64_t)blockIdx.y * 64;
    const int64_t kb = (int64_t)blockIdx.z * g.kchunk;
    const int64_t ke = kb + g.kchunk < g.K ? kb + g.kchunk : g.K;
    const int64_t am = m0 + (lane & 31);
    const int kq = 8 * (lane >> 5);
    // unit k stride with 16-byte aligned rows in both sources
    const bool vec = g.a1k == 1 && g.a1m % 4 == 0 && (g.K1 >= g.K || (g.a2k == 1 && g.a2m % 4 == 0 && g.K1 % 8 == 0)) &&
                     (reinterpret_cast<uintptr_t>(g.A1) & 15) == 0 &&
                     (g.K1 >= g.K || (reinterpret_cast<uintptr_t>(g.A2) & 15) == 0);
    eft_f16v acc0, acc1;
#pragma unroll
    for (int t = 0; t < 16; ++t) acc0[t] = acc1[t] = 0.0f;
    for (int64_t kt = kb; kt < ke; kt += GKT) {
        __syncthreads();
        for (int t = threadIdx.x; t < GKT * 64; t += 256) {
            const int r = t >> 6, c = t & 63;
            const int64_t k = kt + r, col = n0 + c;
            Bs[r][c] = (__bf16)((k < ke && col < g.N) ? g.B[k * g.bk + col * g.bn] : 0.0f);
        }
        __syncthreads();
        const int64_t kend = kt + GKT < ke ? kt + GKT : ke;
        for (int64_t k0 = kt; k0 < kend; k0 += 16) {
            eft_bf8 a, b0, b1;
            a_row8(g, am, k0 + kq, kend, vec, a);
            const int r0 = (int)(k0 - kt) + kq;   // < GKT: k0 - kt <= GKT - 16
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                b0[t] = Bs[r0 + t][lane & 31];
                b1[t] = Bs[r0 + t][32 + (lane & 31)];
            }
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b1, acc1, 0, 0, 0);
        }
    }
    float *C = g.C + (int64_t)blockIdx.z * g.csplit;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int64_t col = n0 + 32 * j + (lane & 31);
        if (col >= g.N) continue;
        const float bb = g.bias ? g.bias[col] : 0.0f;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int64_t row = m0 + 8 * (t >> 2) + 4 * (lane >> 5) + (t & 3);
            if (row >= g.M) continue;
            const float v = (j == 0 ? acc0[t] : acc1[t]) + bb;
            C[row * g.cm + col] = v;
            if (g.Crelu) g.Crelu[row * g.cm + col] = v > 0.0f ? v : 0.0f;
        }
    }
}

// out[i] (+)= sum over splits z of part[z][i]; eight running sums per
// thread keep eight loads in flight (fixed order: deterministic)
__global__ void k_sum_splits(const float *part, int64_t nsplit, int64_t n, float *out, int accumulate)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    int64_t z = 0;
    for (; z + 8 <= nsplit; z += 8)
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] += part[(z + u) * n + i];
    for (; z < nsplit; ++z) s[0] += part[z * n + i];
    const float t = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    out[i] = accumulate ? out[i] + t : t;
}

// --------------------------------------------------------- node kernels --

// u = D^-1 r (node blocks), and per-block partial sums of u^2
__global__ __launch_bounds__(NB) void k_bj_u(int64_t n, int bs, const double *Dinv, const double *r, double *u,
                                             double *part, const int32_t *flag)
{
    __shared__ double lds[NB / 64];
    if (gated_off(flag)) return;
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    double v = 0.0;
    if (t < n * bs) {
        const int64_t i = t / bs;
        const int c = (int)(t - i * bs);
        const double *D = Dinv + i * bs * bs + c * bs;
        for (int q = 0; q < bs; ++q) v += D[q] * r[i * bs + q];
        u[t] = v;
    }
    const double s = block_sum<NB>(v * v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// sum of squares of an FP32 vector converted into u (training input)
__global__ __launch_bounds__(NB) void k_load_u(int64_t nd, const float *src, double *u, double *part)
{
    __shared__ double lds[NB / 64];
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    double v = 0.0;
    if (t < nd) {
        v = (double)src[t];
        u[t] = v;
    }
    const double s = block_sum<NB>(v * v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// FP64 copy into u with per-block partial sums of u^2
__global__ __launch_bounds__(NB) void k_copy_u(int64_t nd, const double *src, double *u, double *part)
{
    __shared__ double lds[NB / 64];
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    double v = 0.0;
    if (t < nd) {
        v = src[t];
        u[t] = v;
    }
    const double s = block_sum<NB>(v * v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// red[slot] = sqrt(sum(part) / nd), 1 when zero (fixed summation order)
__global__ __launch_bounds__(NB) void k_scale(const double *part, int nblk, int64_t nd, double *out,
                                              const int32_t *flag)
{
    __shared__ double lds[NB / 64];
    if (gated_off(flag)) return;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += NB) s += part[b];
    s = block_sum<NB>(s, lds);
    if (threadIdx.x == 0) {
        const double v = sqrt(s / (double)nd);
        *out = v > 0.0 ? v : 1.0;
    }
}

__global__ void k_features(int64_t n, int bs, const double *u, const float *mask, const double *sc, float *f,
                           const int32_t *flag)
{
    if (gated_off(flag)) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * bs) return;
    const int64_t i = t / bs;
    const int c = (int)(t - i * bs);
    const double inv = 1.0 / *sc;
    f[i * 2 * bs + c] = (float)(u[t] * inv);
    f[i * 2 * bs + bs + c] = mask[t];
}

// g_i = mean over the row pattern of i of h_j (64 lanes = 64 features)
__global__ __launch_bounds__(256) void k_agg(int64_t n, int H, const int32_t *rowptr, const int32_t *col,
                                             const float *h, float *g, const int32_t *flag)
{
    if (gated_off(flag)) return;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int c = threadIdx.x & 63;
    if (i >= n || c >= H) return;
    const int k0 = rowptr[i], k1 = rowptr[i + 1];
    float s = 0.0f;
    for (int k = k0; k < k1; ++k) s += h[(int64_t)col[k] * H + c];
    g[i * H + c] = s / (float)(k1 - k0);
}

// dh_j = dX[j][0..H) + sum over rows i of the pattern of j of dX[i][H..2H) / deg_i
// (the transpose of the mean; the node graph is symmetric)
__global__ __launch_bounds__(256) void k_agg_t(int64_t n, int H, const int32_t *rowptr, const int32_t *col,
                                               const float *dX, float *dh)
{
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int c = threadIdx.x & 63;
    if (j >= n || c >= H) return;
    const int k0 = rowptr[j], k1 = rowptr[j + 1];
    float s = dX[j * 2 * H + c];
    for (int k = k0; k < k1; ++k) {
        const int64_t i = col[k];
        s += dX[i * 2 * H + H + c] / (float)(rowptr[i + 1] - rowptr[i]);
    }
    dh[j * H + c] = s;
}

// delta = h W_out;  z = u + s (m * delta)
__global__ void k_output(int64_t n, int bs, int H, const float *h, const float *Wout, const double *u,
                         const float *mask, const double *sc, float *delta, double *z, const int32_t *flag)
{
    if (gated_off(flag)) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * bs) return;
    const int64_t i = t / bs;
    const int c = (int)(t - i * bs);
    float d = 0.0f;
    for (int k = 0; k < H; ++k) d += h[i * H + k] * Wout[k * bs + c];
    delta[t] = d;
    z[t] = u[t] + *sc * (double)(mask[t] * d);
}

// loss pieces of a pair: partial sums of (m (z - e))^2 and (m e)^2
__global__ __launch_bounds__(NB) void k_pair_sums(int64_t nd, const double *z, const float *e, const float *mask,
                                                  double *part, int nblk)
{
    __shared__ double lds[NB / 64];
    const int64_t t = (int64_t)blockIdx.x * NB + threadIdx.x;
    double a = 0.0, b = 0.0;
    if (t < nd) {
        const double m = mask[t], d = m * (z[t] - (double)e[t]), ee = m * (double)e[t];
        a = d * d;
        b = ee * ee;
    }
    a = block_sum<NB>(a, lds);
    b = block_sum<NB>(b, lds);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = a;
        part[nblk + blockIdx.x] = b;
    }
}

// out[0] = loss = sum a / E, out[1] = E (1 when zero)
__global__ __launch_bounds__(NB) void k_pair_loss(const double *part, int nblk, double *out)
{
    __shared__ double lds[NB / 64];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nblk; k += NB) {
        a += part[k];
        b += part[nblk + k];
    }
    a = block_sum<NB>(a, lds);
    b = block_sum<NB>(b, lds);
    if (threadIdx.x == 0) {
        const double E = b > 0.0 ? b : 1.0;
        out[0] = a / E;
        out[1] = E;
    }
}

// ddelta = 2 s m (z - e) / E;  dh = ddelta W_out^T
__global__ void k_out_back(int64_t n, int bs, int H, const double *z, const float *e, const float *mask,
                           const double *sc, const double *lossE, const float *Wout, float *ddelta, float *dh)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double f = 2.0 * *sc / lossE[1];
    float dd[8];
    for (int c = 0; c < bs; ++c) {
        const int64_t t = i * bs + c;
        dd[c] = (float)(f * mask[t] * (z[t] - (double)e[t]));
        ddelta[t] = dd[c];
    }
    for (int k = 0; k < H; ++k) {
        float s = 0.0f;
        for (int c = 0; c < bs; ++c) s += dd[c] * Wout[k * bs + c];
        dh[i * H + k] = s;
    }
}

// x *= (pre > 0)
__global__ void k_relu_mask(int64_t n, const float *pre, float *x)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n && !(pre[t] > 0.0f)) x[t] = 0.0f;
}

// column sums of x [n][H] (H <= 64): part[blk][c] over rows_per_blk rows; the
// 256 threads of a block take 4 interleaved row sequences per column, summed
// in LDS at the end
__global__ __launch_bounds__(256) void k_colsum(int64_t n, int H, const float *x, int64_t rows_per_blk, float *part)
{
    __shared__ float ls[4][64];
    const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk, r1 = r0 + rows_per_blk < n ? r0 + rows_per_blk : n;
    float s = 0.0f;
    if (c < H)
        for (int64_t r = r0 + q; r < r1; r += 4) s += x[r * H + c];
    ls[q][c] = s;
    __syncthreads();
    if (q == 0 && c < H) part[(int64_t)blockIdx.x * H + c] = ls[0][c] + ls[1][c] + ls[2][c] + ls[3][c];
}

__global__ void k_adam(int64_t n, float *theta, const float *grad, float *m1, float *m2, float lr, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i];
    const float a = 0.9f * m1[i] + 0.1f * g, b = 0.999f * m2[i] + 0.001f * g * g;
    m1[i] = a;
    m2[i] = b;
    theta[i] -= lr * (a / c1) / (sqrtf(b / c2) + 1e-8f);
}

// counter-based initial parameters: uniform(-lim, lim) from a 64-bit mix of
// (seed, index) (splitmix64)
__global__ void k_init_uniform(float *p, int64_t n, float lim, uint64_t seed, int64_t base)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(base + i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double u01 = (double)(z >> 11) * (1.0 / 9007199254740992.0);
    p[i] = (float)((2.0 * u01 - 1.0) * lim);
}

__global__ void k_fill_f(float *p, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// harvest one pair: hu = D^-1 r, he = e (FP32), gated by the Krylov flag
__global__ void k_store_pair(int64_t n, int bs, const double *Dinv, const double *r, const double *e, float *hu,
                             float *he, const int32_t *flag)
{
    if (gated_off(flag)) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * bs) return;
    double v = r[t];   // the base itself (multigrid base) when Dinv is null
    if (Dinv) {
        const int64_t i = t / bs;
        const int c = (int)(t - i * bs);
        const double *D = Dinv + i * bs * bs + c * bs;
        v = 0.0;
        for (int q = 0; q < bs; ++q) v += D[q] * r[i * bs + q];
    }
    hu[t] = (float)v;
    he[t] = (float)e[t];
}

__global__ void k_dir_mask(int64_t n_dir, const int32_t *node, const uint8_t *mask, int bs, float *m)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_dir) return;
    for (int c = 0; c < bs; ++c)
        if ((mask[t] >> c) & 1) m[(int64_t)node[t] * bs + c] = 0.0f;
}

int grid_of(int64_t n, int per) { return (int)((n + per - 1) / per); }

template <typename T> eft_status nmal(eft_ctx *ctx, T **p, int64_t count)
{
    *p = nullptr;
    if (count <= 0) count = 1;
    if (hipMalloc((void **)p, sizeof(T) * (size_t)count) != hipSuccess) {
        ctx->err = "out of device memory (learned preconditioner)";
        return EFT_ENOMEM;
    }
    return EFT_OK;
}

void gemm(eft_ctx *ctx, GemmArgs a)
{
    const int64_t nsplit = a.kchunk > 0 ? (a.K + a.kchunk - 1) / a.kchunk : 1;
    if (a.kchunk <= 0) a.kchunk = a.K;
    dim3 grid((unsigned)grid_of(a.M, 128), (unsigned)grid_of(a.N, 64), (unsigned)std::max<int64_t>(1, nsplit));
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, ctx->stream, a);
}

// nodes per split of the weight-gradient GEMMs and of the bias sums (short
// splits: enough workgroups to fill the GPU at the sizes trained here)
constexpr int64_t KCHUNK = 256;

// forward of the network on ctx->net.u (scale in red[0]); z gets the result
void forward(eft_ctx *ctx, double *z, const int32_t *flag)
{
    NNState &S = ctx->net;
    const Offs o = offs_of(S);
    const int64_t n = ctx->N, H = S.H;
    hipLaunchKernelGGL(k_features, dim3(grid_of(n * S.bs, 256)), dim3(256), 0, ctx->stream, n, S.bs, S.u, S.mask,
                       S.red, S.f, flag);
    GemmArgs a{};
    a.M = n;
    a.N = H;
    a.K = S.F;
    a.K1 = S.F;
    a.A1 = S.f;
    a.a1m = S.F;
    a.a1k = 1;
    a.B = S.theta + o.Win;
    a.bk = H;
    a.bn = 1;
    a.bias = S.theta + o.bin;
    a.C = S.pre;
    a.Crelu = S.h;
    a.cm = H;
    a.flag = flag;
    gemm(ctx, a);
    for (int l = 1; l <= S.L; ++l) {
        const float *hp = S.h + (int64_t)(l - 1) * n * H;
        float *gl = S.g + (int64_t)(l - 1) * n * H;
        hipLaunchKernelGGL(k_agg, dim3(grid_of(n, 4)), dim3(256), 0, ctx->stream, n, (int)H, ctx->J.rowptr,
                           ctx->J.col, hp, gl, flag);
        GemmArgs b{};
        b.M = n;
        b.N = H;
        b.K = 2 * H;
        b.K1 = H;
        b.A1 = hp;
        b.a1m = H;
        b.a1k = 1;
        b.A2 = gl;
        b.a2m = H;
        b.a2k = 1;
        b.B = S.theta + o.W[l];
        b.bk = H;
        b.bn = 1;
        b.bias = S.theta + o.b[l];
        b.C = S.pre + (int64_t)l * n * H;
        b.Crelu = S.h + (int64_t)l * n * H;
        b.cm = H;
        b.flag = flag;
        gemm(ctx, b);
    }
    hipLaunchKernelGGL(k_output, dim3(grid_of(n * S.bs, 256)), dim3(256), 0, ctx->stream, n, S.bs, (int)H,
                       S.h + (int64_t)S.L * n * H, S.theta + o.Wout, S.u, S.mask, S.red, S.delta, z, flag);
}

// weight gradient dW[M][H] += X^T dY over all nodes (X [n][ldx] from column
// offset xo, M columns; dY [n][H]) via split-K partials
void weight_grad(eft_ctx *ctx, const float *X, int64_t ldx, int64_t M, const float *dY, float *dW)
{
    NNState &S = ctx->net;
    const int64_t n = ctx->N, H = S.H;
    GemmArgs a{};
    a.M = M;
    a.N = H;
    a.K = n;
    a.K1 = n;
    a.A1 = X;
    a.a1m = 1;
    a.a1k = ldx;
    a.B = dY;
    a.bk = H;
    a.bn = 1;
    a.C = S.part;
    a.cm = H;
    a.csplit = M * H;
    a.kchunk = KCHUNK;
    gemm(ctx, a);
    const int64_t nsplit = (n + KCHUNK - 1) / KCHUNK;
    hipLaunchKernelGGL(k_sum_splits, dim3(grid_of(M * H, 256)), dim3(256), 0, ctx->stream, S.part, nsplit, M * H, dW,
                       1);
}

void bias_grad(eft_ctx *ctx, const float *dY, float *db)
{
    NNState &S = ctx->net;
    const int64_t n = ctx->N, H = S.H;
    const int64_t nblk = (n + KCHUNK - 1) / KCHUNK;
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)nblk), dim3(256), 0, ctx->stream, n, (int)H, dY, KCHUNK, S.part);
    hipLaunchKernelGGL(k_sum_splits, dim3(grid_of(H, 256)), dim3(256), 0, ctx->stream, S.part, nblk, H, db, 1);
}

// loss of the pair (nn.u, e) and its gradient added into nn.grad; loss in red[1]
void loss_backward(eft_ctx *ctx, double *z, const float *e)
{
    NNState &S = ctx->net;
    const Offs o = offs_of(S);
    const int64_t n = ctx->N, H = S.H, nd = n * S.bs;
    const int nblk = grid_of(nd, NB);
    hipLaunchKernelGGL(k_pair_sums, dim3(nblk), dim3(NB), 0, ctx->stream, nd, z, e, S.mask, S.red + 8, nblk);
    hipLaunchKernelGGL(k_pair_loss, dim3(1), dim3(NB), 0, ctx->stream, S.red + 8, nblk, S.red + 1);
    hipLaunchKernelGGL(k_out_back, dim3(grid_of(n, 256)), dim3(256), 0, ctx->stream, n, S.bs, (int)H, z, e, S.mask,
                       S.red, S.red + 1, S.theta + o.Wout, S.delta, S.d1);
    // W_out gradient: h_L^T ddelta  ([H][bs])
    {
        GemmArgs a{};
        a.M = H;
        a.N = S.bs;
        a.K = n;
        a.K1 = n;
        a.A1 = S.h + (int64_t)S.L * n * H;
        a.a1m = 1;
        a.a1k = H;
        a.B = S.delta;
        a.bk = S.bs;
        a.bn = 1;
        a.C = S.part;
        a.cm = S.bs;
        a.csplit = H * S.bs;
        a.kchunk = KCHUNK;
        gemm(ctx, a);
        const int64_t nsplit = (n + KCHUNK - 1) / KCHUNK;
        hipLaunchKernelGGL(k_sum_splits, dim3(grid_of(H * S.bs, 256)), dim3(256), 0, ctx->stream, S.part, nsplit,
                           H * S.bs, S.grad + o.Wout, 1);
    }
    // d1 holds dh of the current layer's output
    for (int l = S.L; l >= 1; --l) {
        const float *pre = S.pre + (int64_t)l * n * H;
        hipLaunchKernelGGL(k_relu_mask, dim3(grid_of(n * H, 256)), dim3(256), 0, ctx->stream, n * H, pre, S.d1);
        const float *hp = S.h + (int64_t)(l - 1) * n * H, *gl = S.g + (int64_t)(l - 1) * n * H;
        weight_grad(ctx, hp, H, H, S.d1, S.grad + o.W[l]);
        weight_grad(ctx, gl, H, H, S.d1, S.grad + o.W[l] + H * H);
        bias_grad(ctx, S.d1, S.grad + o.b[l]);
        // dX = dpre W_l^T  ([n][2H])
        GemmArgs b{};
        b.M = n;
        b.N = 2 * H;
        b.K = H;
        b.K1 = H;
        b.A1 = S.d1;
        b.a1m = H;
        b.a1k = 1;
        b.B = S.theta + o.W[l];
        b.bk = 1;
        b.bn = H;
        b.C = S.d2;
        b.cm = 2 * H;
        gemm(ctx, b);
        hipLaunchKernelGGL(k_agg_t, dim3(grid_of(n, 4)), dim3(256), 0, ctx->stream, n, (int)H, ctx->J.rowptr,
                           ctx->J.col, S.d2, S.d1);
    }
    hipLaunchKernelGGL(k_relu_mask, dim3(grid_of(n * H, 256)), dim3(256), 0, ctx->stream, n * H, S.pre, S.d1);
    weight_grad(ctx, S.f, S.F, S.F, S.d1, S.grad + o.Win);
    bias_grad(ctx, S.d1, S.grad + o.bin);
}

// nn.u <- FP32 vector, scale into red[0]
void load_u(eft_ctx *ctx, const float *src)
{
    NNState &S = ctx->net;
    const int64_t nd = ctx->N * S.bs;
    const int nblk = grid_of(nd, NB);
    hipLaunchKernelGGL(k_load_u, dim3(nblk), dim3(NB), 0, ctx->stream, nd, src, S.u, S.red + 8);
    hipLaunchKernelGGL(k_scale, dim3(1), dim3(NB), 0, ctx->stream, S.red + 8, nblk, nd, S.red, nullptr);
}

}  // namespace

// Fallback of the learned preconditioner, per node: an output with a non-
// finite entry is replaced by the block-Jacobi vector u of that node.
static __global__ __launch_bounds__(256) void k_nn_guard(int64_t n, int bs, const double *__restrict__ u, double *z,
                                                  int32_t *flag)
{
    if (flag && flag[0] == 0) return;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    bool bad = false;
    for (int c = 0; c < bs; ++c) bad |= !isfinite(z[p * bs + c]);
    if (!bad) return;
    for (int c = 0; c < bs; ++c) z[p * bs + c] = u[p * bs + c];
    if (flag) flag[5] = 1;
}

// ------------------------------------------------------------ host side --

eft_status eft_nn_alloc(eft_ctx *ctx)
{
    NNState &S = ctx->net;
    if (S.ready && S.cap_n == ctx->N) return EFT_OK;
    eft_nn_free(ctx);
    S.bs = ctx->bs;
    S.F = 2 * S.bs;
    const Offs o = offs_of(S);
    S.np = o.n;
    const int64_t n = ctx->N, H = S.H, nd = n * S.bs;
    EFT_TRY(nmal(ctx, &S.theta, S.np));
    EFT_TRY(nmal(ctx, &S.grad, S.np));
    EFT_TRY(nmal(ctx, &S.m1, S.np));
    EFT_TRY(nmal(ctx, &S.m2, S.np));
    EFT_TRY(nmal(ctx, &S.mask, nd));
    EFT_TRY(nmal(ctx, &S.f, n * S.F));
    EFT_TRY(nmal(ctx, &S.pre, (S.L + 1) * n * H));
    EFT_TRY(nmal(ctx, &S.h, (S.L + 1) * n * H));
    EFT_TRY(nmal(ctx, &S.g, S.L * n * H));
    EFT_TRY(nmal(ctx, &S.d1, n * 2 * H));
    EFT_TRY(nmal(ctx, &S.d2, n * 2 * H));
    EFT_TRY(nmal(ctx, &S.delta, nd));
    S.cap_part = ((n + KCHUNK - 1) / KCHUNK) * 2 * H * H + H * 64;
    EFT_TRY(nmal(ctx, &S.part, S.cap_part));
    EFT_TRY(nmal(ctx, &S.u, nd));
    {
        const int32_t one[8] = {1, 0, 0, 0, 0, 0, 0, 0};
        EFT_TRY(nmal(ctx, &S.on, 8));
        EFT_HIP(hipMemcpy(S.on, one, sizeof(one), hipMemcpyHostToDevice));
    }
    EFT_TRY(nmal(ctx, &S.red, 16 + 2 * (int64_t)grid_of(nd, NB)));
    hipLaunchKernelGGL(k_fill_f, dim3(grid_of(nd, 256)), dim3(256), 0, ctx->stream, S.mask, nd, 1.0f);
    if (ctx->n_dir > 0)
        hipLaunchKernelGGL(k_dir_mask, dim3(grid_of(ctx->n_dir, 256)), dim3(256), 0, ctx->stream, ctx->n_dir,
                           ctx->dir_node, ctx->dir_mask, S.bs, S.mask);
    EFT_HIP(hipGetLastError());
    S.cap_n = n;
    S.ready = true;
    return EFT_OK;
}

void eft_nn_free(eft_ctx *ctx)
{
    NNState &S = ctx->net;
    auto fr = [](void *p) {
        if (p) (void)hipFree(p);
    };
    fr(S.theta); fr(S.grad); fr(S.m1); fr(S.m2); fr(S.mask); fr(S.f); fr(S.pre); fr(S.h); fr(S.g); fr(S.d1);
    fr(S.d2); fr(S.delta); fr(S.part); fr(S.u); fr(S.on); fr(S.red); fr(S.losses); fr(S.hu); fr(S.he);
    const int H = S.H, L = S.L;
    S = NNState{};
    S.H = H;
    S.L = L;
}

// z = u + s (m * NN(u / s, m)) with the base u = D^-1 v (nn_base = 0) or
// the multigrid V-cycle applied to v (nn_base = 1); gated by the Krylov
// flag.  A node whose output is not finite takes the base's value instead
// (flag[5] = 1 records the fallback; FGMRES admits a preconditioner that
// changes between columns, so the solve stays valid).
eft_status eft_nn_precond(eft_ctx *ctx, const double *Dinv, const double *v, double *z, int32_t *flag)
{
    NNState &S = ctx->net;
    const int64_t nd = ctx->N * S.bs;
    const int nblk = grid_of(nd, NB);
    if (ctx->par.nn_base == 1) {
        EFT_TRY(eft_mg_vcycle(ctx, v, S.u, flag));
        hipLaunchKernelGGL(k_copy_u, dim3(nblk), dim3(NB), 0, ctx->stream, nd, S.u, S.u, S.red + 8);
    } else {
        hipLaunchKernelGGL(k_bj_u, dim3(nblk), dim3(NB), 0, ctx->stream, ctx->N, S.bs, Dinv, v, S.u, S.red + 8,
                           flag);
    }
    hipLaunchKernelGGL(k_scale, dim3(1), dim3(NB), 0, ctx->stream, S.red + 8, nblk, nd, S.red, flag);
    forward(ctx, z, flag);
    hipLaunchKernelGGL(k_nn_guard, dim3(grid_of(ctx->N, 256)), dim3(256), 0, ctx->stream, ctx->N, S.bs, S.u, z, flag);
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}

// One training pair (base of r, e): the base D^-1 r (nn_base = 0) or the
// V-cycle applied to r (nn_base = 1), in FP32 slot `slot` of the pair store.
eft_status eft_nn_store_pair(eft_ctx *ctx, const double *Dinv, const double *r, const double *e, int64_t slot,
                             const int32_t *flag)
{
    NNState &S = ctx->net;
    const int64_t nd = ctx->N * S.bs;
    if (ctx->par.nn_base == 1) {
        // (the V-cycle's kernels read their gate: an always-active one when
        // the pair is not gated by a solve's flag)
        EFT_TRY(eft_mg_vcycle(ctx, r, S.u, flag ? flag : S.on));
        r = S.u;
        Dinv = nullptr;
    }
    hipLaunchKernelGGL(k_store_pair, dim3(grid_of(nd, 256)), dim3(256), 0, ctx->stream, ctx->N, S.bs, Dinv, r, e,
                       S.hu + slot * nd, S.he + slot * nd, flag);
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}

extern "C" {

eft_status eft_nn_init(eft_ctx *ctx, uint64_t seed)
{
    if (!ctx) return EFT_EINVAL;
    EFT_TRY(eft_nn_alloc(ctx));
    NNState &S = ctx->net;
    const Offs o = offs_of(S);
    auto uni = [&](int64_t off, int64_t cnt, float lim) {
        hipLaunchKernelGGL(k_init_uniform, dim3(grid_of(cnt, 256)), dim3(256), 0, ctx->stream, S.theta + off, cnt, lim,
                           seed, off);
    };
    auto zero = [&](float *p, int64_t off, int64_t cnt) {
        hipLaunchKernelGGL(k_fill_f, dim3(grid_of(cnt, 256)), dim3(256), 0, ctx->stream, p + off, cnt, 0.0f);
    };
    const int64_t H = S.H;
    uni(o.Win, (int64_t)S.F * H, (float)std::sqrt(6.0 / S.F));
    zero(S.theta, o.bin, H);
    for (int l = 1; l <= S.L; ++l) {
        uni(o.W[l], 2 * H * H, (float)std::sqrt(6.0 / (2.0 * H)));
        zero(S.theta, o.b[l], H);
    }
    zero(S.theta, o.Wout, H * S.bs);   // starts as block Jacobi
    zero(S.m1, 0, S.np);
    zero(S.m2, 0, S.np);
    S.adam_t = 0;
    EFT_HIP(hipGetLastError());
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    return EFT_OK;
}

eft_status eft_nn_params(eft_ctx *ctx, float *host, int64_t n, int32_t direction)
{
    if (!ctx || (!host && n > 0)) return EFT_EINVAL;
    NNState &S = ctx->net;
    if (!S.ready) {
        ctx->err = "eft_nn_params: call eft_nn_init first";
        return EFT_EINVAL;
    }
    if (n != S.np) {
        ctx->err = "eft_nn_params: n must equal the parameter count";
        return EFT_EINVAL;
    }
    if (direction == 0)
        EFT_HIP(hipMemcpyAsync(host, S.theta, sizeof(float) * n, hipMemcpyDeviceToHost, ctx->stream));
    else
        EFT_HIP(hipMemcpyAsync(S.theta, host, sizeof(float) * n, hipMemcpyHostToDevice, ctx->stream));
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    return EFT_OK;
}

eft_status eft_nn_shape(eft_ctx *ctx, int32_t *hidden, int32_t *layers, int64_t *n_params, int64_t *pairs)
{
    if (!ctx) return EFT_EINVAL;
    if (hidden) *hidden = ctx->net.H;
    if (layers) *layers = ctx->net.L;
    if (n_params) *n_params = ctx->net.ready ? ctx->net.np : 0;
    if (pairs) *pairs = std::min<int64_t>(ctx->net.stored, ctx->net.cap_pairs);
    return EFT_OK;
}

eft_status eft_nn_harvest(eft_ctx *ctx, int32_t capacity)
{
    if (!ctx || capacity < 0) return EFT_EINVAL;
    EFT_TRY(eft_nn_alloc(ctx));
    NNState &S = ctx->net;
    if (S.hu) (void)hipFree(S.hu);
    if (S.he) (void)hipFree(S.he);
    S.hu = S.he = nullptr;
    S.cap_pairs = 0;
    S.stored = S.next = 0;
    if (capacity == 0) return EFT_OK;
    const int64_t nd = ctx->N * S.bs;
    EFT_TRY(nmal(ctx, &S.hu, (int64_t)capacity * nd));
    EFT_TRY(nmal(ctx, &S.he, (int64_t)capacity * nd));
    S.cap_pairs = capacity;
    return EFT_OK;
}

eft_status eft_nn_loss_grad(eft_ctx *ctx, const double *u, const double *e, float *grad_host, double *loss)
{
    if (!ctx || !u || !e) return EFT_EINVAL;
    NNState &S = ctx->net;
    if (!S.ready) {
        ctx->err = "eft_nn_loss_grad: call eft_nn_init first";
        return EFT_EINVAL;
    }
    const int64_t nd = ctx->N * S.bs;
    float *u32 = nullptr, *e32 = nullptr;
    double *z = nullptr;
    EFT_TRY(nmal(ctx, &u32, nd));
    EFT_TRY(nmal(ctx, &e32, nd));
    EFT_TRY(nmal(ctx, &z, nd));
    std::vector<double> hu(nd), he(nd);
    std::vector<float> fu(nd), fe(nd);
    EFT_HIP(hipMemcpy(hu.data(), u, sizeof(double) * nd, hipMemcpyDeviceToHost));
    EFT_HIP(hipMemcpy(he.data(), e, sizeof(double) * nd, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < nd; ++i) {
        fu[i] = (float)hu[i];
        fe[i] = (float)he[i];
    }
    EFT_HIP(hipMemcpy(u32, fu.data(), sizeof(float) * nd, hipMemcpyHostToDevice));
    EFT_HIP(hipMemcpy(e32, fe.data(), sizeof(float) * nd, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_fill_f, dim3(grid_of(S.np, 256)), dim3(256), 0, ctx->stream, S.grad, S.np, 0.0f);
    load_u(ctx, u32);
    forward(ctx, z, nullptr);
    loss_backward(ctx, z, e32);
    EFT_HIP(hipGetLastError());
    double lv = 0.0;
    EFT_HIP(hipMemcpyAsync(&lv, S.red + 1, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    if (grad_host) EFT_HIP(hipMemcpyAsync(grad_host, S.grad, sizeof(float) * S.np, hipMemcpyDeviceToHost, ctx->stream));
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    if (loss) *loss = lv;
    (void)hipFree(u32);
    (void)hipFree(e32);
    (void)hipFree(z);
    return EFT_OK;
}

eft_status eft_nn_apply(eft_ctx *ctx, const double *u, double *z)
{
    if (!ctx || !u || !z) return EFT_EINVAL;
    NNState &S = ctx->net;
    if (!S.ready) {
        ctx->err = "eft_nn_apply: call eft_nn_init first";
        return EFT_EINVAL;
    }
    const int64_t nd = ctx->N * S.bs;
    const int nblk = grid_of(nd, NB);
    hipLaunchKernelGGL(k_copy_u, dim3(nblk), dim3(NB), 0, ctx->stream, nd, u, S.u, S.red + 8);
    hipLaunchKernelGGL(k_scale, dim3(1), dim3(NB), 0, ctx->stream, S.red + 8, nblk, nd, S.red, nullptr);
    forward(ctx, z, nullptr);
    EFT_HIP(hipGetLastError());
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    return EFT_OK;
}

eft_status eft_nn_train(eft_ctx *ctx, int32_t steps, int32_t batch, double lr, uint64_t seed, double *losses)
{
    if (!ctx || steps < 0 || batch < 1 || !(lr > 0.0)) return EFT_EINVAL;
    NNState &S = ctx->net;
    if (!S.ready) {
        ctx->err = "eft_nn_train: call eft_nn_init first";
        return EFT_EINVAL;
    }
    const int64_t npairs = std::min<int64_t>(S.stored, S.cap_pairs);
    if (npairs < 1) {
        ctx->err = "eft_nn_train: no harvested pairs";
        return EFT_EINVAL;
    }
    if (S.cap_steps < steps) {
        if (S.losses) (void)hipFree(S.losses);
        EFT_TRY(nmal(ctx, &S.losses, steps));
        S.cap_steps = steps;
    }
    const int64_t nd = ctx->N * S.bs;
    double *z = nullptr;
    EFT_TRY(nmal(ctx, &z, nd));
    uint64_t st = seed ^ 0x2545F4914F6CDD1Dull;
    for (int32_t it = 0; it < steps; ++it) {
        hipLaunchKernelGGL(k_fill_f, dim3(grid_of(S.np, 256)), dim3(256), 0, ctx->stream, S.grad, S.np, 0.0f);
        for (int32_t b = 0; b < batch; ++b) {
            st ^= st << 13;
            st ^= st >> 7;
            st ^= st << 17;
            const int64_t p = (int64_t)(st % (uint64_t)npairs);
            load_u(ctx, S.hu + p * nd);
            forward(ctx, z, nullptr);
            loss_backward(ctx, z, S.he + p * nd);
            if (b == 0)
                EFT_HIP(hipMemcpyAsync(S.losses + it, S.red + 1, sizeof(double), hipMemcpyDeviceToDevice,
                                       ctx->stream));
        }
        S.adam_t += 1;
        const float c1 = 1.0f - std::pow(0.9f, (float)S.adam_t), c2 = 1.0f - std::pow(0.999f, (float)S.adam_t);
        hipLaunchKernelGGL(k_adam, dim3(grid_of(S.np, 256)), dim3(256), 0, ctx->stream, S.np, S.theta, S.grad, S.m1,
                           S.m2, (float)lr, c1, c2);
        EFT_HIP(hipGetLastError());
    }
    if (losses && steps > 0)
        EFT_HIP(hipMemcpyAsync(losses, S.losses, sizeof(double) * steps, hipMemcpyDeviceToHost, ctx->stream));
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    (void)hipFree(z);
    return EFT_OK;
}

}  // extern "C"
