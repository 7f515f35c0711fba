// Order parameter of a solid given by a closed triangle surface mesh (the
// paper's phase-field interface processing: grid cells, Algorithm
// "distance", ray casting with non-duplicated plane partitioning,
// Algorithm "sign"), 3D.
//
//   grid cells      ncell cells over the bounding box of the mesh nodes; a
//                   triangle belongs to every cell its bounding box grown by
//                   3 eps overlaps (CSR lists built with counting atomics)
//   distance        a node of a cell with triangles: |d| = shortest distance
//                   to the vertices of those triangles, |phi| = tanh(|d| /
//                   (sqrt2 eps)); other nodes |phi| = 1
//   sign            ray in +X over the cells (i..n_x-1, j, k); in the node's
//                   own cell only triangles with a vertex at x > x_p; the Y-Z
//                   projection crosses when A1 + A2 + A3 - A0 <= 2 chi and the
//                   crossing point lies at x > x_p; element / edge / node
//                   crosses recorded by their vertex ids, distinct ones
//                   counted; odd: inside (phi > 0).  A cell without
//                   triangles takes the sign of its lowest-index node.
// One thread per node; the per-ray set of crossings lives in registers and
// private memory (at most MAX_CROSS; more sets a flag).
#include <climits>

#include "dev_common.h"
#include "eft_internal.h"

namespace {

constexpr int MAX_CROSS = 32;

struct InitArgs {
    int64_t N;
    const double *xyz;
    double lo[3], h[3];
    int nc[3];
    const double *vert;
    const int32_t *tri;
    int ntri;
    const int32_t *off, *list;   // triangles of each cell
    const int32_t *ncl, *rep;    // cell of each node, lowest node of each cell
    double eps, chi;
    double *phi;
    int32_t *csign;              // sign of the representative of each cell without triangles
    int32_t *flags;              // [0] most crossings of one ray, [1] overflow
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ int cell_axis(double x, double lo, double h, int n)
{
    return clampi((int)floor((x - lo) / h), 0, n - 1);
}

// cell range [r0, r1] per axis of triangle t's bounding box grown by 3 eps
__device__ __forceinline__ void tri_range(const InitArgs &a, int t, int (&r)[6])
{
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double mn = 1e300, mx = -1e300;
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const double x = a.vert[(int64_t)a.tri[(int64_t)t * 3 + v] * 3 + i];
            mn = x < mn ? x : mn;
            mx = x > mx ? x : mx;
        }
        r[2 * i] = cell_axis(mn - 3.0 * a.eps, a.lo[i], a.h[i], a.nc[i]);
        r[2 * i + 1] = cell_axis(mx + 3.0 * a.eps, a.lo[i], a.h[i], a.nc[i]);
    }
}

__global__ void k_tri_count(InitArgs a, int32_t *cnt)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.ntri) return;
    int r[6];
    tri_range(a, t, r);
    for (int k = r[4]; k <= r[5]; ++k)
        for (int j = r[2]; j <= r[3]; ++j)
            for (int i = r[0]; i <= r[1]; ++i) atomicAdd(cnt + i + a.nc[0] * (j + a.nc[1] * k), 1);
}

__global__ void k_tri_fill(InitArgs a, int32_t *cur, int32_t *list)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.ntri) return;
    int r[6];
    tri_range(a, t, r);
    for (int k = r[4]; k <= r[5]; ++k)
        for (int j = r[2]; j <= r[3]; ++j)
            for (int i = r[0]; i <= r[1]; ++i) {
                const int c = i + a.nc[0] * (j + a.nc[1] * k);
                list[a.off[c] + atomicAdd(cur + c, 1)] = t;
            }
}

__global__ void k_node_cell(InitArgs a, int32_t *ncl, int32_t *rep)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.N) return;
    int ci[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) ci[i] = cell_axis(a.xyz[p * 3 + i], a.lo[i], a.h[i], a.nc[i]);
    const int c = ci[0] + a.nc[0] * (ci[1] + a.nc[1] * ci[2]);
    ncl[p] = c;
    atomicMin(rep + c, (int32_t)p);
}

__device__ __forceinline__ double area2d(double ax, double ay, double bx, double by, double cx, double cy)
{
    return 0.5 * fabs((bx - ax) * (cy - ay) - (cx - ax) * (by - ay));
}

// crossings of the +X ray from node p: parity of the distinct crossings
__device__ int ray_parity(const InitArgs &a, const double *xp, int c)
{
    const int ci = c % a.nc[0], cj = (c / a.nc[0]) % a.nc[1], ck = c / (a.nc[0] * a.nc[1]);
    int tup[MAX_CROSS][3];
    int ntup = 0, over = 0;
    for (int ii = ci; ii < a.nc[0]; ++ii) {
        const int cc = ii + a.nc[0] * (cj + a.nc[1] * ck);
        for (int q = a.off[cc]; q < a.off[cc + 1]; ++q) {
            const int t = a.list[q];
            int tv[3];
            double X[3][3];
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                tv[v] = a.tri[(int64_t)t * 3 + v];
#pragma unroll
                for (int i = 0; i < 3; ++i) X[v][i] = a.vert[(int64_t)tv[v] * 3 + i];
            }
            if (ii == ci && !(X[0][0] > xp[0] || X[1][0] > xp[0] || X[2][0] > xp[0])) continue;
            const double A0 = area2d(X[0][1], X[0][2], X[1][1], X[1][2], X[2][1], X[2][2]);
            if (A0 <= a.chi) continue;
            const double A[3] = {area2d(xp[1], xp[2], X[1][1], X[1][2], X[2][1], X[2][2]),
                                 area2d(xp[1], xp[2], X[2][1], X[2][2], X[0][1], X[0][2]),
                                 area2d(xp[1], xp[2], X[0][1], X[0][2], X[1][1], X[1][2])};
            if (A[0] + A[1] + A[2] - A0 > 2.0 * a.chi) continue;
            const double xc = (A[0] * X[0][0] + A[1] * X[1][0] + A[2] * X[2][0]) / A0;
            if (!(xc > xp[0])) continue;
            int small[3], ns = 0;
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                small[v] = A[v] <= a.chi;
                ns += small[v];
            }
            int id[3] = {-1, -1, -1};
            if (ns == 0) {
                id[0] = tv[0];
                id[1] = tv[1];
                id[2] = tv[2];
            } else if (ns == 1) {
                const int m = small[0] ? 0 : (small[1] ? 1 : 2);
                int o = 0;
#pragma unroll
                for (int v = 0; v < 3; ++v)
                    if (v != m) id[o++] = tv[v];
            } else if (ns == 2) {
                id[0] = tv[!small[0] ? 0 : (!small[1] ? 1 : 2)];
            } else {
                continue;
            }
            // descending ids, -1 last
#pragma unroll
            for (int u = 0; u < 3; ++u)
#pragma unroll
                for (int w = u + 1; w < 3; ++w)
                    if (id[w] > id[u]) {
                        const int s = id[u];
                        id[u] = id[w];
                        id[w] = s;
                    }
            bool dup = false;
            for (int u = 0; u < ntup && !dup; ++u) dup = tup[u][0] == id[0] && tup[u][1] == id[1] && tup[u][2] == id[2];
            if (dup) continue;
            if (ntup < MAX_CROSS) {
                tup[ntup][0] = id[0];
                tup[ntup][1] = id[1];
                tup[ntup][2] = id[2];
                ++ntup;
            } else {
                over = 1;
            }
        }
    }
    atomicMax(a.flags, ntup);
    if (over) atomicOr(a.flags + 1, 1);
    return ntup & 1;
}

__global__ __launch_bounds__(256) void k_phase(InitArgs a)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.N) return;
    const int c = a.ncl[p];
    const bool iface = a.off[c + 1] > a.off[c];
    if (!iface && a.rep[c] != (int32_t)p) return;
    double xp[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) xp[i] = a.xyz[p * 3 + i];
    const int s = ray_parity(a, xp, c) ? 1 : -1;
    if (!iface) {
        a.csign[c] = s;
        return;
    }
    double d2 = 1e300;
    for (int q = a.off[c]; q < a.off[c + 1]; ++q) {
        const int t = a.list[q];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const double *y = a.vert + (int64_t)a.tri[(int64_t)t * 3 + v] * 3;
            double dd = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) dd += (xp[i] - y[i]) * (xp[i] - y[i]);
            d2 = dd < d2 ? dd : d2;
        }
    }
    a.phi[p] = s * tanh(sqrt(d2) / (sqrt(2.0) * a.eps));
}

__global__ void k_copy_sign(InitArgs a)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.N) return;
    const int c = a.ncl[p];
    if (a.off[c + 1] > a.off[c]) return;
    a.phi[p] = a.csign[c] > 0 ? 1.0 : -1.0;
}

__global__ void k_fill_i(int32_t *p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <typename T> eft_status tmp_alloc(eft_ctx *ctx, std::vector<void *> &keep, T **p, int64_t n)
{
    if (hipMalloc((void **)p, sizeof(T) * std::max<int64_t>(n, 1)) != hipSuccess) {
        ctx->err = "out of device memory (phase initialization)";
        return EFT_ENOMEM;
    }
    keep.push_back(*p);
    return EFT_OK;
}

}  // namespace

eft_status eft_init_phase(eft_ctx *ctx, const eft_surface *s, double eps, const int32_t *ncell, double chi,
                          double *phi, int32_t *crossings)
{
    if (!ctx || !s || !ncell || !phi || !s->vert || !s->tri || s->n_vert <= 0 || s->n_tri <= 0) return EFT_EINVAL;
    if (ctx->dim != 3) {
        ctx->err = "phase initialization from a surface mesh is 3D";
        return EFT_EUNSUPPORTED;
    }
    if (!(eps > 0.0) || !(chi >= 0.0) || ncell[0] < 1 || ncell[1] < 1 || ncell[2] < 1 ||
        (int64_t)ncell[0] * ncell[1] * ncell[2] > (1 << 24)) {
        ctx->err = "eps > 0, chi >= 0, 1 <= cells per axis, at most 2^24 cells";
        return EFT_EINVAL;
    }
    for (int64_t t = 0; t < 3 * (int64_t)s->n_tri; ++t)
        if (s->tri[t] < 0 || s->tri[t] >= s->n_vert) {
            ctx->err = "triangle vertex index out of range";
            return EFT_EINVAL;
        }
    std::vector<void *> keep;
    auto release = [&]() {
        for (void *q : keep) (void)hipFree(q);
    };
    InitArgs a{};
    a.N = ctx->N;
    a.xyz = ctx->xyz;
    for (int i = 0; i < 3; ++i) {
        a.lo[i] = ctx->bb_lo[i];
        a.nc[i] = ncell[i];
        a.h[i] = (ctx->bb_hi[i] - ctx->bb_lo[i]) / ncell[i];
    }
    a.ntri = s->n_tri;
    a.eps = eps;
    a.chi = chi;
    a.phi = phi;
    const int64_t nc = (int64_t)ncell[0] * ncell[1] * ncell[2];
    double *vert = nullptr;
    int32_t *tri = nullptr, *cnt = nullptr, *off = nullptr, *list = nullptr, *ncl = nullptr, *rep = nullptr,
            *csign = nullptr, *flags = nullptr;
    eft_status st = EFT_OK;
    if ((st = tmp_alloc(ctx, keep, &vert, 3 * (int64_t)s->n_vert)) != EFT_OK ||
        (st = tmp_alloc(ctx, keep, &tri, 3 * (int64_t)s->n_tri)) != EFT_OK ||
        (st = tmp_alloc(ctx, keep, &cnt, nc)) != EFT_OK || (st = tmp_alloc(ctx, keep, &off, nc + 1)) != EFT_OK ||
        (st = tmp_alloc(ctx, keep, &ncl, ctx->N)) != EFT_OK || (st = tmp_alloc(ctx, keep, &rep, nc)) != EFT_OK ||
        (st = tmp_alloc(ctx, keep, &csign, nc)) != EFT_OK || (st = tmp_alloc(ctx, keep, &flags, 2)) != EFT_OK) {
        release();
        return st;
    }
    a.vert = vert;
    a.tri = tri;
    a.ncl = ncl;
    a.rep = rep;
    a.csign = csign;
    a.flags = flags;
    hipStream_t sm = ctx->stream;
    auto fill = [&](int32_t *p, int64_t n, int32_t v) {
        hipLaunchKernelGGL(k_fill_i, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, sm, p, n, v);
    };
    if (hipMemcpyAsync(vert, s->vert, sizeof(double) * 3 * s->n_vert, hipMemcpyHostToDevice, sm) != hipSuccess ||
        hipMemcpyAsync(tri, s->tri, sizeof(int32_t) * 3 * s->n_tri, hipMemcpyHostToDevice, sm) != hipSuccess) {
        release();
        ctx->err = "upload of the surface mesh failed";
        return EFT_EDEVICE;
    }
    fill(cnt, nc, 0);
    fill(flags, 2, 0);
    const dim3 gt((unsigned)((s->n_tri + 255) / 256)), gn((unsigned)((ctx->N + 255) / 256));
    hipLaunchKernelGGL(k_tri_count, gt, dim3(256), 0, sm, a, cnt);
    // exclusive scan of the cell counts on the host (an initialization step)
    std::vector<int32_t> hc(nc), ho(nc + 1);
    if (hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, sm) != hipSuccess ||
        hipStreamSynchronize(sm) != hipSuccess) {
        release();
        ctx->err = "triangle-to-cell count failed";
        return EFT_EDEVICE;
    }
    int64_t tot = 0;
    for (int64_t c = 0; c < nc; ++c) {
        ho[c] = (int32_t)tot;
        tot += hc[c];
    }
    ho[nc] = (int32_t)tot;
    if (tot > INT_MAX / 2) {
        release();
        ctx->err = "too many triangle-cell pairs (use fewer cells or a coarser surface)";
        return EFT_EINVAL;
    }
    if ((st = tmp_alloc(ctx, keep, &list, tot)) != EFT_OK) {
        release();
        return st;
    }
    a.off = off;
    a.list = list;
    EFT_HIP(hipMemcpyAsync(off, ho.data(), sizeof(int32_t) * (nc + 1), hipMemcpyHostToDevice, sm));
    fill(cnt, nc, 0);
    hipLaunchKernelGGL(k_tri_fill, gt, dim3(256), 0, sm, a, cnt, list);
    fill(rep, nc, INT_MAX);
    hipLaunchKernelGGL(k_node_cell, gn, dim3(256), 0, sm, a, ncl, rep);
    hipLaunchKernelGGL(k_phase, gn, dim3(256), 0, sm, a);
    hipLaunchKernelGGL(k_copy_sign, gn, dim3(256), 0, sm, a);
    int32_t hf[2] = {0, 0};
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, sm);
    const hipError_t e3 = hipStreamSynchronize(sm);
    release();
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        ctx->err = "phase initialization kernels failed";
        return EFT_EDEVICE;
    }
    if (crossings) {
        crossings[0] = hf[0];
        crossings[1] = hf[1];
    }
    return EFT_OK;
}
