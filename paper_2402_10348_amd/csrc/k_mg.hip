// Geometric multigrid preconditioner for the momentum/mass system on nested
// Kuhn (Freudenthal) meshes of a box.
//
// The structured simplex mesh of n cells per axis is the regular refinement of
// the one with n/2 cells: every coarse node is a fine node and every other
// fine node is the midpoint of a coarse edge (a Kuhn direction, i.e. a
// non-zero 0/1 offset).  The P1 spaces are nested, so prolongation is linear
// interpolation (weights 1 and 1/2) and restriction its transpose, both
// evaluated in gather form from structured indices.  Coarse operators are
// rediscretized: the same element kernels assemble the coarse Jacobian from
// node fields injected from the fine mesh.  Smoothing is damped point-block
// Jacobi, i.e. the node-wise Vanka smoother of the (d+1)x(d+1) node blocks of
// the equal-order stabilized system; the coarsest level is inverted exactly.
// Dirichlet dofs are removed from the coarse space (masked in transfer).
#include <algorithm>
#include <type_traits>

#include "bsr_rows.h"
#include "dev_common.h"
#include "eft_internal.h"

namespace {

// ------------------------------------------------------------- helpers ----

struct Dims {
    int n[3];   // cells per axis (0 for the unused axis in 2D)
};

__device__ __forceinline__ int64_t node_id(const Dims &d, int i, int j, int k)
{
    return i + (int64_t)(d.n[0] + 1) * (j + (int64_t)(d.n[1] + 1) * k);
}

// Kuhn stencil offsets (D = 3: 0 and +-{x, y, z, x+y, y+z, x+z, x+y+z};
// D = 2: 0 and +-{x, y, x+y})
template <int D> struct Stencil;
template <> struct Stencil<3> {
    static constexpr int S = 15;
    __device__ static void off(int s, int &a, int &b, int &c)
    {
        const int t[8][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {0, 1, 1}, {1, 0, 1}, {1, 1, 1}};
        const int q = s < 8 ? s : s - 7;
        const int sg = s < 8 ? 1 : -1;
        a = sg * t[q][0];
        b = sg * t[q][1];
        c = sg * t[q][2];
    }
};
template <> struct Stencil<2> {
    static constexpr int S = 7;
    __device__ static void off(int s, int &a, int &b, int &c)
    {
        const int t[4][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};
        const int q = s < 4 ? s : s - 3;
        const int sg = s < 4 ? 1 : -1;
        a = sg * t[q][0];
        b = sg * t[q][1];
        c = 0;
    }
};

// ---------------------------------------------------------- injection -----

struct InjArgs {
    int64_t Nc, Nf;
    int d, bs, nv, n_s;
    double alpha;
    const int32_t *inj;
    const double *va, *acc, *rho, *mu, *vp;
    const uint64_t *smask;
    const double *lphi, *iphi, *lB, *iB;   // fine level: phi^n, phi, B^n, B (fractions and B at n+alpha)
    const int32_t *solid_ind;
    double *cva, *cacc, *crho, *cmu, *cas, *cBa, *cvp;
    uint64_t *csmask;
};

__global__ __launch_bounds__(256) void k_inject(InjArgs a)
{
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= a.Nc) return;
    const int64_t f = a.inj[I];
    for (int i = 0; i < a.d; ++i) {
        a.cva[I * a.d + i] = a.va[f * a.d + i];
        a.cacc[I * a.d + i] = a.acc[f * a.d + i];
    }
    for (int i = 0; i < a.bs; ++i) a.cvp[I * a.bs + i] = a.vp[f * a.bs + i];
    a.crho[I] = a.rho[f];
    a.cmu[I] = a.mu[f];
    const uint64_t sm = a.n_s > 0 ? a.smask[f] : 0;
    if (a.n_s > 0) a.csmask[I] = sm;
    for (int s = 0; s < a.n_s; ++s) {
        // (fraction and B at n+alpha: the expressions of the fine level)
        const bool on = (sm >> s) & 1;
        const int64_t k = a.solid_ind[s];
        double al = 0.0;
        if (on) {
            const double fn = a.lphi[k * a.Nf + f], f1 = a.iphi[k * a.Nf + f];
            const double fa = fn + a.alpha * (f1 - fn);
            al = fmin(fmax(0.5 * (1.0 + fa), 0.0), 1.0);
        }
        a.cas[(int64_t)s * a.Nc + I] = al;
        for (int c = 0; c < a.nv; ++c) {
            const int64_t o = ((int64_t)s * a.Nf + f) * a.nv + c;
            a.cBa[((int64_t)s * a.Nc + I) * a.nv + c] = a.lB[o] + a.alpha * (a.iB[o] - a.lB[o]);
        }
    }
}

// ----------------------------------------------------------- smoothing ----

// x_out = x_in + omega D^-1 (b - A x_in), bs = 4, one wavefront per block row
// x_out = x + omega D^-1 (b - A x) for bs in {3, 4}: SWEEP_R block rows per
// wavefront (bsr_rows.h) with streamed value loads; lanes 0..bs-1 finish the
// rows.  Values FP64, FP32 or BF16; block inverses FP64 or FP32 (TD).
constexpr int SWEEP_R = 2;

template <int BS, typename TV, typename TD>
__global__ __launch_bounds__(256) void k_sweep_rows(int64_t n, const int32_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ col, const TV *__restrict__ val,
                                                    const TD *__restrict__ Dinv, double omega,
                                                    const double *__restrict__ b, const double *__restrict__ x,
                                                    double *__restrict__ xo, const int32_t *flag)
{
    const int64_t w = (int64_t)blockIdx.x * 4 + wave_id();
    int64_t row[SWEEP_R];
#pragma unroll
    for (int q = 0; q < SWEEP_R; ++q) row[q] = w * SWEEP_R + q;
    int k0[SWEEP_R], k1[SWEEP_R];
    row_extents<SWEEP_R>(row, n, rowptr, k0, k1);
    if (*flag == 0 || row[0] >= n) return;
    const int lane = threadIdx.x & 63;
    // row data of the update, loaded ahead of the product (lanes >= bs, and
    // rows past n, read the first row of the wavefront: in bounds, unused)
    const int rl = lane < BS ? lane : 0;
    double br[SWEEP_R], xr[SWEEP_R], d[SWEEP_R][BS], ax[SWEEP_R];
#pragma unroll
    for (int q = 0; q < SWEEP_R; ++q) {
        const int64_t rr = row[q] < n ? row[q] : row[0];
        br[q] = b[rr * BS + rl];
        xr[q] = x[rr * BS + rl];
        RowLoad<BS, TD, false>::get(Dinv + (rr * BS + rl) * BS, d[q]);
    }
    bsr_rows_dot<BS, TV, SWEEP_R, true>(k0, k1, col, val, x, lane, ax);
#pragma unroll
    for (int q = 0; q < SWEEP_R; ++q) {
        const double res = br[q] - ax[q];
        double u = 0.0;
#pragma unroll
        for (int c = 0; c < BS; ++c) u += d[q][c] * __shfl(res, c, 64);
        if (lane < BS && row[q] < n) xo[row[q] * BS + lane] = xr[q] + omega * u;
    }
}

// The same sweep with one block per lane (narrow values, bs 3 or 4): lane j
// < bs of a row's segment finishes component j of the row.
template <int BS, typename TV, typename TD, bool STN, typename TX, typename TO>
__device__ __forceinline__ void sweep_blk_rows(int64_t row0, int64_t n, const int32_t *__restrict__ rowptr,
                                               const int32_t *__restrict__ col, const uint16_t *__restrict__ smask,
                                               const int32_t *__restrict__ soff, const TV *__restrict__ val,
                                               const TD *__restrict__ Dinv, double omega,
                                               const double *__restrict__ b, const TX *__restrict__ x,
                                               TO *__restrict__ xo)
{
    constexpr int SEG = BlockSeg<BS>::SEG, RPW = BlockSeg<BS>::RPW;
    const int lane = threadIdx.x & 63, q = lane / SEG, j = lane - q * SEG;
    const int64_t row = row0 + q, rr = row < n ? row : row0;   // rr: in bounds, unused past n
    const int jj = j < BS ? j : 0;
    uint32_t m = 0;
    int oj = 0;
    if constexpr (STN) {
        m = row < n ? smask[rr] : 0u;
        oj = soff[j];
    }
    // row data of the update, loaded ahead of the product
    double bb[BS], d[BS];
    x_get<BS>(b, rr, bb);
    RowLoad<BS, TD, false>::get(Dinv + (rr * BS + jj) * BS, d);
    const double xr = (double)x[rr * BS + jj];
    int k0, k1;
    seg_extents<RPW>(row0, n, rowptr, q, k0, k1);
    double ax[BS];
    if constexpr (STN) bsr_stencil_dot<BS, TV, SEG>(k0, m, rr, oj, val, x, j, ax);
    else bsr_block_dot<BS, TV, SEG>(k0, k1, col, val, x, j, ax);
    double u = 0.0;
#pragma unroll
    for (int c = 0; c < BS; ++c) u += d[c] * (bb[c] - ax[c]);
    if (j < BS && row < n) xo[row * BS + j] = (TO)(xr + omega * u);
}

// The same sweep with one block per lane (narrow values, bs 3 or 4): lane j
// < bs of a row's segment finishes component j of the row; x and x_out in
// FP64 or FP32 (b FP64, arithmetic FP64).
// With the pattern in stencil form (smask, soff: see bsr_stencil_dot) no
// column index is read.
template <int BS, typename TV, typename TD, bool STN, typename TX, typename TO>
__global__ __launch_bounds__(256) void k_sweep_blk(int64_t n, const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ col, const uint16_t *__restrict__ smask,
                                                   const int32_t *__restrict__ soff, const TV *__restrict__ val,
                                                   const TD *__restrict__ Dinv, double omega,
                                                   const double *__restrict__ b, const TX *__restrict__ x,
                                                   TO *__restrict__ xo, const int32_t *flag)
{
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave_id()) * BlockSeg<BS>::RPW;
    if (*flag == 0 || row0 >= n) return;
    sweep_blk_rows<BS, TV, TD, STN, TX, TO>(row0, n, rowptr, col, smask, soff, val, Dinv, omega, b, x, xo);
}

// Block Gauss-Seidel on the rows of one colour, in place:
// x_r <- x_r + omega D_r^-1 (b - A x)_r for r in rows[0..nc).  No two rows of
// a colour are neighbours, so the rows of one launch read only values of
// other colours (or their own old value).
template <int BS, typename TV, typename TD>
__global__ __launch_bounds__(256) void k_gs_rows(int64_t nc, const int32_t *__restrict__ rows,
                                                 const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                                 const TV *__restrict__ val, const TD *__restrict__ Dinv, double omega,
                                                 const double *__restrict__ b, double *x, const int32_t *flag)
{
    if (*flag == 0) return;
    const int64_t w = (int64_t)blockIdx.x * 4 + wave_id();
    if (w * SWEEP_R >= nc) return;
    int64_t row[SWEEP_R];
#pragma unroll
    for (int q = 0; q < SWEEP_R; ++q) row[q] = rows[w * SWEEP_R + q < nc ? w * SWEEP_R + q : w * SWEEP_R];
    const int64_t n_end = w * SWEEP_R + SWEEP_R <= nc ? SWEEP_R : nc - w * SWEEP_R;   // valid rows of this wave
    int k0[SWEEP_R], k1[SWEEP_R];
#pragma unroll
    for (int q = 0; q < SWEEP_R; ++q) {
        k0[q] = q < n_end ? rowptr[row[q]] : 0;
        k1[q] = q < n_end ? rowptr[row[q] + 1] : 0;
    }
    const int lane = threadIdx.x & 63;
    const int rl = lane < BS ? lane : 0;
    double br[SWEEP_R], xr[SWEEP_R], d[SWEEP_R][BS], ax[SWEEP_R];
#pragma unroll
    for (int q = 0; q < SWEEP_R; ++q) {
        br[q] = b[row[q] * BS + rl];
        xr[q] = x[row[q] * BS + rl];
        RowLoad<BS, TD, false>::get(Dinv + (row[q] * BS + rl) * BS, d[q]);
    }
    bsr_rows_dot<BS, TV, SWEEP_R, true>(k0, k1, col, val, x, lane, ax);
#pragma unroll
    for (int q = 0; q < SWEEP_R; ++q) {
        const double res = br[q] - ax[q];
        double u = 0.0;
#pragma unroll
        for (int c = 0; c < BS; ++c) u += d[q][c] * __shfl(res, c, 64);
        if (lane < BS && q < n_end) x[row[q] * BS + lane] = xr[q] + omega * u;
    }
}

// x = omega D^-1 b (first sweep from x = 0)
template <typename TD>
__global__ __launch_bounds__(256) void k_sweep0(int64_t nd, int bs, const TD *__restrict__ Dinv, double omega,
                                                const double *__restrict__ b, double *__restrict__ x,
                                                const int32_t *flag)
{
    if (*flag == 0) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nd) return;
    const int64_t r = t / bs;
    const int i = (int)(t - r * bs);
    const TD *D = Dinv + r * bs * bs + i * bs;
    double s = 0.0;
    for (int c = 0; c < bs; ++c) s += (double)D[c] * b[r * bs + c];
    x[t] = omega * s;
}

// The same with one node per lane (bs 3 or 4): its block inverse and b read
// as whole rows, several loads in flight per lane.
template <int BS, typename TD, typename TO>
__global__ __launch_bounds__(256) void k_sweep0_nodes(int64_t n, const TD *__restrict__ Dinv, double omega,
                                                      const double *__restrict__ b, TO *__restrict__ x,
                                                      const int32_t *flag)
{
    if (*flag == 0) return;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double bb[BS], d[BS][BS];
    x_get<BS>(b, r, bb);
#pragma unroll
    for (int i = 0; i < BS; ++i) RowLoad<BS, TD, false>::get(Dinv + (r * BS + i) * BS, d[i]);
#pragma unroll
    for (int i = 0; i < BS; ++i) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < BS; ++c) s += d[i][c] * bb[c];
        x[r * BS + i] = (TO)(omega * s);
    }
}

// r = b - A x, RESID_R block rows per wavefront (as the plain product)
constexpr int RESID_R = 2;

template <int BS, typename TV>
__global__ __launch_bounds__(256) void k_resid_rows(int64_t n, const int32_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ col, const TV *__restrict__ val,
                                                    const double *__restrict__ b, const double *__restrict__ x,
                                                    double *__restrict__ r, const int32_t *flag)
{
    const int64_t w = (int64_t)blockIdx.x * 4 + wave_id();
    int64_t row[RESID_R];
#pragma unroll
    for (int q = 0; q < RESID_R; ++q) row[q] = w * RESID_R + q;
    int k0[RESID_R], k1[RESID_R];
    row_extents<RESID_R>(row, n, rowptr, k0, k1);
    if (*flag == 0 || row[0] >= n) return;
    const int lane = threadIdx.x & 63;
    const int rl = lane < BS ? lane : 0;
    double br[RESID_R], ax[RESID_R];
#pragma unroll
    for (int q = 0; q < RESID_R; ++q) br[q] = b[(row[q] < n ? row[q] : row[0]) * BS + rl];
    bsr_rows_dot<BS, TV, RESID_R, false>(k0, k1, col, val, x, lane, ax);
#pragma unroll
    for (int q = 0; q < RESID_R; ++q)
        if (lane < BS && row[q] < n) r[row[q] * BS + lane] = br[q] - ax[q];
}

// r = b - A x with one block per lane (narrow values, bs 3 or 4)
template <int BS, typename TV, bool STN, typename TX, typename TR>
__device__ __forceinline__ void resid_blk_rows(int64_t row0, int64_t n, const int32_t *__restrict__ rowptr,
                                               const int32_t *__restrict__ col, const uint16_t *__restrict__ smask,
                                               const int32_t *__restrict__ soff, const TV *__restrict__ val,
                                               const double *__restrict__ b, const TX *__restrict__ x,
                                               TR *__restrict__ r)
{
    constexpr int SEG = BlockSeg<BS>::SEG, RPW = BlockSeg<BS>::RPW;
    const int lane = threadIdx.x & 63, q = lane / SEG, j = lane - q * SEG;
    const int64_t row = row0 + q, rr = row < n ? row : row0;
    const double br = b[rr * BS + (j < BS ? j : 0)];
    uint32_t m = 0;
    int oj = 0;
    if constexpr (STN) {
        m = row < n ? smask[rr] : 0u;
        oj = soff[j];
    }
    int k0, k1;
    seg_extents<RPW>(row0, n, rowptr, q, k0, k1);
    double ax[BS];
    if constexpr (STN) bsr_stencil_dot<BS, TV, SEG>(k0, m, rr, oj, val, x, j, ax);
    else bsr_block_dot<BS, TV, SEG>(k0, k1, col, val, x, j, ax);
    // component j of the row, stored by lane j (unrolled: no dynamically
    // indexed private array)
#pragma unroll
    for (int c = 0; c < BS; ++c)
        if (j == c && row < n) r[row * BS + c] = br - ax[c];
}

template <int BS, typename TV, bool STN, typename TX, typename TR>
__global__ __launch_bounds__(256) void k_resid_blk(int64_t n, const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ col, const uint16_t *__restrict__ smask,
                                                   const int32_t *__restrict__ soff, const TV *__restrict__ val,
                                                   const double *__restrict__ b, const TX *__restrict__ x,
                                                   TR *__restrict__ r, const int32_t *flag)
{
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave_id()) * BlockSeg<BS>::RPW;
    if (*flag == 0 || row0 >= n) return;
    resid_blk_rows<BS, TV, STN, TX, TR>(row0, n, rowptr, col, smask, soff, val, b, x, r);
}

// --------------------------------------------------------- transfers ------

// coarse b[I] = sum over children i of I (fine nodes 2I + s, s in the Kuhn
// stencil) of w(i, I) r[i], masked by the free dofs of both levels.  Every
// load is issued unconditionally (index 0 and weight 0 outside the mesh, the
// Dirichlet mask applied by a select), so the loads of all stencil points are
// in flight together instead of one round trip per masked branch.
template <int D, typename TR>
__device__ __forceinline__ void restrict_node(const Dims &cd, const Dims &fd, const uint8_t *__restrict__ cmask,
                                              const uint8_t *__restrict__ fmask, const TR *__restrict__ r,
                                              double *__restrict__ bc, int I)
{
    constexpr int BS = D + 1;
    const int nx = cd.n[0] + 1, ny = cd.n[1] + 1;
    const int ci = I % nx, cj = (I / nx) % ny, ck = I / (nx * ny);
    double acc[BS];
#pragma unroll
    for (int c = 0; c < BS; ++c) acc[c] = 0.0;
#pragma unroll
    for (int s = 0; s < Stencil<D>::S; ++s) {
        int a, b, c3;
        Stencil<D>::off(s, a, b, c3);
        const int fi = 2 * ci + a, fj = 2 * cj + b, fk = 2 * ck + c3;
        const bool in = !(fi < 0 || fj < 0 || fk < 0 || fi > fd.n[0] || fj > fd.n[1] || fk > fd.n[2]);
        const int64_t f = in ? node_id(fd, fi, fj, fk) : 0;
        const double w = in ? (s == 0 ? 1.0 : 0.5) : 0.0;
        const int m = fmask[f];
#pragma unroll
        for (int c = 0; c < BS; ++c) {
            const double v = (double)r[f * BS + c];
            acc[c] += ((m >> c) & 1) ? w * v : 0.0;
        }
    }
    const int mc = cmask[I];
#pragma unroll
    for (int c = 0; c < BS; ++c) bc[(int64_t)I * BS + c] = ((mc >> c) & 1) ? acc[c] : 0.0;
}

template <int D, typename TR>
__global__ __launch_bounds__(256) void k_restrict(Dims cd, Dims fd, const uint8_t *__restrict__ cmask,
                                                  const uint8_t *__restrict__ fmask, const TR *__restrict__ r,
                                                  double *__restrict__ bc, const int32_t *flag)
{
    if (*flag == 0) return;
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= (cd.n[0] + 1) * (cd.n[1] + 1) * (cd.n[2] + 1)) return;
    restrict_node<D, TR>(cd, fd, cmask, fmask, r, bc, I);
}

// Restriction fused with the coarse level's first sweep from zero: node I
// gets b[I] and x[I] = omega D_I^-1 b[I] (the arithmetic of k_sweep0 per
// component), one launch instead of two.
template <int D, typename TD, typename TR>
__global__ __launch_bounds__(256) void k_restrict_sweep0(Dims cd, Dims fd, const uint8_t *__restrict__ cmask,
                                                         const uint8_t *__restrict__ fmask,
                                                         const TR *__restrict__ r, double *__restrict__ bc,
                                                         const TD *__restrict__ Dinv, double omega,
                                                         double *__restrict__ xc, const int32_t *flag)
{
    constexpr int BS = D + 1;
    if (*flag == 0) return;
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= (cd.n[0] + 1) * (cd.n[1] + 1) * (cd.n[2] + 1)) return;
    restrict_node<D, TR>(cd, fd, cmask, fmask, r, bc, I);
    double bb[BS];
#pragma unroll
    for (int c = 0; c < BS; ++c) bb[c] = bc[(int64_t)I * BS + c];
#pragma unroll
    for (int i = 0; i < BS; ++i) {
        const TD *Dr = Dinv + ((int64_t)I * BS + i) * BS;
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < BS; ++c) s += (double)Dr[c] * bb[c];
        xc[(int64_t)I * BS + i] = omega * s;
    }
}

// x[i] += sum over parents I of i of w(i, I) xc[I] (free dofs only)
template <int D, typename TX>
__device__ __forceinline__ void prolong_node(const Dims &cd, const Dims &fd, const uint8_t *__restrict__ cmask,
                                             const uint8_t *__restrict__ fmask, const double *__restrict__ xc,
                                             TX *__restrict__ x, int f)
{
    constexpr int BS = D + 1;
    const int nx = fd.n[0] + 1, ny = fd.n[1] + 1;
    const int fi = f % nx, fj = (f / nx) % ny, fk = f / (nx * ny);
    const int64_t I0 = node_id(cd, fi >> 1, fj >> 1, fk >> 1);
    const bool mid = (fi & 1) | (fj & 1) | (fk & 1);
    const int64_t I1 = mid ? node_id(cd, (fi >> 1) + (fi & 1), (fj >> 1) + (fj & 1), (fk >> 1) + (fk & 1)) : I0;
    const int m = fmask[f];
    const int m0 = cmask[I0], m1 = cmask[I1];
    const double w = mid ? 0.5 : 1.0;   // a node of the coarse mesh takes its own value once
#pragma unroll
    for (int c = 0; c < BS; ++c) {
        const double a0 = xc[I0 * BS + c], a1 = xc[I1 * BS + c], xv = (double)x[(int64_t)f * BS + c];
        const double v = ((m0 >> c) & 1 ? a0 : 0.0) + (mid && ((m1 >> c) & 1) ? a1 : 0.0);
        x[(int64_t)f * BS + c] = (TX)(((m >> c) & 1) ? xv + w * v : xv);
    }
}

template <int D, typename TX>
__global__ __launch_bounds__(256) void k_prolong(Dims cd, Dims fd, const uint8_t *__restrict__ cmask,
                                                 const uint8_t *__restrict__ fmask, const double *__restrict__ xc,
                                                 TX *__restrict__ x, const int32_t *flag)
{
    if (*flag == 0) return;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= (fd.n[0] + 1) * (fd.n[1] + 1) * (fd.n[2] + 1)) return;
    prolong_node<D, TX>(cd, fd, cmask, fmask, xc, x, f);
}

// ------------------------------------------------ Galerkin coarsening ----
//
// A_c = P^T A_f P with the transfers of the V-cycle: P interpolates linearly
// on the nested Kuhn meshes (weights 1 and 1/2), masked on the Dirichlet
// dofs of both levels, so that coarse block (I, J) sums
//   w(i, I) w(j, J) M_f(i) A_f(i, j) M_f(j)
// over the fine nodes i of I's star (2I + s, s in the Kuhn stencil) and the
// columns j of row i whose parents J (the coarse node at j, or the two ends
// of the coarse edge j is the midpoint of) lie in row I; then coarse masks,
// unit rows for Dirichlet dofs of the coarse level.  One wavefront per coarse
// row; its blocks accumulate in LDS (FP64); the pattern of row I is the
// coarse mesh's (the product of P1 spaces of nested meshes stays within it).
struct RapArgs {
    Dims cd, fd;
    int64_t nc;
    const int32_t *frow, *fcol, *crow, *ccol;
    const uint8_t *fmask, *cmask;
    int32_t *miss;          // set when a contribution had no slot (never expected)
};

template <int D, typename TF, typename TC>
__global__ __launch_bounds__(256) void k_rap_rows(RapArgs a, const TF *__restrict__ fval, TC *__restrict__ cval,
                                                  uint16_t *__restrict__ cval16)
{
    constexpr int BS = D + 1, B2 = BS * BS, BP = B2 | 1, S = Stencil<D>::S, MAXC = Stencil<D>::S;
    __shared__ double acc[4][MAXC * BP];
    __shared__ int32_t ccol[4][MAXC];
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int64_t I = (int64_t)blockIdx.x * 4 + w;
    const bool live = I < a.nc;
    const int nxc = a.cd.n[0] + 1, nyc = a.cd.n[1] + 1;
    int clen = 0;
    int64_t c0 = 0;
    if (live) {
        c0 = a.crow[I];
        clen = a.crow[I + 1] - (int)c0;
        if (lane < clen) ccol[w][lane] = a.ccol[c0 + lane];
    }
    for (int t = lane; t < MAXC * BP; t += 64) acc[w][t] = 0.0;
    __syncthreads();
    if (live) {
        const int ci = (int)(I % nxc), cj = (int)((I / nxc) % nyc), ck = D == 3 ? (int)(I / ((int64_t)nxc * nyc)) : 0;
        const int nxf = a.fd.n[0] + 1, nyf = a.fd.n[1] + 1;
        for (int t = lane; t < S * MAXC; t += 64) {
            const int s = t / MAXC, kk = t % MAXC;
            int o0, o1, o2;
            Stencil<D>::off(s, o0, o1, o2);
            const int fi = 2 * ci + o0, fj = 2 * cj + o1, fk = 2 * ck + o2;
            if (fi < 0 || fj < 0 || fk < 0 || fi > a.fd.n[0] || fj > a.fd.n[1] || (D == 3 && fk > a.fd.n[2])) continue;
            const int64_t i = node_id(a.fd, fi, fj, fk);
            const int64_t k = a.frow[i] + kk;
            if (k >= a.frow[i + 1]) continue;
            const int mi = a.fmask[i];
            if (mi == 0) continue;
            const int64_t j = a.fcol[k];
            const int mj = a.fmask[j];
            if (mj == 0) continue;
            const double wi = s == 0 ? 1.0 : 0.5;
            // parents of j: the coarse node at j, or the ends of its coarse edge
            const int gi = (int)(j % nxf), gj = (int)((j / nxf) % nyf), gk = D == 3 ? (int)(j / ((int64_t)nxf * nyf)) : 0;
            const int odd = (gi & 1) | (gj & 1) | (gk & 1);
            const int64_t J0 = node_id(a.cd, gi >> 1, gj >> 1, gk >> 1);
            const int64_t J1 = odd ? node_id(a.cd, (gi >> 1) + (gi & 1), (gj >> 1) + (gj & 1), (gk >> 1) + (gk & 1)) : -1;
            const double wj = odd ? 0.5 : 1.0;
            double blk[B2];
            const TF *src = fval + k * B2;
#pragma unroll
            for (int r = 0; r < BS; ++r)
#pragma unroll
                for (int c = 0; c < BS; ++c)
                    blk[r * BS + c] = (((mi >> r) & 1) && ((mj >> c) & 1)) ? wi * wj * (double)src[r * BS + c] : 0.0;
#pragma unroll
            for (int par = 0; par < 2; ++par) {
                const int64_t J = par == 0 ? J0 : J1;
                if (J < 0) continue;
                int q = -1;
                for (int u = 0; u < clen; ++u)
                    if (ccol[w][u] == J) q = u;
                if (q < 0) {
                    *a.miss = 1;
                    continue;
                }
                double *dst = &acc[w][q * BP];
#pragma unroll
                for (int e = 0; e < B2; ++e)
                    if (blk[e] != 0.0) atomicAdd(dst + e, blk[e]);
            }
        }
    }
    __syncthreads();
    if (!live) return;
    const int mI = a.cmask[I];
    for (int t = lane; t < clen * B2; t += 64) {
        const int q = t / B2, e = t % B2, r = e / BS, c = e % BS;
        const int64_t J = ccol[w][q];
        const int mJ = a.cmask[J];
        double v;
        if (!((mI >> r) & 1)) v = (J == I && r == c) ? 1.0 : 0.0;   // Dirichlet dof: unit row
        else v = ((mJ >> c) & 1) ? acc[w][q * BP + e] : 0.0;
        cval[(c0 + q) * B2 + e] = (TC)v;
        if (cval16) cval16[(c0 + q) * B2 + e] = to_bf16_rne((float)v);
    }
}

// -------------------------------------------------------- coarsest level --

// Dense matrix of the coarsest level restricted to its free dofs: fidx maps a
// dof to its free index (-1 for Dirichlet dofs, whose rows are unit rows).
// M must be zero beforehand; one thread per (block, row of the block) writes
// the free entries of that block row.
template <typename TV>
__global__ void k_dense_fill(int64_t nnzb, int bs, const int32_t *rowptr, const int32_t *col, const TV *val,
                             const int32_t *fidx, double *M, int64_t nd, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nnzb * bs) return;
    const int64_t k = t / bs;
    const int i = (int)(t - k * bs);
    // block row of block k: the last r with rowptr[r] <= k
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (rowptr[mid] <= k) lo = mid;
        else hi = mid - 1;
    }
    const int fi = fidx[lo * bs + i];
    if (fi < 0) return;
    const int64_t c = col[k];
    for (int j = 0; j < bs; ++j) {
        const int fj = fidx[c * bs + j];
        if (fj >= 0) M[fi * nd + fj] = (double)val[(k * bs + i) * bs + j];
    }
}

// Gauss-Jordan inversion with partial pivoting, one workgroup; M is
// destroyed, Inv receives the inverse.
__global__ __launch_bounds__(256) void k_gauss_jordan(double *M, double *Inv, int nd)
{
    __shared__ double sv[256];
    __shared__ int si[256];
    __shared__ int piv;
    const int t = threadIdx.x;
    for (int64_t e = t; e < (int64_t)nd * nd; e += 256) Inv[e] = (e / nd == e % nd) ? 1.0 : 0.0;
    __syncthreads();
    for (int k = 0; k < nd; ++k) {
        double best = -1.0;
        int bi = k;
        for (int i = k + t; i < nd; i += 256) {
            const double a = fabs(M[(int64_t)i * nd + k]);
            if (a > best) {
                best = a;
                bi = i;
            }
        }
        sv[t] = best;
        si[t] = bi;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (t < off && sv[t + off] > sv[t]) {
                sv[t] = sv[t + off];
                si[t] = si[t + off];
            }
            __syncthreads();
        }
        if (t == 0) piv = si[0];
        __syncthreads();
        const int p = piv;
        if (p != k)
            for (int j = t; j < nd; j += 256) {
                double a = M[(int64_t)k * nd + j];
                M[(int64_t)k * nd + j] = M[(int64_t)p * nd + j];
                M[(int64_t)p * nd + j] = a;
                a = Inv[(int64_t)k * nd + j];
                Inv[(int64_t)k * nd + j] = Inv[(int64_t)p * nd + j];
                Inv[(int64_t)p * nd + j] = a;
            }
        __syncthreads();
        const double d = M[(int64_t)k * nd + k];
        const double inv = d != 0.0 ? 1.0 / d : 0.0;
        __syncthreads();
        for (int j = t; j < nd; j += 256) {
            M[(int64_t)k * nd + j] *= inv;
            Inv[(int64_t)k * nd + j] *= inv;
        }
        __syncthreads();
        for (int64_t e = t; e < (int64_t)nd * nd; e += 256) {
            const int i = (int)(e / nd), j = (int)(e % nd);
            if (i == k) continue;
            const double f = M[(int64_t)i * nd + k];
            if (j != k) M[e] -= f * M[(int64_t)k * nd + j];
            Inv[e] -= f * Inv[(int64_t)k * nd + j];
        }
        __syncthreads();
        for (int i = t; i < nd; i += 256)
            if (i != k) M[(int64_t)i * nd + k] = 0.0;
        __syncthreads();
    }
}

// The same inversion with the augmented matrix [M | I] resident in LDS (nd
// up to GJ_LDS_MAX): no global memory round trip inside the pivot loop.
constexpr int GJ_LDS_MAX = 88;
inline size_t gj_lds_bytes(int nd) { return sizeof(double) * ((size_t)2 * nd * nd + nd); }

__global__ __launch_bounds__(256) void k_gauss_jordan_lds(const double *__restrict__ M, double *__restrict__ Inv, int nd)
{
    // thread j owns column j of [M | I] (2 nd <= blockDim.x columns; one
    // wavefront when 2 nd <= 64): the swap, the scaling and the elimination
    // of a pivot step touch only the thread's own column, so a step needs
    // two barriers (after the pivot search and the broadcast of the pivot
    // column, and after the update)
    extern __shared__ double sm[];
    double *A = sm;                  // [nd][2 nd]
    double *colk = sm + 2 * nd * nd; // [nd] pivot column after the swap, 0 at row k
    __shared__ int piv;
    __shared__ double pinv;
    const int t = threadIdx.x, W = 2 * nd;
    for (int e = t; e < nd * W; e += (int)blockDim.x) {
        const int i = e / W, j = e - i * W;
        A[e] = j < nd ? M[i * nd + j] : (j - nd == i ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int k = 0; k < nd; ++k) {
        if (t < 64) {
            // pivot: largest |A[i][k]| over i >= k (lowest i among equals)
            double best = -1.0;
            int bi = nd;
            for (int i = k + t; i < nd; i += 64) {
                const double a = fabs(A[i * W + k]);
                if (a > best) {
                    best = a;
                    bi = i;
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double ob = __shfl_xor(best, o, 64);
                const int oi = __shfl_xor(bi, o, 64);
                if (ob > best || (ob == best && oi < bi)) {
                    best = ob;
                    bi = oi;
                }
            }
            const int p = bi < nd ? bi : k;
            for (int i = t; i < nd; i += 64) colk[i] = i == k ? 0.0 : A[(i == p ? k : i) * W + k];
            if (t == 0) {
                piv = p;
                const double d = A[p * W + k];
                pinv = d != 0.0 ? 1.0 / d : 0.0;
            }
        }
        __syncthreads();
        if (t < W) {
            const int p = piv;
            const double akj = A[p * W + t] * pinv;
            if (p != k) A[p * W + t] = A[k * W + t];
            A[k * W + t] = akj;
            for (int i = 0; i < nd; ++i)
                if (i != k) A[i * W + t] = t == k ? 0.0 : A[i * W + t] - colk[i] * akj;
        }
        __syncthreads();
    }
    for (int e = t; e < nd * nd; e += (int)blockDim.x) {
        const int i = e / nd, j = e - i * nd;
        Inv[e] = A[i * W + nd + j];
    }
}

// x = A^-1 b on the coarsest level: free dofs from the dense inverse, the
// Dirichlet dofs zero
template <int T>
__device__ __forceinline__ void dense_apply_block(const double *Inv, int nd, const int32_t *free_dof, int64_t ndof,
                                                  const double *b, double *x, double *bl /* LDS, nd */)
{
    for (int j = threadIdx.x; j < nd; j += T) bl[j] = b[free_dof[j]];
    for (int64_t i = threadIdx.x; i < ndof; i += T) x[i] = 0.0;
    __syncthreads();
    for (int i = threadIdx.x; i < nd; i += T) {
        const double *row = Inv + (int64_t)i * nd;
        double s = 0.0;
#pragma unroll 8
        for (int j = 0; j < nd; ++j) s += row[j] * bl[j];
        x[free_dof[i]] = s;
    }
}

__global__ __launch_bounds__(256) void k_dense_apply(const double *Inv, int nd, const int32_t *free_dof, int64_t ndof,
                                                     const double *b, double *x, const int32_t *flag)
{
    __shared__ double bl[512];   // the free entries of b (nd <= 512)
    if (*flag == 0) return;
    dense_apply_block<256>(Inv, nd, free_dof, ndof, b, x, bl);
}

// FP32 copy of a matrix's values (multigrid works on FP32 matrices)
__global__ void k_to_f32(const double *a, float *b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

// BF16 copy (round to nearest even)
template <typename T> __global__ void k_to_bf16(const T *a, uint16_t *b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = to_bf16_rne((float)a[i]);
}

// ------------------------------------------------------------------ host --

eft_status kuhn_mesh(int d, const int n[3], std::vector<int32_t> &conn)
{
    conn.clear();
    if (d == 2) {
        const int64_t nx1 = n[0] + 1;
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                const int32_t v00 = (int32_t)(i + nx1 * j), v10 = v00 + 1, v01 = (int32_t)(v00 + nx1), v11 = v01 + 1;
                const int32_t t[6] = {v00, v10, v11, v00, v11, v01};
                conn.insert(conn.end(), t, t + 6);
            }
        return EFT_OK;
    }
    const int64_t sx = 1, sy = n[0] + 1, sz = (int64_t)(n[0] + 1) * (n[1] + 1);
    const int64_t st[3] = {sx, sy, sz};
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    const bool even[6] = {true, false, false, true, true, false};
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                const int64_t v0 = i * sx + j * sy + k * sz;
                for (int p = 0; p < 6; ++p) {
                    const int64_t a = v0 + st[perms[p][0]], b = a + st[perms[p][1]], c = b + st[perms[p][2]];
                    if (even[p]) {
                        const int32_t t[4] = {(int32_t)v0, (int32_t)a, (int32_t)b, (int32_t)c};
                        conn.insert(conn.end(), t, t + 4);
                    } else {
                        const int32_t t[4] = {(int32_t)v0, (int32_t)b, (int32_t)a, (int32_t)c};
                        conn.insert(conn.end(), t, t + 4);
                    }
                }
            }
    return EFT_OK;
}

template <typename T> eft_status dmal(eft_ctx *ctx, T **p, int64_t count)
{
    *p = nullptr;
    if (count <= 0) count = 1;
    if (hipMalloc((void **)p, sizeof(T) * (size_t)count) != hipSuccess) {
        ctx->err = "out of device memory (multigrid)";
        return EFT_ENOMEM;
    }
    return EFT_OK;
}

template <typename T> eft_status dput(eft_ctx *ctx, T **p, const std::vector<T> &h)
{
    EFT_TRY(dmal(ctx, p, (int64_t)h.size()));
    if (!h.empty()) EFT_HIP(hipMemcpy(*p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
    return EFT_OK;
}

Dims dims_of(const MGLevel &L) { return Dims{{L.n[0], L.n[1], L.n[2]}}; }

}  // namespace

// Node graph of a simplex mesh: sorted columns per row (self included), the
// diagonal position per row and, per element, the position of each node
// pair (a, b) in row a.  Grouped by node, the incidence entries (element << 2
// | local node a) and, per entry, the block slots of its row: byte k of
// islot is the position, within row a, of the column of local node
// (a + k) mod nn.
// Stencil form of a block pattern: when the column offsets c - r of all
// entries take at most maxs distinct values, soff gets them in ascending order
// (padded with zeros to maxs) and smask[r] the bits of the offsets row r has.
// Rows list their columns in ascending order, so block k0[r] + (number of set
// bits below s) of row r is the one at column r + soff[s].
bool eft_stencil_form(int64_t n, const std::vector<int32_t> &rowptr, const std::vector<int32_t> &col, int maxs,
                      std::vector<int32_t> &soff, std::vector<uint16_t> &smask)
{
    if (maxs > 16) return false;
    std::vector<int64_t> offs;
    for (int64_t r = 0; r < n; ++r)
        for (int32_t k = rowptr[r]; k < rowptr[r + 1]; ++k) {
            const int64_t o = (int64_t)col[k] - r;
            if (std::find(offs.begin(), offs.end(), o) == offs.end()) {
                if ((int)offs.size() == maxs) return false;
                offs.push_back(o);
            }
        }
    std::sort(offs.begin(), offs.end());
    soff.assign(maxs, 0);
    for (size_t s = 0; s < offs.size(); ++s) soff[s] = (int32_t)offs[s];
    smask.assign(n, 0);
    for (int64_t r = 0; r < n; ++r) {
        uint32_t m = 0;
        for (int32_t k = rowptr[r]; k < rowptr[r + 1]; ++k) {
            const int64_t o = (int64_t)col[k] - r;
            m |= 1u << (int)(std::lower_bound(offs.begin(), offs.end(), o) - offs.begin());
        }
        smask[r] = (uint16_t)m;
    }
    return true;
}

constexpr int64_t NS_PAIRS = 512;   // (row, element) pairs per momentum-assembly workgroup

eft_status eft_build_graph(int64_t N, int64_t E, int nn, const int32_t *conn, std::vector<int32_t> &rowptr,
                           std::vector<int32_t> &col, std::vector<int32_t> &diag, std::vector<int32_t> &epos,
                           std::vector<int32_t> &iptr, std::vector<int32_t> &ient, std::vector<uint32_t> &islot,
                           int &maxc, int &rpb, int &rpb_ns, std::string &err)
{
    if (E >= (1LL << 29) || (int64_t)E * nn >= 2000000000LL) {
        err = "too many elements for 32-bit incidence entries";
        return EFT_EINVAL;
    }
    std::vector<int64_t> ioff(N + 1, 0);
    for (int64_t t = 0; t < E * nn; ++t) ioff[conn[t] + 1]++;
    for (int64_t p = 0; p < N; ++p) ioff[p + 1] += ioff[p];
    std::vector<int32_t> inc(ioff[N]);
    {
        std::vector<int64_t> fill(ioff.begin(), ioff.end() - 1);
        for (int64_t e = 0; e < E; ++e)
            for (int a = 0; a < nn; ++a) inc[fill[conn[e * nn + a]]++] = (int32_t)e;
    }
    rowptr.assign(N + 1, 0);
    col.clear();
    col.reserve((size_t)N * (nn == 4 ? 16 : 8));
    std::vector<int32_t> buf;
    for (int64_t p = 0; p < N; ++p) {
        buf.clear();
        for (int64_t t = ioff[p]; t < ioff[p + 1]; ++t)
            for (int a = 0; a < nn; ++a) buf.push_back(conn[(int64_t)inc[t] * nn + a]);
        if (buf.empty()) buf.push_back((int32_t)p);
        std::sort(buf.begin(), buf.end());
        buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
        col.insert(col.end(), buf.begin(), buf.end());
        if (col.size() > 2000000000ULL) {
            err = "node graph too large for 32-bit indices";
            return EFT_EINVAL;
        }
        rowptr[p + 1] = (int32_t)col.size();
    }
    diag.assign(N, 0);
    epos.assign((size_t)E * nn * nn, 0);
    for (int64_t p = 0; p < N; ++p)
        diag[p] = (int32_t)(std::lower_bound(col.begin() + rowptr[p], col.begin() + rowptr[p + 1], (int32_t)p) - col.begin());
    for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < nn; ++a) {
            const int32_t r = conn[e * nn + a];
            for (int b = 0; b < nn; ++b)
                epos[(size_t)e * nn * nn + a * nn + b] = (int32_t)(
                    std::lower_bound(col.begin() + rowptr[r], col.begin() + rowptr[r + 1], conn[e * nn + b]) - col.begin());
        }
    // node -> incident (element << 2 | local index), grouped by node
    iptr.assign(N + 1, 0);
    ient.assign((size_t)E * nn, 0);
    int maxinc = 1;
    {
        std::vector<int64_t> fill(N, 0);
        for (int64_t p = 0; p < N; ++p) {
            iptr[p + 1] = (int32_t)ioff[p + 1];
            maxinc = std::max<int>(maxinc, (int)(ioff[p + 1] - ioff[p]));
        }
        for (int64_t e = 0; e < E; ++e)
            for (int a = 0; a < nn; ++a) {
                const int32_t p = conn[e * nn + a];
                ient[ioff[p] + fill[p]++] = (int32_t)((e << 2) | a);
            }
    }
    maxc = 1;
    for (int64_t p = 0; p < N; ++p) maxc = std::max(maxc, rowptr[p + 1] - rowptr[p]);
    if (maxc > 255) {
        err = "a node couples to more than 255 nodes";
        return EFT_EINVAL;
    }
    islot.assign((size_t)E * nn, 0);
    for (int64_t p = 0; p < N; ++p)
        for (int64_t t = ioff[p]; t < ioff[p + 1]; ++t) {
            const int64_t e = ient[t] >> 2;
            const int a = ient[t] & 3;
            uint32_t w = 0;
            for (int k = 0; k < nn; ++k) {
                const int b = (a + k) % nn;
                w |= (uint32_t)(epos[(size_t)e * nn * nn + a * nn + b] - rowptr[p]) << (8 * k);
            }
            islot[t] = w;
        }
    // rows per band-assembly workgroup: about two incident elements per
    // thread, and the row accumulators within 40 KB of LDS (a B-system block
    // accumulates 1 + 3 x 3 numbers, 11 doubles with the odd padding; a
    // residual row 7)
    const int64_t rowbytes = (int64_t)maxc * 11 * 8 + 7 * 8;
    // (at most 64: the units stage their rows' metadata in LDS arrays of 64)
    rpb = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(512 / maxinc, 40960 / rowbytes), 64));
    // the momentum/mass assembly (padded nn x nn blocks): about NS_PAIRS
    // (row, element) pairs per 256-thread workgroup, within 64 KB of LDS (its
    // register count allows two workgroups per compute unit)
    const int64_t rowbytes_ns = (int64_t)maxc * ((nn * nn) | 1) * 8 + (nn | 1) * 8;
    rpb_ns = (int)std::max<int64_t>(1, std::min<int64_t>(NS_PAIRS / maxinc, 65536 / rowbytes_ns));
    return EFT_OK;
}

// Build the coarse levels.  grid: cells per axis of the fine mesh (known to be
// a structured Kuhn mesh); dmask0: Dirichlet dof bits of each fine node.
// rows of a structured level ordered by parity colour; per colour the
// number of rows and of matrix blocks (rowptr on the host)
static eft_status colour_rows(eft_ctx *ctx, MGLevel &L, int d, const std::vector<int32_t> &rowptr)
{
    const int64_t n0 = L.n[0] + 1, n1 = L.n[1] + 1;
    L.ncolor = 1 << d;
    std::vector<int64_t> cnt(9, 0);
    std::vector<int> colour(L.N);
    for (int64_t p = 0; p < L.N; ++p) {
        const int64_t i = p % n0, j = (p / n0) % n1, k = p / (n0 * n1);
        colour[p] = (int)((i & 1) | ((j & 1) << 1) | ((k & 1) << 2));
        cnt[colour[p] + 1] += 1;
    }
    for (int c = 0; c < 8; ++c) cnt[c + 1] += cnt[c];
    std::vector<int32_t> rows(L.N);
    std::vector<int64_t> pos(cnt.begin(), cnt.end());
    for (int c = 0; c < 8; ++c) L.cnnz[c] = 0;
    for (int64_t p = 0; p < L.N; ++p) {
        rows[pos[colour[p]]++] = (int32_t)p;
        L.cnnz[colour[p]] += rowptr[p + 1] - rowptr[p];
    }
    for (int c = 0; c <= 8; ++c) L.coff[c] = cnt[c];
    return dput(ctx, &L.crow, rows);
}

eft_status eft_mg_create(eft_ctx *ctx, const int32_t *grid, const std::vector<uint8_t> &dmask0)
{
    const int d = ctx->dim, bs = ctx->bs, nv = ctx->nv, nn = d + 1;
    const int full = (1 << bs) - 1;
    ctx->mg.clear();
    MGLevel L0;
    for (int k = 0; k < 3; ++k) L0.n[k] = k < d ? grid[k] : 0;
    L0.N = ctx->N;
    L0.E = ctx->E;
    std::vector<uint8_t> fm(ctx->N);
    for (int64_t p = 0; p < ctx->N; ++p) fm[p] = (uint8_t)(full & ~dmask0[p]);
    EFT_TRY(dput(ctx, &L0.fmask, fm));
    EFT_TRY(dmal(ctx, &L0.Dinv32, ctx->N * bs * bs));
    EFT_TRY(dmal(ctx, &L0.x, ctx->N * bs));
    EFT_TRY(dmal(ctx, &L0.x2, ctx->N * bs));
    EFT_TRY(dmal(ctx, &L0.r, ctx->N * bs));
    {
        std::vector<int32_t> rp0(ctx->N + 1);
        EFT_HIP(hipMemcpy(rp0.data(), ctx->J.rowptr, sizeof(int32_t) * (ctx->N + 1), hipMemcpyDeviceToHost));
        EFT_TRY(colour_rows(ctx, L0, d, rp0));
    }
    ctx->mg.push_back(L0);
    // level-0 coordinates on the host, to carry to the coarse levels
    std::vector<double> xyz0(ctx->N * d);
    EFT_HIP(hipMemcpy(xyz0.data(), ctx->xyz, sizeof(double) * xyz0.size(), hipMemcpyDeviceToHost));
    std::vector<int64_t> inj_prev(ctx->N);
    for (int64_t p = 0; p < ctx->N; ++p) inj_prev[p] = p;
    for (;;) {
        const MGLevel &F = ctx->mg.back();
        // coarsen while every axis has an even cell count (down to one cell
        // per axis, so that anisotropic boxes still end on a coarsest level
        // small enough for the LDS-resident dense inverse)
        bool can = true;
        for (int k = 0; k < d; ++k) can &= F.n[k] % 2 == 0 && F.n[k] >= 2;
        if (!can) break;
        MGLevel C;
        for (int k = 0; k < 3; ++k) C.n[k] = k < d ? F.n[k] / 2 : 0;
        C.N = 1;
        for (int k = 0; k < d; ++k) C.N *= C.n[k] + 1;
        std::vector<int32_t> conn;
        EFT_TRY(kuhn_mesh(d, C.n, conn));
        C.E = (int64_t)conn.size() / nn;
        std::vector<int64_t> inj(C.N);
        std::vector<int32_t> inj32(C.N);
        std::vector<double> xyz(C.N * d);
        std::vector<uint8_t> cm(C.N);
        std::vector<int32_t> dn;
        std::vector<uint8_t> dmk;
        for (int64_t I = 0; I < C.N; ++I) {
            const int64_t i = I % (C.n[0] + 1), j = (I / (C.n[0] + 1)) % (C.n[1] + 1),
                          k = d == 3 ? I / ((int64_t)(C.n[0] + 1) * (C.n[1] + 1)) : 0;
            const int64_t f = 2 * i + (F.n[0] + 1) * (2 * j + (int64_t)(F.n[1] + 1) * 2 * k);
            inj[I] = inj_prev[f];
            inj32[I] = (int32_t)inj[I];
            for (int c = 0; c < d; ++c) xyz[I * d + c] = xyz0[inj[I] * d + c];
            const uint8_t dm = dmask0[inj[I]];
            cm[I] = (uint8_t)(full & ~dm);
            if (dm) {
                dn.push_back((int32_t)I);
                dmk.push_back(dm);
            }
        }
        std::vector<int32_t> rowptr, col, diag, epos, iptr, ient;
        std::vector<uint32_t> islot;
        int rpb_band = 1;   // (no band systems on the coarse levels)
        EFT_TRY(eft_build_graph(C.N, C.E, nn, conn.data(), rowptr, col, diag, epos, iptr, ient, islot, C.maxc,
                                rpb_band, C.rpb, ctx->err));
        EFT_TRY(dput(ctx, &C.iptr, iptr));
        EFT_TRY(dput(ctx, &C.ient, ient));
        EFT_TRY(dput(ctx, &C.islot, islot));
        EFT_TRY(dput(ctx, &C.conn, conn));
        EFT_TRY(dput(ctx, &C.epos, epos));
        EFT_TRY(dput(ctx, &C.inj, inj32));
        EFT_TRY(dput(ctx, &C.xyz, xyz));
        EFT_TRY(dput(ctx, &C.fmask, cm));
        C.n_dir = (int64_t)dn.size();
        EFT_TRY(dput(ctx, &C.dir_node, dn));
        EFT_TRY(dput(ctx, &C.dir_mask, dmk));
        C.A.bs = bs;
        C.A.n = C.N;
        C.A.nnzb = (int64_t)col.size();
        EFT_TRY(dput(ctx, &C.A.rowptr, rowptr));
        EFT_TRY(dput(ctx, &C.A.col, col));
        EFT_TRY(dput(ctx, &C.A.diag, diag));
        {
            std::vector<int32_t> so;
            std::vector<uint16_t> sm;
            if (eft_stencil_form(C.N, rowptr, col, bs == 4 ? 16 : 8, so, sm)) {
                EFT_TRY(dput(ctx, &C.A.stn_mask, sm));
                EFT_TRY(dput(ctx, &C.A.stn_off, so));
            }
        }
        EFT_TRY(dmal(ctx, &C.A.val, C.A.nnzb * bs * bs));
        EFT_TRY(dmal(ctx, &C.va, C.N * d));
        EFT_TRY(dmal(ctx, &C.acc, C.N * d));
        EFT_TRY(dmal(ctx, &C.rho, C.N));
        EFT_TRY(dmal(ctx, &C.mu, C.N));
        EFT_TRY(dmal(ctx, &C.as, C.N * std::max(ctx->n_s, 1)));
        EFT_TRY(dmal(ctx, &C.Ba, C.N * nv * std::max(ctx->n_s, 1)));
        EFT_TRY(dmal(ctx, &C.smask, C.N));
        EFT_TRY(dmal(ctx, &C.vp, C.N * bs));
        EFT_TRY(dmal(ctx, &C.R, C.N * bs));
        EFT_TRY(dmal(ctx, &C.Dinv, C.N * bs * bs));
        EFT_TRY(dmal(ctx, &C.x, C.N * bs));
        EFT_TRY(dmal(ctx, &C.x2, C.N * bs));
        EFT_TRY(dmal(ctx, &C.b, C.N * bs));
        EFT_TRY(dmal(ctx, &C.r, C.N * bs));
        EFT_TRY(colour_rows(ctx, C, d, rowptr));
        inj_prev = inj;
        ctx->mg.push_back(C);
    }
    if (ctx->mg.size() < 2) {
        eft_mg_free(ctx);
        return EFT_OK;
    }
    // the fine-level smoother works on an FP32 copy of the Jacobian (the
    // preconditioner only shapes the Krylov space; FGMRES keeps FP64), which
    // halves the bytes of the most expensive kernel of the cycle.  The coarse
    // levels are assembled in FP32 as well, except the coarsest, whose FP64
    // values feed the dense inverse.
    for (size_t l = 1; l + 1 < ctx->mg.size(); ++l) {
        MGLevel &C = ctx->mg[l];
        C.A.fp32 = true;
        EFT_TRY(dmal(ctx, &C.A.val32, C.A.nnzb * bs * bs));
        EFT_TRY(dmal(ctx, &C.A.val16, C.A.nnzb * bs * bs));
        EFT_TRY(dmal(ctx, &C.Dinv32, C.N * bs * bs));
    }
    EFT_TRY(dmal(ctx, &ctx->mg_miss, 1));
    EFT_HIP(hipMemset(ctx->mg_miss, 0, sizeof(int32_t)));
    MGLevel &F0 = ctx->mg[0];
    F0.A.bs = bs;
    F0.A.n = ctx->N;
    F0.A.nnzb = ctx->J.nnzb;
    F0.A.rowptr = ctx->J.rowptr;
    F0.A.col = ctx->J.col;
    F0.A.diag = ctx->J.diag;
    F0.A.stn_mask = ctx->J.stn_mask;
    F0.A.stn_off = ctx->J.stn_off;
    if (bs == 3 || bs == 4) {   // FP32 iterate and residual of the finest level's cycle
        EFT_TRY(dmal(ctx, &F0.xf, F0.A.n * bs));
        EFT_TRY(dmal(ctx, &F0.xf2, F0.A.n * bs));
        EFT_TRY(dmal(ctx, &F0.rf, F0.A.n * bs));
        EFT_TRY(dmal(ctx, &F0.Dinv16, F0.A.n * bs * bs));
    }
    F0.A.fp32 = true;   // storage (FP32 or BF16) is chosen and allocated in eft_mg_setup
    // coarsest level: dense inverse over its free dofs
    const MGLevel &Lc = ctx->mg.back();
    std::vector<uint8_t> cmh(Lc.N);
    EFT_HIP(hipMemcpy(cmh.data(), Lc.fmask, Lc.N, hipMemcpyDeviceToHost));
    std::vector<int32_t> fidx(Lc.N * bs, -1), fdof;
    for (int64_t I = 0; I < Lc.N; ++I)
        for (int c = 0; c < bs; ++c)
            if ((cmh[I] >> c) & 1) {
                fidx[I * bs + c] = (int32_t)fdof.size();
                fdof.push_back((int32_t)(I * bs + c));
            }
    ctx->mg_nd = (int64_t)fdof.size();
    if (ctx->mg_nd > 0 && ctx->mg_nd <= 512) {
        EFT_TRY(dput(ctx, &ctx->mg_fidx, fidx));
        EFT_TRY(dput(ctx, &ctx->mg_free, fdof));
        EFT_TRY(dmal(ctx, &ctx->mg_dense, ctx->mg_nd * ctx->mg_nd));
        EFT_TRY(dmal(ctx, &ctx->mg_inv, ctx->mg_nd * ctx->mg_nd));
        if (ctx->mg_nd <= GJ_LDS_MAX)
            EFT_HIP(hipFuncSetAttribute((const void *)k_gauss_jordan_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)gj_lds_bytes(GJ_LDS_MAX)));
    }
    return EFT_OK;
}

void eft_mg_free(eft_ctx *ctx)
{
    auto fr = [](void *p) {
        if (p) (void)hipFree(p);
    };
    for (size_t l = 0; l < ctx->mg.size(); ++l) {
        MGLevel &L = ctx->mg[l];
        if (l > 0) {
            fr(L.conn); fr(L.epos); fr(L.inj); fr(L.xyz); fr(L.va); fr(L.acc); fr(L.rho); fr(L.mu); fr(L.as);
            fr(L.Ba); fr(L.smask); fr(L.vp); fr(L.R); fr(L.dir_node); fr(L.dir_mask); fr(L.A.rowptr); fr(L.A.col); fr(L.A.diag); fr(L.A.stn_mask); fr(L.A.stn_off);
            fr(L.A.val); fr(L.b); fr(L.iptr); fr(L.ient); fr(L.islot);
        }
        fr(L.fmask); fr(L.Dinv); fr(L.Dinv32); fr(L.x); fr(L.x2); fr(L.r); fr(L.A.val32); fr(L.A.val16);
        fr(L.xf); fr(L.xf2); fr(L.rf); fr(L.Dinv16);
        fr(L.crow);
    }
    ctx->mg.clear();
    fr(ctx->mg_dense);
    fr(ctx->mg_inv);
    fr(ctx->mg_fidx);
    fr(ctx->mg_free);
    fr(ctx->mg_miss);
    ctx->mg_fidx = ctx->mg_free = ctx->mg_miss = nullptr;
    ctx->mg_dense = ctx->mg_inv = nullptr;
    ctx->mg_nd = 0;
}

bool eft_mg_enabled(const eft_ctx *ctx, const eft_matrix *A)
{
    // the V-cycle preconditions the momentum solves, or is the base the
    // learned preconditioner corrects
    return (ctx->par.precond == 1 || (ctx->par.precond == 2 && ctx->par.nn_base == 1)) && ctx->mg.size() >= 2 &&
           A == &ctx->J;
}

bool eft_mg_active(const eft_ctx *ctx, const eft_matrix *A)
{
    return eft_mg_enabled(ctx, A) && ctx->mg_valid;
}

// Storage of the finest level's narrow copy (BF16 with mg_bf16, else FP32),
// reserved at creation and when mg_bf16 changes, so that the set-up inside a
// time step allocates nothing.
eft_status eft_mg_reserve(eft_ctx *ctx)
{
    if (ctx->mg.size() < 2) return EFT_OK;
    MGLevel &F0 = ctx->mg[0];
    const int64_t nv = ctx->J.nnzb * ctx->bs * ctx->bs;
    if (ctx->par.mg_bf16 && !F0.A.val16) EFT_TRY(dmal(ctx, &F0.A.val16, nv));
    if (!ctx->par.mg_bf16 && !F0.A.val32) EFT_TRY(dmal(ctx, &F0.A.val32, nv));
    return EFT_OK;
}

// Refresh the hierarchy for the current Jacobian: inject node fields,
// rediscretize the coarse Jacobians, block inverses and the coarsest inverse.
// BF16 copy of the finest level's FP32 block inverses, read by the sweeps of
// the FP32-vector cycle
static eft_status dinv_bf16(eft_ctx *ctx, MGLevel &F0)
{
    if (!F0.Dinv16) return EFT_OK;
    const int64_t n = F0.A.n * ctx->bs * ctx->bs;
    hipLaunchKernelGGL(k_to_bf16<float>, dim3((int)std::min<int64_t>(8192, (n + 255) / 256)), dim3(256), 0,
                       ctx->stream, F0.Dinv32, F0.Dinv16, n);
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}

eft_status eft_mg_setup(eft_ctx *ctx, const double *vp, bool coarse)
{
    const int bs = ctx->bs;
    const int64_t L = (int64_t)ctx->mg.size();
    MGLevel &F0 = ctx->mg[0];
    const int64_t nv = ctx->J.nnzb * bs * bs;
    const int cgrid = (int)std::min<int64_t>(8192, (nv + 255) / 256);
    if (ctx->par.mg_bf16) {
        // BF16 copy of the Jacobian; block inverses of its exact diagonal
        if (!F0.A.val16) {
            ctx->err = "multigrid BF16 copy not reserved";
            return EFT_EINVAL;
        }
        F0.A.bf16 = true;
        F0.A.fp32 = false;
        if (ctx->J.fp32)
            hipLaunchKernelGGL(k_to_bf16<float>, dim3(cgrid), dim3(256), 0, ctx->stream, ctx->J.val32, F0.A.val16, nv);
        else if (!ctx->mg_f32_fresh)   // (else the assembly wrote the copy)
            hipLaunchKernelGGL(k_to_bf16<double>, dim3(cgrid), dim3(256), 0, ctx->stream, ctx->J.val, F0.A.val16, nv);
        ctx->mg_f32_fresh = false;
        EFT_HIP(hipGetLastError());
        EFT_TRY(eft_bj_setup32(ctx, &ctx->J, F0.Dinv32));
        EFT_TRY(dinv_bf16(ctx, F0));
    } else {
        if (!F0.A.val32) {
            ctx->err = "multigrid FP32 copy not reserved";
            return EFT_EINVAL;
        }
        F0.A.bf16 = false;
        F0.A.fp32 = true;
        if (ctx->J.fp32) {
            EFT_HIP(hipMemcpyAsync(F0.A.val32, ctx->J.val32, sizeof(float) * nv, hipMemcpyDeviceToDevice,
                                   ctx->stream));
        } else if (!ctx->mg_f32_fresh) {   // (else the assembly wrote the copy)
            hipLaunchKernelGGL(k_to_f32, dim3(cgrid), dim3(256), 0, ctx->stream, ctx->J.val, F0.A.val32, nv);
            EFT_HIP(hipGetLastError());
        }
        ctx->mg_f32_fresh = false;
        EFT_TRY(eft_bj_setup32(ctx, &F0.A, F0.Dinv32));
        EFT_TRY(dinv_bf16(ctx, F0));
    }
    if (!coarse) {   // the coarse levels of the previous refresh are kept
        ctx->mg_valid = true;
        return EFT_OK;
    }
    for (int64_t l = 1; l < L && ctx->par.mg_galerkin; ++l) {
        // Galerkin coarse operator from the level above
        MGLevel &C = ctx->mg[l];
        const MGLevel &F = ctx->mg[l - 1];
        C.A.bf16 = C.A.fp32 && ctx->par.mg_bf16 != 0;
        RapArgs ra;
        ra.cd = dims_of(C);
        ra.fd = dims_of(F);
        ra.nc = C.N;
        ra.frow = F.A.rowptr;
        ra.fcol = F.A.col;
        ra.crow = C.A.rowptr;
        ra.ccol = C.A.col;
        ra.fmask = F.fmask;
        ra.cmask = C.fmask;
        ra.miss = ctx->mg_miss;
        const dim3 g(eft_grid(C.N, 4)), t(256);
        uint16_t *c16 = C.A.bf16 ? C.A.val16 : nullptr;
        auto launch = [&](auto fv) {
            using TF = std::remove_cv_t<std::remove_pointer_t<decltype(fv)>>;
            if (ctx->dim == 2) {
                if (C.A.fp32) hipLaunchKernelGGL((k_rap_rows<2, TF, float>), g, t, 0, ctx->stream, ra, fv, C.A.val32, c16);
                else hipLaunchKernelGGL((k_rap_rows<2, TF, double>), g, t, 0, ctx->stream, ra, fv, C.A.val, c16);
            } else {
                if (C.A.fp32) hipLaunchKernelGGL((k_rap_rows<3, TF, float>), g, t, 0, ctx->stream, ra, fv, C.A.val32, c16);
                else hipLaunchKernelGGL((k_rap_rows<3, TF, double>), g, t, 0, ctx->stream, ra, fv, C.A.val, c16);
            }
        };
        if (l == 1) {
            if (ctx->J.fp32) launch((const float *)ctx->J.val32);
            else launch((const double *)ctx->J.val);
        } else {
            if (F.A.fp32) launch((const float *)F.A.val32);
            else launch((const double *)F.A.val);
        }
        EFT_HIP(hipGetLastError());
        if (C.A.fp32) EFT_TRY(eft_bj_setup32(ctx, &C.A, C.Dinv32));
        else EFT_TRY(eft_bj_setup(ctx, &C.A, C.Dinv));
    }
    for (int64_t l = 1; l < L && !ctx->par.mg_galerkin; ++l) {
        MGLevel &C = ctx->mg[l];
        InjArgs a;
        a.Nc = C.N;
        a.Nf = ctx->N;
        a.d = ctx->dim;
        a.bs = bs;
        a.nv = ctx->nv;
        a.n_s = ctx->n_s;
        a.inj = C.inj;
        a.va = ctx->va;
        a.acc = ctx->acc;
        a.rho = ctx->rho;
        a.mu = ctx->mu;
        a.alpha = ga_of(ctx->par.rho_inf, ctx->par.dt).alpha;
        a.smask = ctx->smask;
        a.lphi = ctx->src_lphi;
        a.iphi = ctx->src_iphi;
        a.lB = ctx->src_lB;
        a.iB = ctx->src_iB;
        a.solid_ind = ctx->solid_ind_d;
        a.vp = vp;
        a.cva = C.va;
        a.cacc = C.acc;
        a.crho = C.rho;
        a.cmu = C.mu;
        a.cas = C.as;
        a.cBa = C.Ba;
        a.cvp = C.vp;
        a.csmask = C.smask;
        hipLaunchKernelGGL(k_inject, dim3(eft_grid(C.N, 256)), dim3(256), 0, ctx->stream, a);
        EFT_HIP(hipGetLastError());
        MeshView M;
        M.N = C.N;
        M.E = C.E;
        M.conn = C.conn;
        M.epos = C.epos;
        M.xyz = C.xyz;
        M.va = C.va;
        M.acc = C.acc;
        M.rho = C.rho;
        M.mu = C.mu;
        M.as = C.as;
        M.Ba = C.Ba;
        M.smask = C.smask;
        M.n_dir = C.n_dir;
        M.dir_node = C.dir_node;
        M.dir_mask = C.dir_mask;
        M.fmask = C.fmask;
        M.iptr = C.iptr;
        M.ient = C.ient;
        M.islot = C.islot;
        M.maxc = C.maxc;
        M.rpb = C.rpb;
        // intermediate levels: FP32 values (block inverses) and, with
        // mg_bf16, a BF16 copy for the sweeps and residuals
        C.A.bf16 = C.A.fp32 && ctx->par.mg_bf16 != 0;
        EFT_TRY(eft_ns_level(ctx, M, C.vp, C.R, &C.A, nullptr, C.A.bf16 ? C.A.val16 : nullptr));
        if (C.A.fp32) EFT_TRY(eft_bj_setup32(ctx, &C.A, C.Dinv32));
        else EFT_TRY(eft_bj_setup(ctx, &C.A, C.Dinv));
    }
    if (ctx->mg_inv) {
        const MGLevel &Cc = ctx->mg.back();
        EFT_TRY(eft_fill(ctx, ctx->mg_dense, ctx->mg_nd * ctx->mg_nd, 0.0));
        hipLaunchKernelGGL(k_dense_fill<double>, dim3(eft_grid(Cc.A.nnzb * bs, 64)), dim3(64), 0, ctx->stream,
                           Cc.A.nnzb, bs, Cc.A.rowptr, Cc.A.col, Cc.A.val, ctx->mg_fidx, ctx->mg_dense, ctx->mg_nd,
                           Cc.N);
        const int nd = (int)ctx->mg_nd;
        if (nd <= GJ_LDS_MAX)   // (one wavefront when the 2 nd columns fit in it)
            hipLaunchKernelGGL(k_gauss_jordan_lds, dim3(1), dim3(2 * nd <= 64 ? 64 : 256), gj_lds_bytes(nd),
                               ctx->stream, ctx->mg_dense, ctx->mg_inv, nd);
        else
            hipLaunchKernelGGL(k_gauss_jordan, dim3(1), dim3(256), 0, ctx->stream, ctx->mg_dense, ctx->mg_inv, nd);
        EFT_HIP(hipGetLastError());
    }
    ctx->mg_valid = true;
    return EFT_OK;
}

namespace {

template <typename TV, typename TD, typename TX = double, typename TO = double>
void launch_sweep(eft_ctx *ctx, const eft_matrix &A, const TV *val, const TD *Dinv, double omega, const double *b,
                  const TX *x, TO *xo, const int32_t *flag)
{
    const dim3 t(256);
    if constexpr (sizeof(TV) < 8) {   // narrow values: one block per lane
#define EFT_SWEEP_BLK(B_, S_)                                                                                       \
    hipLaunchKernelGGL((k_sweep_blk<B_, TV, TD, S_, TX, TO>), dim3(eft_grid(A.n, 4 * BlockSeg<B_>::RPW)), t, 0,     \
                       ctx->stream, A.n, A.rowptr, A.col, A.stn_mask, A.stn_off, val, Dinv, omega, b, x, xo, flag)
        const bool stn = A.stn_mask != nullptr;
        if (A.bs == 3) {
            if (stn) EFT_SWEEP_BLK(3, true);
            else EFT_SWEEP_BLK(3, false);
        } else {
            if (stn) EFT_SWEEP_BLK(4, true);
            else EFT_SWEEP_BLK(4, false);
        }
#undef EFT_SWEEP_BLK
        return;
    } else {
        static_assert(sizeof(TX) == 8 && sizeof(TO) == 8, "FP64 values: FP64 vectors");
        const dim3 g(eft_grid(A.n, 4 * SWEEP_R));
        if (A.bs == 3)
            hipLaunchKernelGGL((k_sweep_rows<3, TV, TD>), g, t, 0, ctx->stream, A.n, A.rowptr, A.col, val, Dinv, omega,
                               b, x, xo, flag);
        else
            hipLaunchKernelGGL((k_sweep_rows<4, TV, TD>), g, t, 0, ctx->stream, A.n, A.rowptr, A.col, val, Dinv, omega,
                               b, x, xo, flag);
    }
}

template <typename TV, typename TX = double, typename TR = double>
void launch_resid(eft_ctx *ctx, const eft_matrix &A, const TV *val, const double *b, const TX *x, TR *r,
                  const int32_t *flag)
{
    const dim3 t(256);
    if constexpr (sizeof(TV) < 8) {   // narrow values: one block per lane
#define EFT_RESID_BLK(B_, S_)                                                                                      \
    hipLaunchKernelGGL((k_resid_blk<B_, TV, S_, TX, TR>), dim3(eft_grid(A.n, 4 * BlockSeg<B_>::RPW)), t, 0,        \
                       ctx->stream, A.n, A.rowptr, A.col, A.stn_mask, A.stn_off, val, b, x, r, flag)
        const bool stn = A.stn_mask != nullptr;
        if (A.bs == 3) {
            if (stn) EFT_RESID_BLK(3, true);
            else EFT_RESID_BLK(3, false);
        } else {
            if (stn) EFT_RESID_BLK(4, true);
            else EFT_RESID_BLK(4, false);
        }
#undef EFT_RESID_BLK
        return;
    } else {
        static_assert(sizeof(TX) == 8 && sizeof(TR) == 8, "FP64 values: FP64 vectors");
        const dim3 g(eft_grid(A.n, 4 * RESID_R));
        if (A.bs == 3)
            hipLaunchKernelGGL((k_resid_rows<3, TV>), g, t, 0, ctx->stream, A.n, A.rowptr, A.col, val, b, x, r, flag);
        else
            hipLaunchKernelGGL((k_resid_rows<4, TV>), g, t, 0, ctx->stream, A.n, A.rowptr, A.col, val, b, x, r, flag);
    }
}

// (the momentum/mass system has bs = d + 1, 3 or 4)
void sweep(eft_ctx *ctx, const MGLevel &L, const double *b, const double *x, double *xo, const int32_t *flag)
{
    const double om = ctx->par.mg_omega;
    if (L.A.bf16)
        launch_sweep<eft_bf16, float>(ctx, L.A, reinterpret_cast<const eft_bf16 *>(L.A.val16), L.Dinv32, om, b, x, xo,
                                      flag);
    else if (L.A.fp32)
        launch_sweep<float, float>(ctx, L.A, L.A.val32, L.Dinv32, om, b, x, xo, flag);
    else
        launch_sweep<double, double>(ctx, L.A, L.A.val, L.Dinv, om, b, x, xo, flag);
}

// first sweep from x = 0
void sweep0(eft_ctx *ctx, const MGLevel &L, const double *b, double *x, const int32_t *flag)
{
    const int64_t nd = L.N * ctx->bs;
    const dim3 gn(eft_grid(L.N, 256));
    if ((L.A.fp32 || L.A.bf16) && ctx->bs == 4)
        hipLaunchKernelGGL((k_sweep0_nodes<4, float, double>), gn, dim3(256), 0, ctx->stream, L.N, L.Dinv32,
                           ctx->par.mg_omega, b, x, flag);
    else if ((L.A.fp32 || L.A.bf16) && ctx->bs == 3)
        hipLaunchKernelGGL((k_sweep0_nodes<3, float, double>), gn, dim3(256), 0, ctx->stream, L.N, L.Dinv32,
                           ctx->par.mg_omega, b, x, flag);
    else if (L.A.fp32 || L.A.bf16)
        hipLaunchKernelGGL(k_sweep0<float>, dim3(eft_grid(nd, 256)), dim3(256), 0, ctx->stream, nd, ctx->bs, L.Dinv32,
                           ctx->par.mg_omega, b, x, flag);
    else
        hipLaunchKernelGGL(k_sweep0<double>, dim3(eft_grid(nd, 256)), dim3(256), 0, ctx->stream, nd, ctx->bs, L.Dinv,
                           ctx->par.mg_omega, b, x, flag);
}

// Algorithmic bytes of one sweep: values, column indices (or, in stencil
// form, the row masks) and row pointers once, the block inverses, b and x
// read and x_out written once.
double sweep_bytes(const eft_matrix &A, double xb = 8.0, double xob = 8.0, double dbo = 0.0)
{
    const double vb = A.bf16 ? 2.0 : A.fp32 ? 4.0 : 8.0, db = dbo > 0.0 ? dbo : (A.bf16 || A.fp32) ? 4.0 : 8.0;
    const double b2 = (double)A.bs * A.bs;
    const double cols = A.stn_mask ? (double)A.n * 2.0 : (double)A.nnzb * 4.0;
    return (double)A.nnzb * b2 * vb + cols + (double)(A.n + 1) * 4.0 +
           (double)A.n * (b2 * db + A.bs * (8.0 + xb + xob));
}

// fine-level sweeps carry the kernel-timing hook
void timed_sweep(eft_ctx *ctx, int l, const MGLevel &L, const double *b, const double *x, double *xo,
                 const int32_t *flag)
{
    const int64_t slot = l == 0 ? eft_kt_begin(ctx, EFT_KT_SMOOTH) : -1;
    sweep(ctx, L, b, x, xo, flag);
    eft_kt_end(ctx, slot, sweep_bytes(L.A), EFT_KT_SMOOTH);
}

template <typename TV, typename TD>
void launch_gs(eft_ctx *ctx, const MGLevel &L, int c, const TV *val, const TD *Dinv, const double *b, double *x,
               const int32_t *flag)
{
    const int64_t nc = L.coff[c + 1] - L.coff[c];
    if (nc == 0) return;
    const dim3 g(eft_grid(nc, 4 * SWEEP_R)), t(256);
    const double om = ctx->par.mg_omega;
    if (L.A.bs == 3)
        hipLaunchKernelGGL((k_gs_rows<3, TV, TD>), g, t, 0, ctx->stream, nc, L.crow + L.coff[c], L.A.rowptr, L.A.col,
                           val, Dinv, om, b, x, flag);
    else
        hipLaunchKernelGGL((k_gs_rows<4, TV, TD>), g, t, 0, ctx->stream, nc, L.crow + L.coff[c], L.A.rowptr, L.A.col,
                           val, Dinv, om, b, x, flag);
}

// One Gauss-Seidel sweep over all colours (reverse order when backward), in
// place on x; on the finest level every colour launch carries the timing hook
// with its own algorithmic bytes
void gs_sweep(eft_ctx *ctx, int l, const MGLevel &L, const double *b, double *x, const int32_t *flag, bool backward)
{
    const int bs = L.A.bs;
    for (int cc = 0; cc < L.ncolor; ++cc) {
        const int c = backward ? L.ncolor - 1 - cc : cc;
        const int64_t nc = L.coff[c + 1] - L.coff[c];
        const double vb = L.A.bf16 ? 2.0 : L.A.fp32 ? 4.0 : 8.0, db = (L.A.bf16 || L.A.fp32) ? 4.0 : 8.0;
        const double bytes = (double)L.cnnz[c] * (bs * bs * vb + 4.0) + (double)nc * (4.0 + 8.0 + bs * bs * db) +
                             (double)nc * 3.0 * bs * 8.0;
        const int64_t slot = l == 0 ? eft_kt_begin(ctx, EFT_KT_SMOOTH) : -1;
        if (L.A.bf16)
            launch_gs<eft_bf16, float>(ctx, L, c, reinterpret_cast<const eft_bf16 *>(L.A.val16), L.Dinv32, b, x, flag);
        else if (L.A.fp32)
            launch_gs<float, float>(ctx, L, c, L.A.val32, L.Dinv32, b, x, flag);
        else
            launch_gs<double, double>(ctx, L, c, L.A.val, L.Dinv, b, x, flag);
        eft_kt_end(ctx, slot, bytes, EFT_KT_SMOOTH);
    }
}

// The finest level with FP32 iterate and residual vectors (b and the
// output FP64, arithmetic FP64): narrow matrix values, Jacobi smoothing.
template <typename TX, typename TO>
void sweep_f(eft_ctx *ctx, const MGLevel &L, const double *b, const TX *x, TO *xo, const int32_t *flag)
{
    const double om = ctx->par.mg_omega;
    const int64_t slot = eft_kt_begin(ctx, EFT_KT_SMOOTH);
    const eft_bf16 *D16 = reinterpret_cast<const eft_bf16 *>(L.Dinv16);
    if (L.A.bf16)
        launch_sweep<eft_bf16, eft_bf16, TX, TO>(ctx, L.A, reinterpret_cast<const eft_bf16 *>(L.A.val16), D16, om, b,
                                                 x, xo, flag);
    else
        launch_sweep<float, eft_bf16, TX, TO>(ctx, L.A, L.A.val32, D16, om, b, x, xo, flag);
    eft_kt_end(ctx, slot, sweep_bytes(L.A, sizeof(TX), sizeof(TO), 2.0), EFT_KT_SMOOTH);
}

void resid(eft_ctx *ctx, const eft_matrix &A, const double *b, const double *x, double *r, const int32_t *flag)
{
    if (A.bf16) launch_resid<eft_bf16>(ctx, A, reinterpret_cast<const eft_bf16 *>(A.val16), b, x, r, flag);
    else if (A.fp32) launch_resid<float>(ctx, A, A.val32, b, x, r, flag);
    else launch_resid<double>(ctx, A, A.val, b, x, r, flag);
}

// V-cycle on level l with right-hand side b; returns the buffer holding x
// (out, when given, receives the last post-smoothing sweep)
// (x0_done: the first sweep from zero was fused into the restriction that
// produced b and already sits in the level's x)
double *vcycle(eft_ctx *ctx, int l, const double *b, const int32_t *flag, double *out = nullptr,
               bool x0_done = false)
{
    MGLevel &L = ctx->mg[l];
    const eft_matrix &A = L.A;
    const int bs = ctx->bs;
    const int64_t nd = L.N * bs;
    double *cur = L.x, *oth = L.x2;
    const bool last = l + 1 == (int)ctx->mg.size();
    if (last && ctx->mg_inv) {
        hipLaunchKernelGGL(k_dense_apply, dim3(1), dim3(256), 0, ctx->stream, ctx->mg_inv, (int)ctx->mg_nd,
                           ctx->mg_free, nd, b, cur, flag);
        return cur;
    }
    const bool gs = ctx->par.mg_smoother == 1 && L.ncolor > 0;
    if (gs && out) cur = out;   // in-place smoothing works on the output directly
    if (!x0_done) sweep0(ctx, L, b, cur, flag);
    // (levels below the finest may smooth more: the coarse correction sets
    // the convergence of the cycle)
    const int nu = last ? 40 : l == 0 || ctx->par.mg_cnu == 0 ? ctx->par.mg_nu : ctx->par.mg_cnu;
    for (int s = 1; s < nu; ++s) {
        if (gs) {
            gs_sweep(ctx, l, L, b, cur, flag, false);
        } else {
            timed_sweep(ctx, l, L, b, cur, oth, flag);
            std::swap(cur, oth);
        }
    }
    if (last) return cur;
    MGLevel &C = ctx->mg[l + 1];
    resid(ctx, A, b, cur, L.r, flag);
    const Dims fd = dims_of(L), cd = dims_of(C);
    // the coarse level starts with a sweep from zero into its x unless it
    // is the coarsest with a dense solve: fuse that sweep into the restriction
    const bool c_last = l + 2 == (int)ctx->mg.size();
    const bool fuse = !(c_last && ctx->mg_inv);
    const dim3 gr(eft_grid(C.N, 256)), tr(256);
    const bool c32 = C.A.fp32 || C.A.bf16;
    const double om = ctx->par.mg_omega;
    if (!fuse) {
        if (ctx->dim == 2)
            hipLaunchKernelGGL((k_restrict<2, double>), gr, tr, 0, ctx->stream, cd, fd, C.fmask, L.fmask, L.r, C.b, flag);
        else
            hipLaunchKernelGGL((k_restrict<3, double>), gr, tr, 0, ctx->stream, cd, fd, C.fmask, L.fmask, L.r, C.b, flag);
    } else if (ctx->dim == 2) {
        if (c32)
            hipLaunchKernelGGL((k_restrict_sweep0<2, float, double>), gr, tr, 0, ctx->stream, cd, fd, C.fmask, L.fmask, L.r,
                               C.b, C.Dinv32, om, C.x, flag);
        else
            hipLaunchKernelGGL((k_restrict_sweep0<2, double, double>), gr, tr, 0, ctx->stream, cd, fd, C.fmask, L.fmask, L.r,
                               C.b, C.Dinv, om, C.x, flag);
    } else {
        if (c32)
            hipLaunchKernelGGL((k_restrict_sweep0<3, float, double>), gr, tr, 0, ctx->stream, cd, fd, C.fmask, L.fmask, L.r,
                               C.b, C.Dinv32, om, C.x, flag);
        else
            hipLaunchKernelGGL((k_restrict_sweep0<3, double, double>), gr, tr, 0, ctx->stream, cd, fd, C.fmask, L.fmask, L.r,
                               C.b, C.Dinv, om, C.x, flag);
    }
    double *xc = vcycle(ctx, l + 1, C.b, flag, nullptr, fuse);
    if (ctx->dim == 2)
        hipLaunchKernelGGL((k_prolong<2, double>), dim3(eft_grid(L.N, 256)), dim3(256), 0, ctx->stream, cd, fd, C.fmask, L.fmask,
                           xc, cur, flag);
    else
        hipLaunchKernelGGL((k_prolong<3, double>), dim3(eft_grid(L.N, 256)), dim3(256), 0, ctx->stream, cd, fd, C.fmask, L.fmask,
                           xc, cur, flag);
    const int npost = l == 0 || ctx->par.mg_cnu_post == 0 ? ctx->par.mg_nu_post : ctx->par.mg_cnu_post;
    if (gs) {
        for (int s = 0; s < npost; ++s) gs_sweep(ctx, l, L, b, cur, flag, true);
        return cur;
    }
    for (int s = 0; s < npost; ++s) {
        double *dst = (out && s + 1 == npost) ? out : oth;
        timed_sweep(ctx, l, L, b, cur, dst, flag);
        oth = cur;
        cur = dst;
    }
    return cur;
}

}  // namespace

// z = M^-1 b0 with one V-cycle
// The finest level's part of the cycle with FP32 iterate and residual
// vectors and BF16 block inverses (the same steps as vcycle at level 0 with
// Jacobi smoothing; the last post-sweep writes the FP64 output z).  Halves
// the vector and inverse bytes of the level's sweeps and their x gathers.
static bool vcycle0_f32_ok(const eft_ctx *ctx)
{
    if (ctx->mg.size() < 2) return false;
    const MGLevel &L = ctx->mg[0];
    return L.xf && L.Dinv16 && (L.A.bf16 || L.A.fp32) && (ctx->bs == 3 || ctx->bs == 4) &&
           ctx->par.mg_smoother == 0;
}

static void vcycle0_f32(eft_ctx *ctx, const double *b, double *z, const int32_t *flag)
{
    MGLevel &L = ctx->mg[0];
    MGLevel &C = ctx->mg[1];
    const double om = ctx->par.mg_omega;
    float *cur = L.xf, *oth = L.xf2;
    const dim3 gn(eft_grid(L.N, 256)), t(256);
    const eft_bf16 *D16 = reinterpret_cast<const eft_bf16 *>(L.Dinv16);
    if (ctx->bs == 4)
        hipLaunchKernelGGL((k_sweep0_nodes<4, eft_bf16, float>), gn, t, 0, ctx->stream, L.N, D16, om, b, cur, flag);
    else
        hipLaunchKernelGGL((k_sweep0_nodes<3, eft_bf16, float>), gn, t, 0, ctx->stream, L.N, D16, om, b, cur, flag);
    for (int s = 1; s < ctx->par.mg_nu; ++s) {
        sweep_f<float, float>(ctx, L, b, cur, oth, flag);
        std::swap(cur, oth);
    }
    if (L.A.bf16)
        launch_resid<eft_bf16, float, float>(ctx, L.A, reinterpret_cast<const eft_bf16 *>(L.A.val16), b, cur, L.rf,
                                             flag);
    else
        launch_resid<float, float, float>(ctx, L.A, L.A.val32, b, cur, L.rf, flag);
    const Dims fd = dims_of(L), cd = dims_of(C);
    const bool c_last = ctx->mg.size() == 2;
    const bool fuse = !(c_last && ctx->mg_inv);
    const dim3 gr(eft_grid(C.N, 256));
    const bool c32 = C.A.fp32 || C.A.bf16;
    if (!fuse) {
        if (ctx->dim == 2)
            hipLaunchKernelGGL((k_restrict<2, float>), gr, t, 0, ctx->stream, cd, fd, C.fmask, L.fmask, L.rf, C.b, flag);
        else
            hipLaunchKernelGGL((k_restrict<3, float>), gr, t, 0, ctx->stream, cd, fd, C.fmask, L.fmask, L.rf, C.b, flag);
    } else if (ctx->dim == 2) {
        if (c32)
            hipLaunchKernelGGL((k_restrict_sweep0<2, float, float>), gr, t, 0, ctx->stream, cd, fd, C.fmask, L.fmask,
                               L.rf, C.b, C.Dinv32, om, C.x, flag);
        else
            hipLaunchKernelGGL((k_restrict_sweep0<2, double, float>), gr, t, 0, ctx->stream, cd, fd, C.fmask, L.fmask,
                               L.rf, C.b, C.Dinv, om, C.x, flag);
    } else {
        if (c32)
            hipLaunchKernelGGL((k_restrict_sweep0<3, float, float>), gr, t, 0, ctx->stream, cd, fd, C.fmask, L.fmask,
                               L.rf, C.b, C.Dinv32, om, C.x, flag);
        else
            hipLaunchKernelGGL((k_restrict_sweep0<3, double, float>), gr, t, 0, ctx->stream, cd, fd, C.fmask, L.fmask,
                               L.rf, C.b, C.Dinv, om, C.x, flag);
    }
    const double *xc = vcycle(ctx, 1, C.b, flag, nullptr, fuse);
    if (ctx->dim == 2)
        hipLaunchKernelGGL((k_prolong<2, float>), gn, t, 0, ctx->stream, cd, fd, C.fmask, L.fmask, xc, cur, flag);
    else
        hipLaunchKernelGGL((k_prolong<3, float>), gn, t, 0, ctx->stream, cd, fd, C.fmask, L.fmask, xc, cur, flag);
    const int npost = ctx->par.mg_nu_post;   // >= 1
    for (int s = 0; s + 1 < npost; ++s) {
        sweep_f<float, float>(ctx, L, b, cur, oth, flag);
        std::swap(cur, oth);
    }
    sweep_f<float, double>(ctx, L, b, cur, z, flag);
}

eft_status eft_mg_vcycle(eft_ctx *ctx, const double *b0, double *z, const int32_t *flag)
{
    MGLevel &L0 = ctx->mg[0];
    if (vcycle0_f32_ok(ctx)) {
        vcycle0_f32(ctx, b0, z, flag);
        EFT_HIP(hipGetLastError());
        return EFT_OK;
    }
    double *x = vcycle(ctx, 0, b0, flag, z);
    EFT_HIP(hipGetLastError());
    if (x != z)
        EFT_HIP(hipMemcpyAsync(z, x, sizeof(double) * L0.N * ctx->bs, hipMemcpyDeviceToDevice, ctx->stream));
    return EFT_OK;
}

namespace {
__global__ void k_widen32(const float *a, double *b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (double)a[i];
}
}  // namespace

extern "C" eft_status eft_mg_export(eft_ctx *ctx, int32_t level, int32_t *levels, int64_t *n, int64_t *nnzb,
                                    int32_t *rowptr, int32_t *col, double *val)
{
    if (!ctx) return EFT_EINVAL;
    if (levels) *levels = (int32_t)ctx->mg.size();
    if (ctx->mg.size() < 2 || level < 0 || level >= (int)ctx->mg.size()) {
        ctx->err = "no multigrid level " + std::to_string(level);
        return EFT_EINVAL;
    }
    const MGLevel &L = ctx->mg[level];
    const eft_matrix &A = level == 0 ? ctx->J : L.A;
    if (n) *n = A.n;
    if (nnzb) *nnzb = A.nnzb;
    if (rowptr) EFT_HIP(hipMemcpyAsync(rowptr, A.rowptr, sizeof(int32_t) * (A.n + 1), hipMemcpyDeviceToDevice, ctx->stream));
    if (col) EFT_HIP(hipMemcpyAsync(col, A.col, sizeof(int32_t) * A.nnzb, hipMemcpyDeviceToDevice, ctx->stream));
    const int64_t nv = A.nnzb * A.bs * A.bs;
    if (val) {
        if (A.fp32) {
            hipLaunchKernelGGL(k_widen32, dim3((int)std::min<int64_t>(8192, (nv + 255) / 256)), dim3(256), 0,
                               ctx->stream, A.val32, val, nv);
            EFT_HIP(hipGetLastError());
        } else {
            EFT_HIP(hipMemcpyAsync(val, A.val, sizeof(double) * nv, hipMemcpyDeviceToDevice, ctx->stream));
        }
    }
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    return EFT_OK;
}
