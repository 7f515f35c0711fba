// Order-parameter and left-Cauchy-Green transport restricted to the grid-cell
// band of every indicator:
//   band build   grid cells (Sec. 3.1 grid-cell method) seeded where
//                |phi^n| < 1 - band_flat, dilated by band_halo cell layers;
//                band nodes/elements compacted, band pattern carved out of the
//                global node graph;
//   mobility     eq. (tdm-num): element quotient (grad phi)^T grad v
//                (grad phi) / |grad phi|^2, L2 projection to nodes (Appendix A),
//                RMS over |phi| <= di_cut, divided by eta;
//   beta         int F'(phi) / int sqrt(F(phi)) over the band (Sec. 2.2.1);
//   Allen-Cahn   eq. (PPV_AC) residual and tangent, SUPG with tau_phi;
//   B            eq. (semiCGT) residual and tangent, SUPG with tau_B;
// each band system is solved with the same FGMRES as the momentum block.
#include <algorithm>

#include "dev_common.h"
#include "eft_internal.h"

namespace {

constexpr int SB = 1024;     // scan block
constexpr int ST = 4;        // items per thread
constexpr int TILE = SB * ST;

__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t *lds, int32_t *total)
{
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < SB; off <<= 1) {
        int32_t a = t >= off ? lds[t - off] : 0;
        __syncthreads();
        lds[t] += a;
        __syncthreads();
    }
    int32_t incl = lds[t];
    *total = lds[SB - 1];
    __syncthreads();
    return incl - v;
}

template <typename TI>
__global__ __launch_bounds__(SB) void k_scan_count(const TI *in, int64_t n, int32_t *bsum)
{
    __shared__ int32_t lds[SB];
    const int64_t base = (int64_t)blockIdx.x * TILE + threadIdx.x * ST;
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < ST; ++k)
        if (base + k < n) s += (int32_t)in[base + k];
    int32_t tot;
    block_excl_scan(s, lds, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SB) void k_scan_blocks(int32_t *bsum, int nb, int32_t *total)
{
    __shared__ int32_t lds[SB];
    int32_t carry = 0;
    for (int c = 0; c < nb; c += SB) {
        const int i = c + threadIdx.x;
        const int32_t v = i < nb ? bsum[i] : 0;
        int32_t tot;
        const int32_t ex = block_excl_scan(v, lds, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

// Exclusive offsets out[i] (optional), compacted indices idx[] of nonzero
// entries (optional, for flags), map[i] = position or -1 (optional).
template <typename TI>
__global__ __launch_bounds__(SB) void k_scan_write(const TI *in, int64_t n, const int32_t *bsum,
                                                   int32_t *out, int32_t *idx, int32_t *map)
{
    __shared__ int32_t lds[SB];
    const int64_t base = (int64_t)blockIdx.x * TILE + threadIdx.x * ST;
    int32_t v[ST], s = 0;
#pragma unroll
    for (int k = 0; k < ST; ++k) {
        v[k] = base + k < n ? (int32_t)in[base + k] : 0;
        s += v[k];
    }
    int32_t tot;
    int32_t pos = block_excl_scan(s, lds, &tot) + bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < ST; ++k) {
        const int64_t i = base + k;
        if (i < n) {
            if (out) out[i] = pos;
            if (idx && v[k]) idx[pos] = (int32_t)i;
            if (map) map[i] = v[k] ? pos : -1;
        }
        pos += v[k];
    }
}

// ---------------------------------------------------------------- band ----

template <int D>
__global__ __launch_bounds__(256) void k_seed(int64_t E, const int32_t *conn, const int32_t *cell_of,
                                              const double *phi, double thr, uint8_t *seed)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    bool iface = false;
#pragma unroll
    for (int a = 0; a < D + 1; ++a) iface |= fabs(phi[conn[e * (D + 1) + a]]) < thr;
    if (iface) seed[cell_of[e]] = 1;
}

__global__ __launch_bounds__(256) void k_dilate(int nx, int ny, int nz, int H, const uint8_t *seed, uint8_t *active)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ncell = (int64_t)nx * ny * nz;
    if (c >= ncell) return;
    const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((int64_t)nx * ny));
    uint8_t act = 0;
    for (int dk = -H; dk <= H && !act; ++dk)
        for (int dj = -H; dj <= H && !act; ++dj)
            for (int di = -H; di <= H; ++di) {
                const int ii = i + di, jj = j + dj, kk = k + dk;
                if (ii < 0 || jj < 0 || kk < 0 || ii >= nx || jj >= ny || kk >= nz) continue;
                if (seed[ii + (int64_t)nx * (jj + (int64_t)ny * kk)]) {
                    act = 1;
                    break;
                }
            }
    active[c] = act;
}

template <int D>
__global__ __launch_bounds__(256) void k_mark(int64_t E, const int32_t *conn, const int32_t *cell_of,
                                              const uint8_t *active, uint8_t *ein, uint8_t *nin, uint8_t *nout)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const uint8_t inb = active[cell_of[e]];
    ein[e] = inb;
#pragma unroll
    for (int a = 0; a < D + 1; ++a) {
        const int p = conn[e * (D + 1) + a];
        if (inb) nin[p] = 1;
        else nout[p] = 1;
    }
}

__global__ __launch_bounds__(256) void k_band_free(int64_t n, const int32_t *node, const uint8_t *nout, uint8_t *fre)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    fre[r] = nout[node[r]] ? 0 : 1;
}

__global__ __launch_bounds__(256) void k_band_rowcount(int64_t n, const int32_t *node, const int32_t *grow,
                                                       const int32_t *gcol, const int32_t *g2b, int32_t *cnt)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int g = node[r];
    int c = 0;
    for (int k = grow[g]; k < grow[g + 1]; ++k) c += g2b[gcol[k]] >= 0 ? 1 : 0;
    cnt[r] = c;
}

__global__ __launch_bounds__(256) void k_band_fill(int64_t n, const int32_t *node, const int32_t *grow,
                                                   const int32_t *gcol, const int32_t *g2b, const int32_t *rowptr,
                                                   int32_t *col, int32_t *diag, int32_t *gpos2b)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int g = node[r];
    int pos = rowptr[r];
    for (int k = grow[g]; k < grow[g + 1]; ++k) {
        const int b = g2b[gcol[k]];
        if (b < 0) continue;
        col[pos] = b;
        if (b == r) diag[r] = pos;
        gpos2b[k] = pos;
        ++pos;
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_band_epos(int64_t ne, const int32_t *__restrict__ elem,
                                                   const int32_t *__restrict__ conn, const int32_t *__restrict__ epos,
                                                   const int32_t *__restrict__ gpos2b, const int32_t *__restrict__ g2b,
                                                   int32_t *__restrict__ bepos, int32_t *__restrict__ bconn)
{
    const int64_t be = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (be >= ne) return;
    constexpr int NN = D + 1;
    const int64_t e = elem[be];
    // all indices, then all gathers, then the stores: three round trips
    int32_t c[NN], ep[NN * NN];
#pragma unroll
    for (int a = 0; a < NN; ++a) c[a] = conn[e * NN + a];
#pragma unroll
    for (int t = 0; t < NN * NN; ++t) ep[t] = epos[e * NN * NN + t];
#pragma unroll
    for (int a = 0; a < NN; ++a) c[a] = g2b[c[a]];
#pragma unroll
    for (int t = 0; t < NN * NN; ++t) ep[t] = gpos2b[ep[t]];
#pragma unroll
    for (int a = 0; a < NN; ++a) bconn[be * NN + a] = c[a];
#pragma unroll
    for (int t = 0; t < NN * NN; ++t) bepos[be * NN * NN + t] = ep[t];
}

// ------------------------------------------------------------ mobility ----

template <int D>
__global__ __launch_bounds__(256) void k_mob_elem(int64_t ne, const int32_t *elem, const int32_t *bconn,
                                                  const int32_t *conn, const double *xyz, const double *va,
                                                  const double *lphi, const double *iphi, double alpha, double *num,
                                                  double *den)
{
    const int64_t be = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (be >= ne) return;
    constexpr int NN = D + 1;
    const int64_t e = elem[be];
    double X[NN][D], v[NN][D], f[NN];
#pragma unroll
    for (int a = 0; a < NN; ++a) {
        const int64_t g = conn[e * NN + a];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            X[a][i] = xyz[g * D + i];
            v[a][i] = va[g * D + i];
        }
        f[a] = lphi[g] + alpha * (iphi[g] - lphi[g]);
    }
    double dN[NN][D], G[D][D];
    const double vol = simplex_geom<D>(X, dN, G);
    double gf[D], L[D][D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < NN; ++a) s += f[a] * dN[a][j];
        gf[j] = s;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double t = 0.0;
#pragma unroll
            for (int a = 0; a < NN; ++a) t += v[a][i] * dN[a][j];
            L[i][j] = t;
        }
    }
    double g2 = 0.0, gLg = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        g2 += gf[i] * gf[i];
#pragma unroll
        for (int j = 0; j < D; ++j) gLg += gf[i] * L[i][j] * gf[j];
    }
    const double q = g2 > 0.0 ? gLg / g2 : 0.0;
    // int_e N_p with the degree-2 rule
    const double share = vol * Rule<D>::WF * (Rule<D>::QA + (Rule<D>::NQ - 1) * Rule<D>::QB);
#pragma unroll
    for (int a = 0; a < NN; ++a) {
        const int l = bconn[be * NN + a];
        unsafeAtomicAdd(num + l, q * share);
        unsafeAtomicAdd(den + l, share);
    }
}

__global__ __launch_bounds__(256) void k_mob_node(int64_t n, const int32_t *node, const double *lphi,
                                                  const double *iphi, double alpha, double cut, const double *num,
                                                  const double *den, double *part)
{
    __shared__ double lds[4];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0, c = 0.0;
    if (r < n) {
        const int g = node[r];
        const double f = lphi[g] + alpha * (iphi[g] - lphi[g]);
        if (fabs(f) <= cut) {
            const double Q = fabs(den[r] > 0.0 ? num[r] / den[r] : 0.0);
            s = Q * Q;
            c = 1.0;
        }
    }
    s = block_sum<256>(s, lds);
    c = block_sum<256>(c, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s;
        part[2 * blockIdx.x + 1] = c;
    }
}

// --------------------------------------------------------------- beta -----

template <int D>
__global__ __launch_bounds__(256) void k_beta_elem(int64_t ne, const int32_t *elem, const int32_t *conn,
                                                   const double *xyz, const double *lphi, const double *iphi,
                                                   double alpha, double *part)
{
    __shared__ double lds[4];
    const int64_t be = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    constexpr int NN = D + 1, NQ = Rule<D>::NQ;
    double sn = 0.0, sd = 0.0;
    if (be < ne) {
        const int64_t e = elem[be];
        double X[NN][D], f[NN];
#pragma unroll
        for (int a = 0; a < NN; ++a) {
            const int64_t g = conn[e * NN + a];
#pragma unroll
            for (int i = 0; i < D; ++i) X[a][i] = xyz[g * D + i];
            f[a] = lphi[g] + alpha * (iphi[g] - lphi[g]);
        }
        double dN[NN][D], G[D][D];
        const double w = simplex_geom<D>(X, dN, G) * Rule<D>::WF;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double fq = 0.0;
#pragma unroll
            for (int a = 0; a < NN; ++a) fq += shape_at<D>(q, a) * f[a];
            sn += w * (fq * fq * fq - fq);
            sd += w * 0.5 * fabs(fq * fq - 1.0);
        }
    }
    sn = block_sum<256>(sn, lds);
    sd = block_sum<256>(sd, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sn;
        part[2 * blockIdx.x + 1] = sd;
    }
}

__global__ __launch_bounds__(256) void k_sum2(const double *part, int nb, double *out)
{
    __shared__ double lds[4];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    a = block_sum<256>(a, lds);
    b = block_sum<256>(b, lds);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
    }
}

// ------------------------------------- mobility and beta, all indicators --
//
// The same arithmetic as k_mob_elem, k_mob_node and k_beta_elem for every
// indicator in one launch each: work units are the single-indicator
// launches' blocks, their partial sums land in one array, and k_seg_sum2
// adds each indicator's partials in the single-indicator order.  (The
// member descriptors are declared with the band-system kernels below.)

// ---------------------------------------------- band systems, row-owned ----
//
// Same organization as the momentum assembly: a workgroup owns a block of
// band rows; every (band row, incident band element) pair is one thread that
// evaluates the element and adds only that row's residual and blocks into LDS
// accumulators indexed by the slot of the column in the global row; the
// write-out compacts global slots to the band pattern.

struct TrArgs {
    int64_t n;                              // band rows
    int rpb, maxc;                          // rows per workgroup, longest global row
    const int32_t *node;                    // band row -> global node
    const int32_t *iptr, *ient;             // global node -> (element << 2 | local node)
    const uint8_t *eflag;                   // [E] 1 for band elements
    const int32_t *conn, *epos, *grow, *gcol;
    const uint32_t *islot;                  // per incidence entry: its row's block slots (eft_build_graph)
    const int32_t *brow, *bcol;             // band pattern, band-local columns
    const uint8_t *fre;                     // band row is free (else a unit row with residual 0)
    const double *xyz, *va;
    const double *lx, *ldx, *ix;            // level value, level rate, iterate of the field
    double alpha, alpha_m, vs, dt, ct;
    double *R, *J;
    double *Jc;      // optional compact blocks (s1, M) of J (B systems)
    int full_b;      // B systems with Jc: 1 writes every block of J in full, 0 only the diagonal
                     // blocks, into Jd (one per band row)
    double *Jd;      // B systems, full_b = 0: diagonal blocks [n][nv*nv] by band row
};

// What differs between the members of a batched launch (the band systems of
// the indicators, or of the solids): the band, the field, the outputs.
struct MemberDesc {
    int64_t n;                                  // band rows
    const int32_t *node, *brow, *bcol;
    const uint8_t *fre, *eflag;
    const double *lx, *ldx, *ix;                // the member's field: level value, level rate, iterate
    double *R, *J, *Jc, *Jd;
    const double *gb;                           // Allen-Cahn: gamma, beta
    const double *lphi, *iphi;                  // B: the solid's order parameter (level, iterate)
    int64_t ne;                                 // band elements
    const int32_t *elem, *bconn;                // band elements, their band-local nodes
    int64_t noff;                               // first pool node of the band (mobility sums)
};

__device__ __forceinline__ void apply_member(TrArgs &a, const MemberDesc &m)
{
    a.n = m.n;
    a.node = m.node;
    a.brow = m.brow;
    a.bcol = m.bcol;
    a.fre = m.fre;
    a.eflag = m.eflag;
    a.lx = m.lx;
    a.ldx = m.ldx;
    a.ix = m.ix;
    a.R = m.R;
    a.J = m.J;
    a.Jc = m.Jc;
    a.Jd = m.Jd;
}

// member m with off[m] <= u < off[m + 1] (off ascending, off[0] = 0)
__device__ __forceinline__ int member_of(const int32_t *__restrict__ off, int nmem, int u)
{
    int lo = 0, hi = nmem - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= u) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int D>
__global__ __launch_bounds__(256) void k_mob_elem_all(int64_t ne_tot, const int32_t *__restrict__ eoff, int nmem,
                                                      const MemberDesc *__restrict__ mem, const int32_t *conn,
                                                      const double *xyz, const double *va, double alpha, double *num,
                                                      double *den)
{
    const int64_t bg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (bg >= ne_tot) return;
    const int m = member_of(eoff, nmem, (int)bg);
    const MemberDesc &M = mem[m];
    const int64_t be = bg - eoff[m];
    constexpr int NN = D + 1;
    const int64_t e = M.elem[be];
    double X[NN][D], v[NN][D], f[NN];
#pragma unroll
    for (int a = 0; a < NN; ++a) {
        const int64_t g = conn[e * NN + a];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            X[a][i] = xyz[g * D + i];
            v[a][i] = va[g * D + i];
        }
        f[a] = M.lx[g] + alpha * (M.ix[g] - M.lx[g]);
    }
    double dN[NN][D], G[D][D];
    const double vol = simplex_geom<D>(X, dN, G);
    double gf[D], L[D][D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        double sg = 0.0;
#pragma unroll
        for (int a = 0; a < NN; ++a) sg += f[a] * dN[a][j];
        gf[j] = sg;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double t = 0.0;
#pragma unroll
            for (int a = 0; a < NN; ++a) t += v[a][i] * dN[a][j];
            L[i][j] = t;
        }
    }
    double g2 = 0.0, gLg = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        g2 += gf[i] * gf[i];
#pragma unroll
        for (int j = 0; j < D; ++j) gLg += gf[i] * L[i][j] * gf[j];
    }
    const double q = g2 > 0.0 ? gLg / g2 : 0.0;
    const double share = vol * Rule<D>::WF * (Rule<D>::QA + (Rule<D>::NQ - 1) * Rule<D>::QB);
#pragma unroll
    for (int a = 0; a < NN; ++a) {
        const int64_t l = M.noff + M.bconn[be * NN + a];
        unsafeAtomicAdd(num + l, q * share);
        unsafeAtomicAdd(den + l, share);
    }
}

__global__ __launch_bounds__(256) void k_mob_node_all(const int32_t *__restrict__ uoff, int nmem,
                                                      const MemberDesc *__restrict__ mem, double alpha, double cut,
                                                      const double *num, const double *den, double *part)
{
    __shared__ double lds[4];
    const int u = blockIdx.x;
    const int m = member_of(uoff, nmem, u);
    const MemberDesc &M = mem[m];
    const int64_t r = (int64_t)(u - uoff[m]) * blockDim.x + threadIdx.x;
    double sq = 0.0, c = 0.0;
    if (r < M.n) {
        const int g = M.node[r];
        const double f = M.lx[g] + alpha * (M.ix[g] - M.lx[g]);
        if (fabs(f) <= cut) {
            const double nu = num[M.noff + r], de = den[M.noff + r];
            const double Q = fabs(de > 0.0 ? nu / de : 0.0);
            sq = Q * Q;
            c = 1.0;
        }
    }
    sq = block_sum<256>(sq, lds);
    c = block_sum<256>(c, lds);
    if (threadIdx.x == 0) {
        part[2 * u] = sq;
        part[2 * u + 1] = c;
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_beta_elem_all(const int32_t *__restrict__ uoff, int nmem,
                                                       const MemberDesc *__restrict__ mem, const int32_t *conn,
                                                       const double *xyz, double alpha, double *part)
{
    __shared__ double lds[4];
    const int u = blockIdx.x;
    const int m = member_of(uoff, nmem, u);
    const MemberDesc &M = mem[m];
    const int64_t be = (int64_t)(u - uoff[m]) * blockDim.x + threadIdx.x;
    constexpr int NN = D + 1, NQ = Rule<D>::NQ;
    double sn = 0.0, sd = 0.0;
    if (be < M.ne) {
        const int64_t e = M.elem[be];
        double X[NN][D], f[NN];
#pragma unroll
        for (int a = 0; a < NN; ++a) {
            const int64_t g = conn[e * NN + a];
#pragma unroll
            for (int i = 0; i < D; ++i) X[a][i] = xyz[g * D + i];
            f[a] = M.lx[g] + alpha * (M.ix[g] - M.lx[g]);
        }
        double dN[NN][D], G[D][D];
        const double w = simplex_geom<D>(X, dN, G) * Rule<D>::WF;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double fq = 0.0;
#pragma unroll
            for (int a = 0; a < NN; ++a) fq += shape_at<D>(q, a) * f[a];
            sn += w * (fq * fq * fq - fq);
            sd += w * 0.5 * fabs(fq * fq - 1.0);
        }
    }
    sn = block_sum<256>(sn, lds);
    sd = block_sum<256>(sd, lds);
    if (threadIdx.x == 0) {
        part[2 * u] = sn;
        part[2 * u + 1] = sd;
    }
}

// out[m * stride + 0..1] = the sums of member m's (pair) partials
// part[2u], part[2u + 1], u in [uoff[m], uoff[m+1]), in the order of k_sum2
__global__ __launch_bounds__(256) void k_seg_sum2(const double *part, const int32_t *__restrict__ uoff, double *out,
                                                  int stride)
{
    __shared__ double lds[4];
    const int m = blockIdx.x;
    const int u0 = uoff[m], nb = uoff[m + 1] - u0;
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        a += part[2 * (u0 + i)];
        b += part[2 * (u0 + i) + 1];
    }
    a = block_sum<256>(a, lds);
    b = block_sum<256>(b, lds);
    if (threadIdx.x == 0) {
        out[m * stride] = a;
        out[m * stride + 1] = b;
    }
}

// Rows of one work unit staged in LDS by the assembly units: per row its
// first block in the band pattern (kb[nrow] closes the range: the unit's
// rows are consecutive band rows, so their blocks are contiguous), the first
// block and the length of its global row, and whether it is solved for.
struct UnitRows {
    const int *kb, *gb0, *glen, *fre;
    int nrow;
};

// Local row of block k of the unit's block range (the last row starting at
// or before it; every row has its diagonal block).
__device__ __forceinline__ int unit_row(const UnitRows &u, int k)
{
    int lo = 0, hi = u.nrow - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (u.kb[mid] <= k) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Slot of band block kb (row lr) among the global row's columns: the
// accumulators are laid out by global row position.
__device__ __forceinline__ int unit_slot(const TrArgs &a, const UnitRows &u, int lr, int64_t kb)
{
    const int32_t col = a.node[a.bcol[kb]];
    const int32_t *gc = a.gcol + u.gb0[lr];
    int lo = 0, hi = u.glen[lr] - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (gc[mid] < col) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Rows [r0, r0 + nrow) of a scalar or block band system out of LDS, flat
// over the unit's residual entries and blocks (one block per thread); rows
// that keep their value become unit rows with residual 0.
template <int BS>
__device__ __forceinline__ void band_rows_out(const TrArgs &a, int64_t r0, const UnitRows &u, const double *accJ,
                                              const double *accR)
{
    constexpr int B2 = BS * BS, BP = B2 | 1, RP = BS | 1;
    for (int t = threadIdx.x; t < u.nrow * BS; t += blockDim.x) {
        const int lr = t / BS, i = t - lr * BS;
        a.R[r0 * BS + t] = u.fre[lr] ? accR[lr * RP + i] : 0.0;
    }
    const int kb0 = u.kb[0], nblk = u.kb[u.nrow] - kb0;
    for (int t = threadIdx.x; t < nblk; t += blockDim.x) {
        const int lr = unit_row(u, kb0 + t);
        const int64_t kb = kb0 + t;
        double *dst = a.J + kb * B2;
        if (!u.fre[lr]) {
            const bool dg = a.bcol[kb] == r0 + lr;
#pragma unroll
            for (int v = 0; v < B2; ++v) dst[v] = (dg && v % (BS + 1) == 0) ? 1.0 : 0.0;
            continue;
        }
        const double *src = accJ + ((int64_t)lr * a.maxc + unit_slot(a, u, lr, kb)) * BP;
#pragma unroll
        for (int v = 0; v < B2; ++v) dst[v] = src[v];
    }
}

// Accumulator of one B-system block in LDS: s1, then M[i][k] (D x D).
template <int D> struct BAcc {
    static constexpr int N = 1 + D * D;
    static constexpr int P = N | 1;   // odd stride
};

// Block (c, cc) of the B tangent from its accumulator: s1 delta(c, cc) -
// LE(M)[c][cc], LE(M)[c][cc] = (M E + E M^T)_{ij} for the symmetric unit
// direction E of Voigt index cc and (i, j) the pair of Voigt index c.
template <int D>
__device__ __forceinline__ double b_block_entry(const double *acc, int c, int cc)
{
    int i, j, k, l;
    vpair<D>(c, i, j);
    vpair<D>(cc, k, l);
    const double *M = acc + 1;
    double s = 0.0;
    if (l == j) s += M[i * D + k];
    if (k == j && k != l) s += M[i * D + l];
    if (l == i) s += M[j * D + k];
    if (k == i && k != l) s += M[j * D + l];
    return (c == cc ? acc[0] : 0.0) - s;
}

// Rows [r0, r0 + nrow) of the B system out of LDS (blocks expanded from
// their accumulators), flat over the unit's blocks, one block per thread.
template <int D>
__device__ __forceinline__ void band_rows_out_b(const TrArgs &a, int64_t r0, const UnitRows &u, const double *accJ,
                                                const double *accR)
{
    constexpr int NVv = NV<D>::v, B2 = NVv * NVv, BP = BAcc<D>::P, RP = NVv | 1;
    for (int t = threadIdx.x; t < u.nrow * NVv; t += blockDim.x) {
        const int lr = t / NVv, i = t - lr * NVv;
        a.R[r0 * NVv + t] = u.fre[lr] ? accR[lr * RP + i] : 0.0;
    }
    const bool full = a.full_b || !a.Jc;
    const int kb0 = u.kb[0], nblk = u.kb[u.nrow] - kb0;
    for (int t = threadIdx.x; t < nblk; t += blockDim.x) {
        const int lr = unit_row(u, kb0 + t);
        const int64_t kb = kb0 + t, r = r0 + lr;
        const bool dg = a.bcol[kb] == r;
        double *dst = full ? a.J + kb * B2 : a.Jd + r * B2;
        if (!u.fre[lr]) {   // a node that keeps its value: unit row
            if (dg || full)
#pragma unroll
                for (int v = 0; v < B2; ++v) dst[v] = (dg && v % (NVv + 1) == 0) ? 1.0 : 0.0;
            if (a.Jc) {   // compact unit block: s1 = 1, M = 0
                double *dc = a.Jc + kb * BAcc<D>::N;
#pragma unroll
                for (int v = 0; v < BAcc<D>::N; ++v) dc[v] = (dg && v == 0) ? 1.0 : 0.0;
            }
            continue;
        }
        const double *src = accJ + ((int64_t)lr * a.maxc + unit_slot(a, u, lr, kb)) * BP;
        if (full || dg)   // (the diagonal blocks feed the block inverses)
#pragma unroll
            for (int c = 0; c < NVv; ++c)
#pragma unroll
                for (int cc = 0; cc < NVv; ++cc) dst[c * NVv + cc] = b_block_entry<D>(src, c, cc);
        if (a.Jc) {   // the accumulators themselves: s1, then M
            double *dc = a.Jc + kb * BAcc<D>::N;
#pragma unroll
            for (int v = 0; v < BAcc<D>::N; ++v) dc[v] = src[v];
        }
    }
}

template <int D>
__device__ __forceinline__ void ac_rows_unit(const TrArgs &a, int64_t r0, double eps, const double *gb,
                                             double *lds)
{
    constexpr int NN = D + 1, NQ = Rule<D>::NQ;
    const int64_t r1 = r0 + a.rpb < a.n ? r0 + a.rpb : a.n;
    double *accJ = lds, *accR = lds + (int64_t)a.rpb * a.maxc;
    for (int t = threadIdx.x; t < a.rpb * (a.maxc + 1); t += blockDim.x) lds[t] = 0.0;
    __syncthreads();
    const double gamma = gb[0], beta = gb[1];
    const double kh = eps * eps, al = a.alpha, ct = a.ct, i4 = 4.0 / (a.dt * a.dt);
    // incidences of the workgroup's rows, flattened (band rows are not
    // contiguous global nodes)
    // per row, staged in LDS (at most 64 rows): first incidence, end of the
    // incidences (the first again for a row that keeps its value, written
    // as a unit row), first block of the row in the global pattern
    // and, for the write-out, the row's first band block, the length of its
    // global row and whether it is solved for
    __shared__ int maxinc, s_ip0[64], s_ip1[64], s_gb0[64], s_kb[65], s_glen[64], s_fre[64];
    if (threadIdx.x == 0) maxinc = 0;
    __syncthreads();
    const int nrow = (int)(r1 - r0);
    if (threadIdx.x < nrow) {
        const int64_t gg = a.node[r0 + threadIdx.x];
        const int i0 = a.iptr[gg], i1 = a.iptr[gg + 1];
        const int fr = a.fre[r0 + threadIdx.x];
        s_ip0[threadIdx.x] = i0;
        s_ip1[threadIdx.x] = fr ? i1 : i0;
        s_gb0[threadIdx.x] = a.grow[gg];
        s_glen[threadIdx.x] = a.grow[gg + 1] - a.grow[gg];
        s_fre[threadIdx.x] = fr;
        s_kb[threadIdx.x] = a.brow[r0 + threadIdx.x];
        atomicMax(&maxinc, i1 - i0);
    }
    if (threadIdx.x == 0) s_kb[nrow] = a.brow[r1];
    __syncthreads();
    const UnitRows urows{s_kb, s_gb0, s_glen, s_fre, nrow};
    {
        // pairs dealt row-interleaved: consecutive lanes take different
        // rows, so the LDS atomics of one wavefront rarely hit one block
        for (int t = threadIdx.x; t < nrow * maxinc; t += blockDim.x) {
            const int lr = t % nrow;
            const int ii = s_ip0[lr] + t / nrow;
            if (ii >= s_ip1[lr]) continue;
            const int32_t ent = a.ient[ii];
            const int64_t e = ent >> 2;
            const int la = ent & 3;
            // the element's nodes (loaded together with its band flag),
            // rotated so that the row node comes first: local node b is node
            // (la + b) mod NN of the connectivity, and every index below is a
            // compile-time constant
            int64_t nid[NN];
#pragma unroll
            for (int b = 0; b < NN; ++b) nid[b] = a.conn[e * NN + (la + b < NN ? la + b : la + b - NN)];
            if (!a.eflag[e]) continue;
            double X[NN][D], v[NN][D], f[NN], fd[NN];
#pragma unroll
            for (int b = 0; b < NN; ++b) {
                const int64_t n = nid[b];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    X[b][i] = a.xyz[n * D + i];
                    v[b][i] = a.va[n * D + i];
                }
                const double xn = a.lx[n], xd = a.ldx[n], x1 = a.ix[n];
                const double xd1 = xd + (x1 - xn - a.dt * xd) / (a.vs * a.dt);
                fd[b] = xd + a.alpha_m * (xd1 - xd);
                f[b] = xn + a.alpha * (x1 - xn);
            }
            double dN[NN][D], G[D][D];
            const double vol = simplex_geom<D>(X, dN, G);
            // G belongs to the reference map with its origin at the element's
            // first node in the connectivity (local o0 after the rotation):
            // the sum of grad N grad N^T over the other nodes
            {
                const int o0 = la == 0 ? 0 : NN - la;
#pragma unroll
                for (int i = 0; i < D; ++i)
#pragma unroll
                    for (int j = 0; j < D; ++j) G[i][j] = 0.0;
#pragma unroll
                for (int b = 0; b < NN; ++b) {
                    const double c = b == o0 ? 0.0 : 1.0;
#pragma unroll
                    for (int i = 0; i < D; ++i)
#pragma unroll
                        for (int j = i; j < D; ++j) G[i][j] += c * dN[b][i] * dN[b][j];
                }
#pragma unroll
                for (int i = 0; i < D; ++i)
#pragma unroll
                    for (int j = 0; j < i; ++j) G[i][j] = G[j][i];
            }
            double GG = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) GG += G[i][j] * G[i][j];
            double gf[D];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                double s = 0.0;
#pragma unroll
                for (int b = 0; b < NN; ++b) s += f[b] * dN[b][j];
                gf[j] = s;
            }
            double gga = 0.0, gab[NN];
#pragma unroll
            for (int j = 0; j < D; ++j) gga += dN[0][j] * gf[j];
#pragma unroll
            for (int b = 0; b < NN; ++b) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) s += dN[0][j] * dN[b][j];
                gab[b] = s;
            }
            const double w = vol * Rule<D>::WF;
            const double gk9 = 9.0 * (gamma * kh) * (gamma * kh) * GG;
            double re = 0.0, K[NN];
#pragma unroll
            for (int b = 0; b < NN; ++b) K[b] = 0.0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                double fq = 0.0, fdq = 0.0, vq[D];
#pragma unroll
                for (int i = 0; i < D; ++i) vq[i] = 0.0;
#pragma unroll
                for (int b = 0; b < NN; ++b) {
                    const double Nb = shape_at<D>(q, b);
                    fq += Nb * f[b];
                    fdq += Nb * fd[b];
#pragma unroll
                    for (int i = 0; i < D; ++i) vq[i] += Nb * v[b][i];
                }
                double vg = 0.0, vGv = 0.0;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    vg += vq[i] * gf[i];
#pragma unroll
                    for (int j = 0; j < D; ++j) vGv += vq[i] * G[i][j] * vq[j];
                }
                // derivative of |phi^2 - 1| at the kink |phi| = 1 taken as 0 within
                // 1e-12 (flat regions interpolate to +-1 only up to rounding)
                const double f2m1 = fq * fq - 1.0;
                const double sgn = fabs(f2m1) <= 1e-12 ? 0.0 : (f2m1 > 0.0 ? 1.0 : -1.0);
                const double react = fq * fq * fq - fq - beta * 0.5 * fabs(f2m1);
                const double sh = 3.0 * fq * fq - 1.0 - beta * fq * sgn;
                const double Rphi = fdq + vg + gamma * react;
                const double tau = 1.0 / sqrt(i4 + vGv + gk9 + (gamma * sh) * (gamma * sh));
                double u[NN];
#pragma unroll
                for (int b = 0; b < NN; ++b) {
                    double s = 0.0;
#pragma unroll
                    for (int j = 0; j < D; ++j) s += vq[j] * dN[b][j];
                    u[b] = s;
                }
                const double Na = shape_at<D>(q, 0);
                re += w * (Na * (fdq + vg) + gamma * (kh * gga + Na * react) + tau * u[0] * Rphi);
#pragma unroll
                for (int ib = 0; ib < NN; ++ib) {
                    const double Nb = shape_at<D>(q, ib);
                    const double lin = ct * Nb + al * u[ib];
                    K[ib] += w * (Na * lin + al * gamma * (kh * gab[ib] + Na * sh * Nb) +
                                  tau * u[0] * (lin + al * gamma * sh * Nb));
                }
            }
            atomicAdd(accR + lr, re);
            const uint32_t sl = a.islot[ii];   // byte b: slot of (rotated) local node b
#pragma unroll
            for (int ib = 0; ib < NN; ++ib) atomicAdd(accJ + (int64_t)lr * a.maxc + ((sl >> (8 * ib)) & 0xff), K[ib]);
        }
    }
    __syncthreads();
    band_rows_out<1>(a, r0, urows, accJ, accR);
}

template <int D>
__global__ __launch_bounds__(256, 3) void k_ac_rows(TrArgs a, double eps, const double *gb /* gamma, beta */)
{
    extern __shared__ double lds[];
    ac_rows_unit<D>(a, (int64_t)blockIdx.x * a.rpb, eps, gb, lds);
}

// All Allen-Cahn systems in one launch: a grid-stride loop over work units
// (blocks of rpb rows of one member), the member found from the units'
// prefix offsets; every unit is the single-member kernel's workgroup.
template <int D>
__global__ __launch_bounds__(256, 3) void k_ac_rows_all(TrArgs a, double eps, const MemberDesc *__restrict__ mem,
                                                        const int32_t *__restrict__ uoff, int nmem)
{
    extern __shared__ double lds[];
    const int total = uoff[nmem];
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int m = member_of(uoff, nmem, u);
        TrArgs am = a;
        apply_member(am, mem[m]);
        ac_rows_unit<D>(am, (int64_t)(u - uoff[m]) * a.rpb, eps, mem[m].gb, lds);
        __syncthreads();
    }
}

template <int D>
__device__ __forceinline__ void b_rows_unit(const TrArgs &a, int64_t r0, const double *lphi, const double *iphi,
                                            double *lds)
{
    constexpr int NN = D + 1, NQ = Rule<D>::NQ, NVv = NV<D>::v;
    // A block of the tangent is s1 I - LE(M) with M = sum over elements of
    // s2 L_e (LE linear in its argument, see below), so each block
    // accumulates 1 + D*D numbers instead of NVv^2 (3x fewer LDS atomics in
    // 3D) and is expanded when written out.  LDS strides padded to an odd
    // number of doubles (bank conflicts).
    constexpr int BP = BAcc<D>::P, RP = NVv | 1;
    const int64_t r1 = r0 + a.rpb < a.n ? r0 + a.rpb : a.n;
    double *accJ = lds, *accR = lds + (int64_t)a.rpb * a.maxc * BP;
    for (int t = threadIdx.x; t < a.rpb * (a.maxc * BP + RP); t += blockDim.x) lds[t] = 0.0;
    __syncthreads();
    const double al = a.alpha, ct = a.ct, i4 = 4.0 / (a.dt * a.dt);
    // incidences of the workgroup's rows, flattened (band rows are not
    // contiguous global nodes)
    // per row, staged in LDS (at most 64 rows): first incidence, end of the
    // incidences (the first again for a row that keeps its value, written
    // as a unit row), first block of the row in the global pattern
    // and, for the write-out, the row's first band block, the length of its
    // global row and whether it is solved for
    __shared__ int maxinc, s_ip0[64], s_ip1[64], s_gb0[64], s_kb[65], s_glen[64], s_fre[64];
    if (threadIdx.x == 0) maxinc = 0;
    __syncthreads();
    const int nrow = (int)(r1 - r0);
    if (threadIdx.x < nrow) {
        const int64_t gg = a.node[r0 + threadIdx.x];
        const int i0 = a.iptr[gg], i1 = a.iptr[gg + 1];
        const int fr = a.fre[r0 + threadIdx.x];
        s_ip0[threadIdx.x] = i0;
        s_ip1[threadIdx.x] = fr ? i1 : i0;
        s_gb0[threadIdx.x] = a.grow[gg];
        s_glen[threadIdx.x] = a.grow[gg + 1] - a.grow[gg];
        s_fre[threadIdx.x] = fr;
        s_kb[threadIdx.x] = a.brow[r0 + threadIdx.x];
        atomicMax(&maxinc, i1 - i0);
    }
    if (threadIdx.x == 0) s_kb[nrow] = a.brow[r1];
    __syncthreads();
    const UnitRows urows{s_kb, s_gb0, s_glen, s_fre, nrow};
    {
        // pairs dealt row-interleaved: consecutive lanes take different
        // rows, so the LDS atomics of one wavefront rarely hit one block
        for (int t = threadIdx.x; t < nrow * maxinc; t += blockDim.x) {
            const int lr = t % nrow;
            const int ii = s_ip0[lr] + t / nrow;
            if (ii >= s_ip1[lr]) continue;
            const int32_t ent = a.ient[ii];
            const int64_t e = ent >> 2;
            const int la = ent & 3;
            // the element's nodes are loaded together with its band flag
            int64_t nid[NN];
#pragma unroll
            for (int b = 0; b < NN; ++b) nid[b] = a.conn[e * NN + b];
            if (!a.eflag[e]) continue;
            double X[NN][D], v[NN][D], am[NN];
#pragma unroll
            for (int b = 0; b < NN; ++b) {
                const int64_t n = nid[b];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    X[b][i] = a.xyz[n * D + i];
                    v[b][i] = a.va[n * D + i];
                }
                // the solid's fraction at n+alpha (the same expression as the
                // momentum assembly's): clamp((1 + phi_a)/2, 0, 1)
                const double fn = lphi[n], fa = fn + al * (iphi[n] - fn);
                am[b] = fmin(fmax(0.5 * (1.0 + fa), 0.0), 1.0);
            }
            double dN[NN][D], G[D][D];
            const double vol = simplex_geom<D>(X, dN, G);
            double L[D][D];
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    double s = 0.0;
#pragma unroll
                    for (int b = 0; b < NN; ++b) s += v[b][i] * dN[b][j];
                    L[i][j] = s;
                }
            // Every term of the residual integrand is a quadrature-point
            // scalar times a function linear in the nodal B values (the
            // interpolants B_q, dB/dt_q, the element-constant gradient of B,
            // and L B_q + B_q L^T with L constant on the element), so the
            // quadrature sums reduce to per-node weights and the nodal B
            // values enter once, after the loop:
            //   S2[b] = sum_q W_q a_q N_b(q)          (rate and L terms)
            //   T2[b] = sum_q W_q (1 - a_q) N_b(q),  T3 = sum_q W_q (1 - a_q)
            //   Wv    = sum_q W_q a_q v_q             (advection)
            // with W_q the SUPG-weighted test function of row node la.
            const double w = vol * Rule<D>::WF;
            double S1[NN], S2[NN], T2[NN], T3 = 0.0, Wv[D];
#pragma unroll
            for (int b = 0; b < NN; ++b) S1[b] = S2[b] = T2[b] = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) Wv[i] = 0.0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                double vq[D], aq = 0.0;
#pragma unroll
                for (int i = 0; i < D; ++i) vq[i] = 0.0;
#pragma unroll
                for (int b = 0; b < NN; ++b) {
                    const double Nb = shape_at<D>(q, b);
                    aq += Nb * am[b];
#pragma unroll
                    for (int i = 0; i < D; ++i) vq[i] += Nb * v[b][i];
                }
                double vGv = 0.0;
#pragma unroll
                for (int i = 0; i < D; ++i)
#pragma unroll
                    for (int j = 0; j < D; ++j) vGv += vq[i] * G[i][j] * vq[j];
                const double tau = 1.0 / sqrt(i4 + vGv);
                double U[NN], Ula = 0.0;
#pragma unroll
                for (int b = 0; b < NN; ++b) {
                    double s = 0.0;
#pragma unroll
                    for (int j = 0; j < D; ++j) s += vq[j] * dN[b][j];
                    U[b] = s;
                    if (b == la) Ula = s;
                }
                const double Wl = w * (shape_at<D>(q, la) + tau * Ula);
                const double wa = Wl * aq, wr = Wl * (1.0 - aq);
                T3 += wr;
#pragma unroll
                for (int i = 0; i < D; ++i) Wv[i] += wa * vq[i];
#pragma unroll
                for (int ib = 0; ib < NN; ++ib) {
                    const double Nb = shape_at<D>(q, ib);
                    S1[ib] += Wl * (aq * (ct * Nb + al * U[ib]) + (1.0 - aq) * al * Nb);
                    S2[ib] += wa * Nb;
                    T2[ib] += wr * Nb;
                }
            }
            // residual: nodal B values streamed once
            double re[NVv], P[NVv];
#pragma unroll
            for (int c = 0; c < NVv; ++c) re[c] = P[c] = 0.0;
#pragma unroll
            for (int b = 0; b < NN; ++b) {
                double wu = T2[b];
#pragma unroll
                for (int k = 0; k < D; ++k) wu += Wv[k] * dN[b][k];
                const int64_t n = nid[b];
#pragma unroll
                for (int c = 0; c < NVv; ++c) {
                    const double xn = a.lx[n * NVv + c], xd = a.ldx[n * NVv + c], x1 = a.ix[n * NVv + c];
                    const double xd1 = xd + (x1 - xn - a.dt * xd) / (a.vs * a.dt);
                    const double bd = xd + a.alpha_m * (xd1 - xd);
                    const double bn = xn + a.alpha * (x1 - xn);
                    re[c] += S2[b] * bd + wu * bn;
                    P[c] += S2[b] * bn;
                }
            }
            double Pf[D][D];
            vfull<D>(P, Pf);
#pragma unroll
            for (int c = 0; c < NVv; ++c) {
                int i, j;
                vpair<D>(c, i, j);
                double LP = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k) LP += L[i][k] * Pf[k][j] + Pf[i][k] * L[j][k];
                re[c] -= LP + (i == j ? T3 : 0.0);
            }
#pragma unroll
            for (int c = 0; c < NVv; ++c) atomicAdd(accR + lr * RP + c, re[c]);
            const uint32_t sl = a.islot[ii];   // byte k: slot of local node (la + k) mod NN
#pragma unroll
            for (int ib = 0; ib < NN; ++ib) {
                const double s2 = al * S2[ib];
                double *blk = accJ + ((int64_t)lr * a.maxc + ((sl >> (8 * ((ib - la + NN) % NN))) & 0xff)) * BP;
                atomicAdd(blk, S1[ib]);
#pragma unroll
                for (int i = 0; i < D; ++i)
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const double val = s2 * L[i][k];
                        if (val != 0.0) atomicAdd(blk + 1 + i * D + k, val);
                    }
            }
        }
    }
    __syncthreads();
    band_rows_out_b<D>(a, r0, urows, accJ, accR);
}

template <int D>
__global__ __launch_bounds__(256, 2) void k_b_rows(TrArgs a, const double *lphi /*[N]*/, const double *iphi)
{
    extern __shared__ double lds[];
    b_rows_unit<D>(a, (int64_t)blockIdx.x * a.rpb, lphi, iphi, lds);
}

// All B systems in one launch (as k_ac_rows_all)
template <int D>
__global__ __launch_bounds__(256, 2) void k_b_rows_all(TrArgs a, const MemberDesc *__restrict__ mem,
                                                       const int32_t *__restrict__ uoff, int nmem)
{
    extern __shared__ double lds[];
    const int total = uoff[nmem];
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        const int m = member_of(uoff, nmem, u);
        TrArgs am = a;
        apply_member(am, mem[m]);
        b_rows_unit<D>(am, (int64_t)(u - uoff[m]) * a.rpb, mem[m].lphi, mem[m].iphi, lds);
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_negate(double *x, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = -x[i];
}

__global__ __launch_bounds__(256) void k_narrow_copy(const double *__restrict__ a, float *__restrict__ b, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// member system of a block-diagonal union: rows shifted by roff, blocks by noff
__global__ __launch_bounds__(256) void k_union_fill(int64_t n, int64_t nnz, const int32_t *rowptr,
                                                    const int32_t *col, const int32_t *diag, int64_t roff,
                                                    int64_t noff, int32_t *urow, int32_t *ucol, int32_t *udiag)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        urow[roff + t] = (int32_t)(rowptr[t] + noff);
        udiag[roff + t] = (int32_t)(diag[t] + noff);
    }
    if (t < nnz) ucol[noff + t] = (int32_t)(col[t] + roff);
}

__global__ void k_set_i32(int32_t *p, int32_t v) { *p = v; }

// Largest |v|^2 over the band nodes (all bands): per-thread maxima, a
// wavefront maximum, one atomic maximum per wavefront on the bit pattern
// (non-negative doubles order like their bits).  *out must start at 0.
__global__ __launch_bounds__(256) void k_band_vmax(int64_t n, const int32_t *node, const double *vp, int bs, int d,
                                                   unsigned long long *out)
{
    double m = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const double *v = vp + (int64_t)node[r] * bs;
        double s = 0.0;
        for (int i = 0; i < d; ++i) s += v[i] * v[i];
        m = fmax(m, s);
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0 && m > 0.0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

// Batched per-member work of a union solve (all members in one launch): a
// member's segment is a pointer and a length; the launch's blocks are dealt
// to the segments in order, chunk elements each (boff: first block of each
// segment), so every reduction has a fixed partition and order.
constexpr int SEG_MAX = EFT_MAX_IND;
struct SegSet {
    int nseg;
    int64_t chunk;
    double *ptr[SEG_MAX];
    int64_t len[SEG_MAX];
    int boff[SEG_MAX + 1];
};

// the block's segment (boff ascending; a wave-uniform search)
__device__ __forceinline__ int seg_of_block(const SegSet &s, int b)
{
    int lo = 0, hi = s.nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s.boff[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// partial sums of squares of the segments, one per block
__global__ __launch_bounds__(256) void k_seg_sumsq(SegSet s, double *part)
{
    __shared__ double lds[4];
    const int b = blockIdx.x, q = seg_of_block(s, b);
    const int64_t c0 = (int64_t)(b - s.boff[q]) * s.chunk, c1 = min(c0 + s.chunk, s.len[q]);
    const double *p = s.ptr[q];
    double acc = 0.0;
    for (int64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) acc += p[i] * p[i];
    acc = block_sum<256>(acc, lds);
    if (threadIdx.x == 0) part[b] = acc;
}

// out[q] = the sum of segment q's partials in block order (0 for an empty one)
__global__ __launch_bounds__(256) void k_seg_total(const double *part, SegSet s, double *out)
{
    __shared__ double lds[4];
    const int q = blockIdx.x;
    double acc = 0.0;
    for (int b = s.boff[q] + threadIdx.x; b < s.boff[q + 1]; b += blockDim.x) acc += part[b];
    acc = block_sum<256>(acc, lds);
    if (threadIdx.x == 0) out[q] = acc;
}

// v *= 1/sqrt(nrm2[q]) (unscale: v *= sqrt(nrm2[q])) on every segment; factor
// 1 when nrm2[q] = 0
__global__ __launch_bounds__(256) void k_seg_scale(SegSet s, const double *nrm2, int unscale)
{
    const int b = blockIdx.x, q = seg_of_block(s, b);
    const double s2 = nrm2[q];
    if (!(s2 > 0.0)) return;
    const double sq = sqrt(s2);
    const int64_t c0 = (int64_t)(b - s.boff[q]) * s.chunk, c1 = min(c0 + s.chunk, s.len[q]);
    double *p = s.ptr[q];
    for (int64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) p[i] = unscale ? p[i] * sq : p[i] / sq;
}

// x_q[node_q[r] * bs + c] += dx_q[r * bs + c] on every member (segments of dx
// in rows * bs elements)
struct UpdSet {
    const int32_t *node[SEG_MAX];
    double *x[SEG_MAX];
};
__global__ __launch_bounds__(256) void k_seg_band_update(SegSet s, UpdSet u, int bs)
{
    const int b = blockIdx.x, q = seg_of_block(s, b);
    const int64_t c0 = (int64_t)(b - s.boff[q]) * s.chunk, c1 = min(c0 + s.chunk, s.len[q]);
    const double *dx = s.ptr[q];
    const int32_t *node = u.node[q];
    double *x = u.x[q];
    for (int64_t t = c0 + threadIdx.x; t < c1; t += blockDim.x) {
        const int64_t r = t / bs;
        const int c = (int)(t - r * bs);
        x[(int64_t)node[r] * bs + c] += dx[t];
    }
}


}  // namespace

// ------------------------------------------------------------- host side --

// slots of ctx->tsc: per-indicator sums (S, count, beta numerator and
// denominator), gamma and beta per indicator, per-member squared norms
constexpr int TS_SUM = 0, TS_GB = 4 * EFT_MAX_IND, TS_NRM = 6 * EFT_MAX_IND, TS_DN = TS_NRM + 128,
              TS_XN = TS_DN + 128, TS_VMAX = TS_XN + 128;

// Layout of the descriptor block (host pinned and device): the members of
// the Allen-Cahn launch, then those of the B launch, then the int32 tables
// (element offsets in the pool, node-block units, element-block units, row
// units of the two launches), each EFT_MAX_IND + 1 long.
constexpr int64_t MEM_DESC = 2 * EFT_MAX_IND;
constexpr int64_t MEM_TAB = EFT_MAX_IND + 1;
constexpr int64_t MEM_BYTES = MEM_DESC * (int64_t)sizeof(MemberDesc) + 5 * MEM_TAB * (int64_t)sizeof(int32_t);
struct MemTabs {
    MemberDesc *ac, *b;
    int32_t *eoff, *unode, *uelem, *uac, *ub;
};
static MemTabs mem_tabs(void *base)
{
    MemTabs t;
    t.ac = (MemberDesc *)base;
    t.b = t.ac + EFT_MAX_IND;
    t.eoff = (int32_t *)(t.b + EFT_MAX_IND);
    t.unode = t.eoff + MEM_TAB;
    t.uelem = t.unode + MEM_TAB;
    t.uac = t.uelem + MEM_TAB;
    t.ub = t.uac + MEM_TAB;
    return t;
}



// Exclusive scan over n items of `in` (flags or counts), in two calls: the
// count (returns the total through the host), then the writes (offsets out,
// compacted indices idx, map), so that a caller can check the total against
// its storage before anything is written.  Uses ctx->scan_tmp (reserved with
// the bands).
template <typename TI>
static eft_status scan_count(eft_ctx *ctx, const TI *in, int64_t n, int64_t *count)
{
    const int nb = (int)std::max<int64_t>(1, (n + TILE - 1) / TILE);
    if (ctx->scan_cap < nb + 1) {
        ctx->err = "scan workspace too small";
        return EFT_EINVAL;
    }
    int32_t *bsum = ctx->scan_tmp;
    hipLaunchKernelGGL(k_scan_count<TI>, dim3(nb), dim3(SB), 0, ctx->stream, in, n, bsum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(SB), 0, ctx->stream, bsum, nb, bsum + nb);
    EFT_HIP(hipGetLastError());
    EFT_HIP(hipMemcpyAsync(ctx->hscal, bsum + nb, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    *count = *(int32_t *)ctx->hscal;
    return EFT_OK;
}

template <typename TI>
static eft_status scan_write(eft_ctx *ctx, const TI *in, int64_t n, int32_t *out, int32_t *idx, int32_t *map)
{
    const int nb = (int)std::max<int64_t>(1, (n + TILE - 1) / TILE);
    hipLaunchKernelGGL(k_scan_write<TI>, dim3(nb), dim3(SB), 0, ctx->stream, in, n, ctx->scan_tmp, out, idx, map);
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}

template <typename T> static eft_status tmal(eft_ctx *ctx, T **p, int64_t count)
{
    *p = nullptr;
    if (hipMalloc((void **)p, sizeof(T) * (size_t)std::max<int64_t>(count, 1)) != hipSuccess) {
        ctx->err = "out of device memory (band reserve of " + std::to_string(count) + " entries)";
        return EFT_ENOMEM;
    }
    return EFT_OK;
}

void eft_band_free(eft_ctx *ctx)
{
    auto fr = [](void *p) {
        if (p) (void)hipFree(p);
    };
    BandPool &P = ctx->bp;
    fr(P.elem); fr(P.epos); fr(P.bconn); fr(P.node); fr(P.rowptr); fr(P.diag); fr(P.fre); fr(P.col); fr(P.eflag);
    P = BandPool{};
    for (eft_ctx::BandUnion *U : {&ctx->u_ac, &ctx->u_b}) {
        fr(U->rowptr); fr(U->col); fr(U->diag);
        U->rowptr = U->col = U->diag = nullptr;
        U->cap_n = U->cap_nnz = U->n = U->nnz = 0;
    }
    fr(ctx->bR); fr(ctx->bX); fr(ctx->tnum); fr(ctx->tden); fr(ctx->bval); fr(ctx->bcmp); fr(ctx->bdiag); fr(ctx->bpc32); fr(ctx->bdinv32); fr(ctx->iota);
    fr(ctx->scan_tmp);
    fr(ctx->dmem);
    fr(ctx->tpart);
    if (ctx->hmem) (void)hipHostFree(ctx->hmem);
    ctx->hmem = ctx->dmem = nullptr;
    ctx->tpart = nullptr;
    ctx->tpart_cap = 0;
    ctx->bR = ctx->bX = ctx->tnum = ctx->tden = ctx->bval = ctx->bcmp = ctx->bdiag = nullptr;
    ctx->bpc32 = ctx->bdinv32 = nullptr;
    ctx->iota = nullptr;
    ctx->scan_tmp = nullptr;
    ctx->scan_cap = 0;
    ctx->band.assign(ctx->n_ind, Band{});
    ctx->bands_valid = false;
}

static __global__ void k_iota(int32_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}

eft_status eft_band_reserve(eft_ctx *ctx)
{
    eft_band_free(ctx);
    if (ctx->n_ind == 0) return EFT_OK;
    const int NN = ctx->nn, nv = ctx->nv, K = ctx->n_ind;
    const int64_t N = ctx->N, E = ctx->E, nnzb = ctx->J.nnzb;
    double fr = ctx->par.band_reserve > 0.0 ? ctx->par.band_reserve : 1.0;
    if (ctx->par.band_flat < 0.0) fr = std::max(fr, (double)K);
    BandPool &P = ctx->bp;
    // (by default small meshes reserve for every band covering the whole
    // mesh: at least 2^20 elements, which costs little)
    int64_t want = (int64_t)std::ceil(fr * (double)E);
    if (!(ctx->par.band_reserve > 0.0)) want = std::max<int64_t>(want, 1 << 20);
    P.cap_e = std::max<int64_t>(1, std::min<int64_t>((int64_t)K * E, want));
    P.cap_n = std::max<int64_t>(1, std::min<int64_t>((int64_t)K * N,
                                                     (int64_t)std::ceil(ctx->band_node_ratio * (double)P.cap_e) + 8 * K));
    P.cap_nnz = std::max<int64_t>(1, std::min<int64_t>((int64_t)K * nnzb, (int64_t)ctx->maxc * P.cap_n));
    EFT_TRY(tmal(ctx, &P.elem, P.cap_e));
    EFT_TRY(tmal(ctx, &P.epos, P.cap_e * NN * NN));
    EFT_TRY(tmal(ctx, &P.bconn, P.cap_e * NN));
    EFT_TRY(tmal(ctx, &P.node, P.cap_n));
    EFT_TRY(tmal(ctx, &P.rowptr, P.cap_n + K));
    EFT_TRY(tmal(ctx, &P.diag, P.cap_n));
    EFT_TRY(tmal(ctx, &P.fre, P.cap_n));
    EFT_TRY(tmal(ctx, &P.col, P.cap_nnz));
    EFT_TRY(tmal(ctx, &P.eflag, (int64_t)K * E));
    for (eft_ctx::BandUnion *U : {&ctx->u_ac, &ctx->u_b}) {
        EFT_TRY(tmal(ctx, &U->rowptr, P.cap_n + 1));
        EFT_TRY(tmal(ctx, &U->diag, P.cap_n));
        EFT_TRY(tmal(ctx, &U->col, P.cap_nnz));
        U->cap_n = P.cap_n + 1;
        U->cap_nnz = P.cap_nnz;
    }
    EFT_TRY(tmal(ctx, &ctx->bR, P.cap_n * nv));
    EFT_TRY(tmal(ctx, &ctx->bX, P.cap_n * nv));
    EFT_TRY(tmal(ctx, &ctx->tnum, P.cap_n));
    EFT_TRY(tmal(ctx, &ctx->tden, P.cap_n));
    EFT_TRY(tmal(ctx, &ctx->bval, P.cap_nnz));   // Allen-Cahn values (1 x 1 blocks)
    EFT_TRY(tmal(ctx, &ctx->bcmp, P.cap_nnz * (1 + ctx->dim * ctx->dim)));
    EFT_TRY(tmal(ctx, &ctx->bdiag, P.cap_n * nv * nv));
    EFT_TRY(tmal(ctx, &ctx->bpc32, P.cap_nnz * (1 + ctx->dim * ctx->dim)));
    EFT_TRY(tmal(ctx, &ctx->bdinv32, P.cap_n * nv * nv));
    EFT_TRY(tmal(ctx, &ctx->iota, P.cap_n));
    const int64_t nb = (std::max(E, N) + TILE - 1) / TILE + 1;
    EFT_TRY(tmal(ctx, &ctx->scan_tmp, nb + 1));
    ctx->scan_cap = nb + 1;
    hipLaunchKernelGGL(k_iota, dim3(eft_grid(P.cap_n, 256)), dim3(256), 0, ctx->stream, ctx->iota, P.cap_n);
    // batched transport: member descriptors and unit tables, partial sums
    if (hipHostMalloc(&ctx->hmem, MEM_BYTES, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&ctx->dmem, MEM_BYTES) != hipSuccess) {
        ctx->err = "out of memory (transport descriptors)";
        return EFT_ENOMEM;
    }
    ctx->tpart_cap = 2 * (P.cap_n / 256 + P.cap_e / 256 + 4 * K + 64);
    EFT_TRY(tmal(ctx, &ctx->tpart, ctx->tpart_cap));
    EFT_HIP(hipGetLastError());
    // the band unions are Krylov systems too: the Allen-Cahn union has up to
    // cap_n rows, the B union up to cap_n rows of nv
    EFT_TRY(eft_krylov_reserve(ctx, P.cap_n, nv, ctx->par.restart));
    return EFT_OK;
}

// Descriptors of every Allen-Cahn member (indicator) and every B member
// (solid) for the current bands and fields, uploaded in one copy.
static eft_status upload_members(eft_ctx *ctx, const eft_state *lvl, const eft_iterate *it, int rpb)
{
    const int K = ctx->n_ind, S = ctx->n_s, nv = ctx->nv, d2 = 1 + ctx->dim * ctx->dim;
    const int64_t N = ctx->N;
    MemTabs h = mem_tabs(ctx->hmem);
    const BandPool &P = ctx->bp;
    h.eoff[0] = h.unode[0] = h.uelem[0] = h.uac[0] = h.ub[0] = 0;
    for (int k = 0; k < K; ++k) {
        const Band &B = ctx->band[k];
        MemberDesc &m = h.ac[k];
        m = MemberDesc{};
        m.n = B.n;
        m.node = B.node;
        m.brow = B.rowptr;
        m.bcol = B.col;
        m.fre = B.fre;
        m.eflag = B.eflag;
        m.lx = lvl->phi + (int64_t)k * N;
        m.ldx = lvl->phidot + (int64_t)k * N;
        m.ix = it->phi + (int64_t)k * N;
        m.R = ctx->bR + ctx->u_ac.roff[k];
        m.J = ctx->bval + ctx->u_ac.noff[k];
        m.gb = ctx->tsc + TS_GB + 2 * k;
        m.ne = B.ne;
        m.elem = B.elem;
        m.bconn = B.bconn_;
        m.noff = B.node - P.node;
        h.eoff[k + 1] = h.eoff[k] + (int32_t)B.ne;
        h.unode[k + 1] = h.unode[k] + (int32_t)((B.n + 255) / 256);
        h.uelem[k + 1] = h.uelem[k] + (int32_t)((B.ne + 255) / 256);
        h.uac[k + 1] = h.uac[k] + (int32_t)((B.n + rpb - 1) / rpb);
    }
    for (int sI = 0; sI < S; ++sI) {
        const int k = ctx->solid_ind[sI];
        const Band &B = ctx->band[k];
        MemberDesc &m = h.b[sI];
        m = MemberDesc{};
        m.n = B.n;
        m.node = B.node;
        m.brow = B.rowptr;
        m.bcol = B.col;
        m.fre = B.fre;
        m.eflag = B.eflag;
        m.lx = lvl->B + (int64_t)sI * N * nv;
        m.ldx = lvl->Bdot + (int64_t)sI * N * nv;
        m.ix = it->B + (int64_t)sI * N * nv;
        m.R = ctx->bR + ctx->u_b.roff[sI] * nv;
        m.Jc = ctx->bcmp + ctx->u_b.noff[sI] * d2;
        m.Jd = ctx->bdiag + ctx->u_b.roff[sI] * nv * nv;
        m.lphi = lvl->phi + (int64_t)k * N;
        m.iphi = it->phi + (int64_t)k * N;
        m.ne = B.ne;
        m.elem = B.elem;
        m.bconn = B.bconn_;
        m.noff = B.node - P.node;
        h.ub[sI + 1] = h.ub[sI] + (int32_t)((B.n + rpb - 1) / rpb);
    }
    EFT_HIP(hipMemcpyAsync(ctx->dmem, ctx->hmem, MEM_BYTES, hipMemcpyHostToDevice, ctx->stream));
    return EFT_OK;
}

static eft_status band_full(eft_ctx *ctx, const char *what, int64_t need, int64_t cap)
{
    ctx->bands_valid = false;
    ctx->err = std::string("the bands of all indicators need ") + std::to_string(need) + " " + what +
               ", more than the " + std::to_string(cap) + " reserved (band_reserve = " +
               std::to_string(ctx->par.band_reserve) + "); raise band_reserve with eft_set_params";
    return EFT_ENOMEM;
}

static eft_status build_union(eft_ctx *ctx, eft_ctx::BandUnion &U, const std::vector<int> &bands)
{
    U.band_of = bands;
    U.roff.assign(bands.size(), 0);
    U.noff.assign(bands.size(), 0);
    int64_t n = 0, nnz = 0;
    for (size_t q = 0; q < bands.size(); ++q) {
        U.roff[q] = n;
        U.noff[q] = nnz;
        n += ctx->band[bands[q]].n;
        nnz += ctx->band[bands[q]].nnz;
    }
    if (n + 1 > U.cap_n) return band_full(ctx, "union rows", n + 1, U.cap_n);
    if (nnz > U.cap_nnz) return band_full(ctx, "union pattern entries", nnz, U.cap_nnz);
    U.n = n;
    U.nnz = nnz;
    for (size_t q = 0; q < bands.size(); ++q) {
        const Band &B = ctx->band[bands[q]];
        const int64_t m = std::max(B.n, B.nnz);
        if (m > 0)
            hipLaunchKernelGGL(k_union_fill, dim3(eft_grid(m, 256)), dim3(256), 0, ctx->stream, B.n, B.nnz, B.rowptr,
                               B.col, B.diag, U.roff[q], U.noff[q], U.rowptr, U.col, U.diag);
    }
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, ctx->stream, U.rowptr + n, (int32_t)nnz);
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}

eft_status eft_bands_build_dev(eft_ctx *ctx, const double *phi_n)
{
    const int D = ctx->dim, NN = D + 1;
    const int64_t N = ctx->N, E = ctx->E;
    const int64_t ncell = (int64_t)ctx->ng[0] * ctx->ng[1] * ctx->ng[2];
    BandPool &P = ctx->bp;
    if (!P.elem) {
        ctx->err = "band storage not reserved";
        return EFT_EINVAL;
    }
    ctx->bands_valid = false;
    ctx->band.assign(ctx->n_ind, Band{});
    const double thr = 1.0 - ctx->par.band_flat;
    int64_t eoff = 0, noff = 0, zoff = 0;   // pool slices taken so far
    for (int k = 0; k < ctx->n_ind; ++k) {
        const double *phi = phi_n + (int64_t)k * N;
        Band &B = ctx->band[k];
        EFT_TRY(eft_fill_u8(ctx, ctx->seed, ncell));
        EFT_TRY(eft_fill_u8(ctx, ctx->nin, N));
        EFT_TRY(eft_fill_u8(ctx, ctx->nout, N));
        if (D == 2)
            hipLaunchKernelGGL(k_seed<2>, dim3(eft_grid(E, 256)), dim3(256), 0, ctx->stream, E, ctx->conn, ctx->cell_of,
                               phi, thr, ctx->seed);
        else
            hipLaunchKernelGGL(k_seed<3>, dim3(eft_grid(E, 256)), dim3(256), 0, ctx->stream, E, ctx->conn, ctx->cell_of,
                               phi, thr, ctx->seed);
        hipLaunchKernelGGL(k_dilate, dim3(eft_grid(ncell, 256)), dim3(256), 0, ctx->stream, ctx->ng[0], ctx->ng[1],
                           ctx->ng[2], ctx->par.band_halo, ctx->seed, ctx->active);
        if (D == 2)
            hipLaunchKernelGGL(k_mark<2>, dim3(eft_grid(E, 256)), dim3(256), 0, ctx->stream, E, ctx->conn, ctx->cell_of,
                               ctx->active, ctx->ein, ctx->nin, ctx->nout);
        else
            hipLaunchKernelGGL(k_mark<3>, dim3(eft_grid(E, 256)), dim3(256), 0, ctx->stream, E, ctx->conn, ctx->cell_of,
                               ctx->active, ctx->ein, ctx->nin, ctx->nout);
        EFT_HIP(hipGetLastError());
        B.eflag = P.eflag + (int64_t)k * E;
        EFT_HIP(hipMemcpyAsync(B.eflag, ctx->ein, E, hipMemcpyDeviceToDevice, ctx->stream));
        // element list
        int64_t ne = 0, n = 0, nnz = 0;
        EFT_TRY(scan_count<uint8_t>(ctx, ctx->ein, E, &ne));
        if (eoff + ne > P.cap_e) return band_full(ctx, "elements", eoff + ne, P.cap_e);
        B.elem = P.elem + eoff;
        B.epos = P.epos + eoff * NN * NN;
        B.bconn_ = P.bconn + eoff * NN;
        EFT_TRY(scan_write<uint8_t>(ctx, ctx->ein, E, nullptr, B.elem, nullptr));
        // node list and the global -> band map
        EFT_TRY(scan_count<uint8_t>(ctx, ctx->nin, N, &n));
        if (noff + n > P.cap_n) return band_full(ctx, "nodes", noff + n, P.cap_n);
        B.node = P.node + noff;
        B.fre = P.fre + noff;
        B.diag = P.diag + noff;
        B.rowptr = P.rowptr + noff + k;
        EFT_TRY(scan_write<uint8_t>(ctx, ctx->nin, N, nullptr, B.node, ctx->g2b));
        B.n = n;
        B.ne = ne;
        if (n > 0) {
            hipLaunchKernelGGL(k_band_free, dim3(eft_grid(n, 256)), dim3(256), 0, ctx->stream, n, B.node, ctx->nout,
                               B.fre);
            hipLaunchKernelGGL(k_band_rowcount, dim3(eft_grid(n, 256)), dim3(256), 0, ctx->stream, n, B.node,
                               ctx->J.rowptr, ctx->J.col, ctx->g2b, B.rowptr);
            EFT_HIP(hipGetLastError());
        }
        // exclusive scan of the row counts, in place (rowptr[n] = total)
        EFT_TRY(scan_count<int32_t>(ctx, B.rowptr, n, &nnz));
        if (zoff + nnz > P.cap_nnz) return band_full(ctx, "pattern entries", zoff + nnz, P.cap_nnz);
        EFT_TRY(scan_write<int32_t>(ctx, B.rowptr, n, B.rowptr, nullptr, nullptr));
        hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, ctx->stream, B.rowptr + n, (int32_t)nnz);
        B.nnz = nnz;
        B.col = P.col + zoff;
        if (n > 0) {
            hipLaunchKernelGGL(k_band_fill, dim3(eft_grid(n, 256)), dim3(256), 0, ctx->stream, n, B.node, ctx->J.rowptr,
                               ctx->J.col, ctx->g2b, B.rowptr, B.col, B.diag, ctx->gpos2b);
        }
        if (ne > 0) {
            if (D == 2)
                hipLaunchKernelGGL(k_band_epos<2>, dim3(eft_grid(ne, 256)), dim3(256), 0, ctx->stream, ne, B.elem,
                                   ctx->conn, ctx->epos, ctx->gpos2b, ctx->g2b, B.epos, B.bconn_);
            else
                hipLaunchKernelGGL(k_band_epos<3>, dim3(eft_grid(ne, 256)), dim3(256), 0, ctx->stream, ne, B.elem,
                                   ctx->conn, ctx->epos, ctx->gpos2b, ctx->g2b, B.epos, B.bconn_);
        }
        EFT_HIP(hipGetLastError());
        eoff += ne;
        noff += n;
        zoff += nnz;
    }
    P.used_n = noff;
    // unions of the Allen-Cahn systems (one per indicator) and of the B
    // systems (one per solid, on its indicator's band)
    std::vector<int> ac_bands, b_bands;
    for (int k = 0; k < ctx->n_ind; ++k) ac_bands.push_back(k);
    for (int sI = 0; sI < ctx->n_s; ++sI) b_bands.push_back(ctx->solid_ind[sI]);
    EFT_TRY(build_union(ctx, ctx->u_ac, ac_bands));
    EFT_TRY(build_union(ctx, ctx->u_b, b_bands));
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    ctx->bands_valid = true;
    return EFT_OK;
}



// gamma and beta of every indicator at the iterate (eq. tdm-num with the RMS
// over the diffuse region, and the multiplier of Sec. 2.2.1): the sums of all
// indicators are read back in one transfer; gamma, beta are left on the
// device at tsc[TS_GB + 2k] for the element kernels and returned in gb
static eft_status mobility_beta_all(eft_ctx *ctx, const eft_state *lvl, const eft_iterate *it, double *gb,
                                    double *vmax = nullptr)
{
    const int D = ctx->dim;
    const int64_t N = ctx->N;
    GA ga = ga_of(ctx->par.rho_inf, ctx->par.dt);
    const int K = ctx->n_ind;
    if (K == 0) return EFT_OK;
    EFT_TRY(eft_fill(ctx, ctx->tsc + TS_SUM, 4 * (int64_t)K, 0.0));
    EFT_TRY(eft_fill(ctx, ctx->tsc + TS_VMAX, 1, 0.0));
    if (vmax && ctx->bp.used_n > 0) {
        const int64_t nb = std::min<int64_t>(1024, eft_grid(ctx->bp.used_n, 256));
        hipLaunchKernelGGL(k_band_vmax, dim3(nb), dim3(256), 0, ctx->stream, ctx->bp.used_n, ctx->bp.node, it->vp,
                           ctx->bs, ctx->dim, (unsigned long long *)(ctx->tsc + TS_VMAX));
    }
    // every indicator at once (the member descriptors hold each one's band
    // and field; the sums land per indicator in the single-indicator order)
    EFT_TRY(upload_members(ctx, lvl, it, std::min(ctx->rpb, 64)));
    const MemTabs T = mem_tabs(ctx->dmem);
    const MemTabs H = mem_tabs(ctx->hmem);
    const int64_t ne_tot = H.eoff[K], nu_node = H.unode[K], nu_elem = H.uelem[K];
    if (2 * std::max(nu_node, nu_elem) > ctx->tpart_cap) {
        ctx->err = "transport partial-sum buffer too small";
        return EFT_EINVAL;
    }
    if (ctx->bp.used_n > 0) {
        EFT_TRY(eft_fill(ctx, ctx->tnum, ctx->bp.used_n, 0.0));
        EFT_TRY(eft_fill(ctx, ctx->tden, ctx->bp.used_n, 0.0));
    }
    if (ne_tot > 0) {
        if (D == 2)
            hipLaunchKernelGGL(k_mob_elem_all<2>, dim3(eft_grid(ne_tot, 256)), dim3(256), 0, ctx->stream, ne_tot,
                               T.eoff, K, T.ac, ctx->conn, ctx->xyz, ctx->va, ga.alpha, ctx->tnum, ctx->tden);
        else
            hipLaunchKernelGGL(k_mob_elem_all<3>, dim3(eft_grid(ne_tot, 256)), dim3(256), 0, ctx->stream, ne_tot,
                               T.eoff, K, T.ac, ctx->conn, ctx->xyz, ctx->va, ga.alpha, ctx->tnum, ctx->tden);
    }
    if (nu_node > 0) {
        hipLaunchKernelGGL(k_mob_node_all, dim3(nu_node), dim3(256), 0, ctx->stream, T.unode, K, T.ac, ga.alpha,
                           ctx->par.di_cut, ctx->tnum, ctx->tden, ctx->tpart);
        hipLaunchKernelGGL(k_seg_sum2, dim3(K), dim3(256), 0, ctx->stream, ctx->tpart, T.unode, ctx->tsc + TS_SUM, 4);
    }
    if (nu_elem > 0) {
        if (D == 2)
            hipLaunchKernelGGL(k_beta_elem_all<2>, dim3(nu_elem), dim3(256), 0, ctx->stream, T.uelem, K, T.ac,
                               ctx->conn, ctx->xyz, ga.alpha, ctx->tpart);
        else
            hipLaunchKernelGGL(k_beta_elem_all<3>, dim3(nu_elem), dim3(256), 0, ctx->stream, T.uelem, K, T.ac,
                               ctx->conn, ctx->xyz, ga.alpha, ctx->tpart);
        hipLaunchKernelGGL(k_seg_sum2, dim3(K), dim3(256), 0, ctx->stream, ctx->tpart, T.uelem, ctx->tsc + TS_SUM + 2,
                           4);
    }
    EFT_HIP(hipGetLastError());
    (void)N;
    EFT_HIP(hipMemcpyAsync(ctx->htsc + TS_SUM, ctx->tsc + TS_SUM, sizeof(double) * 4 * K, hipMemcpyDeviceToHost,
                           ctx->stream));
    EFT_HIP(hipMemcpyAsync(ctx->htsc + TS_VMAX, ctx->tsc + TS_VMAX, sizeof(double), hipMemcpyDeviceToHost,
                           ctx->stream));
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    if (vmax) *vmax = std::sqrt(ctx->htsc[TS_VMAX]);
    for (int k = 0; k < K; ++k) {
        const double *h = ctx->htsc + TS_SUM + 4 * k;
        gb[2 * k] = h[1] > 0.0 ? sqrt(h[0] / h[1]) / ctx->par.eta : 0.0;
        gb[2 * k + 1] = h[3] > 0.0 ? h[2] / h[3] : 0.0;
        ctx->htsc[TS_GB + 2 * k] = gb[2 * k];
        ctx->htsc[TS_GB + 2 * k + 1] = gb[2 * k + 1];
    }
    EFT_HIP(hipMemcpyAsync(ctx->tsc + TS_GB, ctx->htsc + TS_GB, sizeof(double) * 2 * K, hipMemcpyHostToDevice,
                           ctx->stream));
    return EFT_OK;
}

static TrArgs tr_args(eft_ctx *ctx, const Band &B, const double *lx, const double *ldx, const double *ix)
{
    GA ga = ga_of(ctx->par.rho_inf, ctx->par.dt);
    TrArgs a;
    a.Jc = nullptr;
    a.full_b = 1;
    a.Jd = nullptr;
    a.fre = B.fre;
    a.n = B.n;
    a.rpb = std::min(ctx->rpb, 64);
    a.maxc = ctx->maxc;
    a.node = B.node;
    a.iptr = ctx->iptr;
    a.ient = ctx->ient;
    a.eflag = B.eflag;
    a.conn = ctx->conn;
    a.epos = ctx->epos;
    a.islot = ctx->islot;
    a.grow = ctx->J.rowptr;
    a.gcol = ctx->J.col;
    a.brow = B.rowptr;
    a.bcol = B.col;
    a.xyz = ctx->xyz;
    a.va = ctx->va;
    a.lx = lx;
    a.ldx = ldx;
    a.ix = ix;
    a.alpha = ga.alpha;
    a.alpha_m = ga.alpha_m;
    a.vs = ga.vs;
    a.dt = ga.dt;
    a.ct = ga.ct;
    a.R = ctx->bR;
    a.J = ctx->bval;
    return a;
}

// Allen-Cahn system of indicator k on its band (unit rows for kept nodes)
// into R, J; gamma, beta at gb (device)
static eft_status assemble_ac(eft_ctx *ctx, const eft_state *lvl, const eft_iterate *it, int k, double *R, double *J,
                              const double *gb)
{
    const int64_t N = ctx->N;
    const Band &B = ctx->band[k];
    TrArgs a = tr_args(ctx, B, lvl->phi + (int64_t)k * N, lvl->phidot + (int64_t)k * N, it->phi + (int64_t)k * N);
    a.R = R;
    a.J = J;
    if (B.n > 0) {
        const size_t shm = (size_t)a.rpb * (a.maxc + 1) * sizeof(double);
        if (ctx->dim == 2)
            hipLaunchKernelGGL(k_ac_rows<2>, dim3(eft_grid(B.n, a.rpb)), dim3(256), shm, ctx->stream, a, ctx->par.eps,
                               gb);
        else
            hipLaunchKernelGGL(k_ac_rows<3>, dim3(eft_grid(B.n, a.rpb)), dim3(256), shm, ctx->stream, a, ctx->par.eps,
                               gb);
    }
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}

// B system of solid s on the band of its indicator into R, J; the solid
// fractions in ctx->as must come from the current order parameters
// (Jc: the compact blocks; full: every block of J also in full, else only
// the diagonal blocks)
static eft_status assemble_b(eft_ctx *ctx, const eft_state *lvl, const eft_iterate *it, int s, double *R, double *J,
                             double *Jc, bool full, double *Jd)
{
    const int64_t N = ctx->N;
    const int nv = ctx->nv;
    const Band &B = ctx->band[ctx->solid_ind[s]];
    TrArgs a = tr_args(ctx, B, lvl->B + (int64_t)s * N * nv, lvl->Bdot + (int64_t)s * N * nv, it->B + (int64_t)s * N * nv);
    a.R = R;
    a.J = J;
    a.Jc = Jc;
    a.full_b = full ? 1 : 0;
    a.Jd = Jd;
    if (B.n > 0) {
        const int bp = ctx->dim == 2 ? BAcc<2>::P : BAcc<3>::P;
        const size_t shm = (size_t)a.rpb * ((size_t)a.maxc * bp + (nv | 1)) * sizeof(double);
        const int64_t ko = (int64_t)ctx->solid_ind[s] * N;
        if (ctx->dim == 2)
            hipLaunchKernelGGL(k_b_rows<2>, dim3(eft_grid(B.n, a.rpb)), dim3(256), shm, ctx->stream, a,
                               lvl->phi + ko, it->phi + ko);
        else
            hipLaunchKernelGGL(k_b_rows<3>, dim3(eft_grid(B.n, a.rpb)), dim3(256), shm, ctx->stream, a,
                               lvl->phi + ko, it->phi + ko);
    }
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}

// Every band system of one kind in one launch (kind 0: the Allen-Cahn
// systems of all indicators, with gamma, beta on the device; kind 1: the B
// systems of all solids, compact blocks and diagonal blocks).  The member
// descriptors were uploaded by mobility_beta_all for these fields.
static eft_status assemble_all(eft_ctx *ctx, const eft_state *lvl, const eft_iterate *it, int kind)
{
    const int K = ctx->n_ind, S = ctx->n_s;
    const MemTabs T = mem_tabs(ctx->dmem), H = mem_tabs(ctx->hmem);
    TrArgs a = tr_args(ctx, ctx->band[0], nullptr, nullptr, nullptr);
    a.full_b = 0;
    const int nmem = kind == 0 ? K : S;
    const int units = kind == 0 ? H.uac[K] : H.ub[S];
    if (units == 0) return EFT_OK;
    const int grid = std::min(units, 4096);
    if (kind == 0) {
        const size_t shm = (size_t)a.rpb * (a.maxc + 1) * sizeof(double);
        if (ctx->dim == 2)
            hipLaunchKernelGGL(k_ac_rows_all<2>, dim3(grid), dim3(256), shm, ctx->stream, a, ctx->par.eps, T.ac, T.uac,
                               nmem);
        else
            hipLaunchKernelGGL(k_ac_rows_all<3>, dim3(grid), dim3(256), shm, ctx->stream, a, ctx->par.eps, T.ac, T.uac,
                               nmem);
    } else {
        const int nv = ctx->nv;
        const int bp = ctx->dim == 2 ? BAcc<2>::P : BAcc<3>::P;
        const size_t shm = (size_t)a.rpb * ((size_t)a.maxc * bp + (nv | 1)) * sizeof(double);
        if (ctx->dim == 2)
            hipLaunchKernelGGL(k_b_rows_all<2>, dim3(grid), dim3(256), shm, ctx->stream, a, T.b, T.ub, nmem);
        else
            hipLaunchKernelGGL(k_b_rows_all<3>, dim3(grid), dim3(256), shm, ctx->stream, a, T.b, T.ub, nmem);
    }
    EFT_HIP(hipGetLastError());
    (void)lvl;
    (void)it;
    return EFT_OK;
}

// A segment set over the given pointers and lengths, its chunk chosen so that
// the blocks fit the reduction buffer (at least 16 blocks of 256 per chunk)
static SegSet seg_set(eft_ctx *ctx, const std::vector<double *> &ptr, const std::vector<int64_t> &len)
{
    SegSet s{};
    s.nseg = (int)ptr.size();
    int64_t total = 0;
    for (int64_t l : len) total += l;
    int64_t chunk = 4096;
    while ((total + chunk - 1) / chunk + s.nseg > (int64_t)ctx->nred) chunk *= 2;
    s.chunk = chunk;
    s.boff[0] = 0;
    for (int q = 0; q < s.nseg; ++q) {
        s.ptr[q] = ptr[q];
        s.len[q] = len[q];
        s.boff[q + 1] = s.boff[q] + (int)((len[q] + chunk - 1) / chunk);
    }
    return s;
}

// out[q] = ||segment q||^2 for every segment: two launches
static void seg_sumsq(eft_ctx *ctx, const SegSet &s, double *out)
{
    if (s.nseg == 0) return;
    const int nb = s.boff[s.nseg];
    if (nb > 0) hipLaunchKernelGGL(k_seg_sumsq, dim3(nb), dim3(256), 0, ctx->stream, s, ctx->red);
    hipLaunchKernelGGL(k_seg_total, dim3(s.nseg), dim3(256), 0, ctx->stream, ctx->red, s, out);
}

// Solve the assembled union system (R in bR, matrix in bval) of one kind:
// rhs = -R; with several members, member k's right-hand side is divided by
// ||R_k|| (its solution multiplied back afterwards), which weights the
// union residual like scaling the member's rows, and FGMRES runs to
// lin_rtol/sqrt(members), so that every member meets lin_rtol; then
// x_k += dx_k on the band nodes.  ratio[q] = ||dx_q|| / ||x_q|| (one
// read-back for all members).
static eft_status union_solve(eft_ctx *ctx, const eft_ctx::BandUnion &U, int bs, const std::vector<double *> &x,
                              const std::vector<int64_t> &xlen, double *ratio, eft_solve_info *si)
{
    const int64_t nd = U.n * bs;
    const int Q = (int)U.band_of.size();
    hipLaunchKernelGGL(k_negate, dim3(eft_grid(nd, 256)), dim3(256), 0, ctx->stream, ctx->bR, nd);
    int members = 0;
    for (int q = 0; q < Q; ++q) members += ctx->band[U.band_of[q]].n > 0 ? 1 : 0;
    const bool scaled = members > 1;
    if (Q > SEG_MAX) {
        ctx->err = "too many members in a union system";
        return EFT_EINVAL;
    }
    // the members' segments of the union vectors (R, then dx), and the fields
    std::vector<double *> rptr(Q), dptr(Q);
    std::vector<int64_t> rlen(Q);
    for (int q = 0; q < Q; ++q) {
        rptr[q] = ctx->bR + U.roff[q] * bs;
        dptr[q] = ctx->bX + U.roff[q] * bs;
        rlen[q] = ctx->band[U.band_of[q]].n * bs;
    }
    const SegSet sR = seg_set(ctx, rptr, rlen), sX = seg_set(ctx, dptr, rlen);
    if (scaled) {   // all members at once: their squared norms, then the scaling
        seg_sumsq(ctx, sR, ctx->tsc + TS_NRM);
        if (sR.boff[Q] > 0)
            hipLaunchKernelGGL(k_seg_scale, dim3(sR.boff[Q]), dim3(256), 0, ctx->stream, sR, ctx->tsc + TS_NRM, 0);
    }
    EFT_HIP(hipGetLastError());
    eft_matrix A;
    A.bs = bs;
    A.n = U.n;
    A.nnzb = U.nnz;
    A.rowptr = U.rowptr;
    A.col = U.col;
    A.diag = U.diag;
    A.val = ctx->bval;
    A.bcmp = nullptr;
    if (bs > 1) {   // B systems: compact blocks for the products, diagonal blocks by row for the inverses
        A.bcmp = ctx->bcmp;
        A.val = ctx->bdiag;
        A.diag = ctx->iota;
    }
    // the Jacobi preconditioner reads FP32 copies (the products and the
    // Krylov vectors stay FP64); the solve's set-up writes the inverses
    const int64_t nc = U.nnz * (bs > 1 ? 1 + ctx->dim * ctx->dim : 1);
    if (nc > 0)
        hipLaunchKernelGGL(k_narrow_copy, dim3(eft_grid(nc, 256)), dim3(256), 0, ctx->stream,
                           bs > 1 ? ctx->bcmp : ctx->bval, ctx->bpc32, nc);
    A.pc32 = ctx->bpc32;
    A.dinv32 = ctx->bdinv32;
    const double rtol = ctx->par.lin_rtol / std::sqrt((double)std::max(members, 1));
    eft_status st = eft_fgmres_dev(ctx, &A, ctx->bR, ctx->bX, si, rtol);
    if (st != EFT_OK && st != EFT_ENOTCONV) return st;
    // all members at once: unscale dx, x_q += dx_q on the band nodes, then
    // ||dx_q||^2 and ||x_q||^2
    if (sX.boff[Q] > 0) {
        if (scaled)
            hipLaunchKernelGGL(k_seg_scale, dim3(sX.boff[Q]), dim3(256), 0, ctx->stream, sX, ctx->tsc + TS_NRM, 1);
        UpdSet u{};
        for (int q = 0; q < Q; ++q) {
            u.node[q] = ctx->band[U.band_of[q]].node;
            u.x[q] = x[q];
        }
        hipLaunchKernelGGL(k_seg_band_update, dim3(sX.boff[Q]), dim3(256), 0, ctx->stream, sX, u, bs);
    }
    seg_sumsq(ctx, sX, ctx->tsc + TS_DN);
    seg_sumsq(ctx, seg_set(ctx, std::vector<double *>(x.begin(), x.end()), xlen), ctx->tsc + TS_XN);
    EFT_HIP(hipGetLastError());
    EFT_HIP(hipMemcpyAsync(ctx->htsc + TS_DN, ctx->tsc + TS_DN, sizeof(double) * 256, hipMemcpyDeviceToHost,
                           ctx->stream));
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    for (int q = 0; q < Q; ++q)
        ratio[q] = std::sqrt(ctx->htsc[TS_DN + q]) / std::max(std::sqrt(ctx->htsc[TS_XN + q]), 1e-300);
    return st;
}

eft_status eft_transport_dev(eft_ctx *ctx, const eft_state *lvl, eft_iterate *it, eft_transport_info *info)
{
    if (!ctx->bands_valid) {
        ctx->err = "eft_bands_build must run before the transport";
        return EFT_EINVAL;
    }
    const int nv = ctx->nv, K = ctx->n_ind, S = ctx->n_s;
    const int64_t N = ctx->N;
    eft_transport_info inf{};
    inf.n_ind = K;
    inf.n_solid = S;
    eft_status worst = EFT_OK;
    EFT_TRY(eft_props(ctx, lvl, it));
    std::vector<double> gb(2 * std::max(K, 1));
    double vmax = 0.0;
    EFT_TRY(mobility_beta_all(ctx, lvl, it, gb.data(), &vmax));
    // the band must hold the interface through the step: its halo covers
    // max|v| dt (grid-cell band; no test for the whole-mesh transport)
    if (ctx->par.band_flat >= 0.0) {
        const double reach = vmax * ctx->par.dt, room = ctx->par.band_halo * ctx->par.band_cell * ctx->h_min;
        if (!(reach < room)) {
            ctx->err = "band overflow: max|v| dt = " + std::to_string(reach) + " on the bands reaches band_halo band_cell h = " +
                       std::to_string(room) + " (raise band_halo or lower dt)";
            return EFT_EBAND_OVERFLOW;
        }
    }
    for (int k = 0; k < K; ++k) {
        inf.band_nodes[k] = ctx->band[k].n;
        inf.band_elems[k] = ctx->band[k].ne;
        inf.gamma[k] = gb[2 * k];
        inf.beta[k] = gb[2 * k + 1];
    }
    // every Allen-Cahn system, one batched solve
    if (K > 0 && ctx->u_ac.n > 0) {
        const eft_ctx::BandUnion &U = ctx->u_ac;
        EFT_TRY(assemble_all(ctx, lvl, it, 0));
        std::vector<double *> x(K);
        std::vector<int64_t> xl(K, N);
        for (int k = 0; k < K; ++k) x[k] = it->phi + (int64_t)k * N;
        eft_solve_info si{};
        eft_status st = union_solve(ctx, U, 1, x, xl, inf.ratio, &si);
        if (st != EFT_OK && st != EFT_ENOTCONV) return st;
        if (st == EFT_ENOTCONV) worst = st;
        inf.ac_iters = si.iters;
        for (int k = 0; k < K; ++k) inf.lin_iters[k] = ctx->band[k].n > 0 ? si.iters : 0;
    }
    // every B system (solid fractions from the new phi, evaluated by the
    // assembly), one batched solve
    if (S > 0 && ctx->u_b.n > 0) {
        const eft_ctx::BandUnion &U = ctx->u_b;
        EFT_TRY(assemble_all(ctx, lvl, it, 1));
        std::vector<double *> x(S);
        std::vector<int64_t> xl(S, N * nv);
        for (int sI = 0; sI < S; ++sI) x[sI] = it->B + (int64_t)sI * N * nv;
        eft_solve_info si{};
        eft_status st = union_solve(ctx, U, nv, x, xl, inf.ratio + K, &si);
        if (st != EFT_OK && st != EFT_ENOTCONV) return st;
        if (st == EFT_ENOTCONV) worst = st;
        inf.b_iters = si.iters;
        for (int sI = 0; sI < S; ++sI) inf.lin_iters[K + sI] = ctx->band[ctx->solid_ind[sI]].n > 0 ? si.iters : 0;
    }
    if (info) *info = inf;
    return worst;
}

// Assemble one band system at the iterate and copy it out (test hook).
eft_status eft_band_system_dev(eft_ctx *ctx, const eft_state *lvl, const eft_iterate *it, int kind, int index,
                               int64_t *n, int64_t *nnz, int32_t *node, int32_t *rowptr, int32_t *col, double *R,
                               double *J, double *gamma_beta)
{
    if (!ctx->bands_valid) {
        ctx->err = "eft_bands_build must run first";
        return EFT_EINVAL;
    }
    if ((kind == 0 && (index < 0 || index >= ctx->n_ind)) || (kind == 1 && (index < 0 || index >= ctx->n_s)) ||
        (kind != 0 && kind != 1)) {
        ctx->err = "band system: bad kind/index";
        return EFT_EINVAL;
    }
    const int bs = kind == 0 ? 1 : ctx->nv;
    const Band &B = ctx->band[kind == 0 ? index : ctx->solid_ind[index]];
    if (n) *n = B.n;
    if (nnz) *nnz = B.nnz;
    if (!node && !rowptr && !col && !R && !J) return EFT_OK;
    EFT_TRY(eft_props(ctx, lvl, it));
    double gb[2] = {0.0, 0.0};
    if (kind == 0) {
        std::vector<double> all(2 * ctx->n_ind);
        EFT_TRY(mobility_beta_all(ctx, lvl, it, all.data()));
        gb[0] = all[2 * index];
        gb[1] = all[2 * index + 1];
        EFT_TRY(assemble_ac(ctx, lvl, it, index, ctx->bR, ctx->bval, ctx->tsc + TS_GB + 2 * index));
    } else if (J) {   // every block in full, straight into the caller's buffer
        EFT_TRY(assemble_b(ctx, lvl, it, index, ctx->bR, J, ctx->bcmp, true, nullptr));
    } else {
        EFT_TRY(assemble_b(ctx, lvl, it, index, ctx->bR, nullptr, ctx->bcmp, false, ctx->bdiag));
    }
    if (gamma_beta) {
        gamma_beta[0] = gb[0];
        gamma_beta[1] = gb[1];
    }
    if (node) EFT_HIP(hipMemcpyAsync(node, B.node, sizeof(int32_t) * B.n, hipMemcpyDeviceToDevice, ctx->stream));
    if (rowptr) EFT_HIP(hipMemcpyAsync(rowptr, B.rowptr, sizeof(int32_t) * (B.n + 1), hipMemcpyDeviceToDevice, ctx->stream));
    if (col) EFT_HIP(hipMemcpyAsync(col, B.col, sizeof(int32_t) * B.nnz, hipMemcpyDeviceToDevice, ctx->stream));
    if (R) EFT_HIP(hipMemcpyAsync(R, ctx->bR, sizeof(double) * B.n * bs, hipMemcpyDeviceToDevice, ctx->stream));
    if (J && kind == 0) EFT_HIP(hipMemcpyAsync(J, ctx->bval, sizeof(double) * B.nnz, hipMemcpyDeviceToDevice, ctx->stream));
    EFT_HIP(hipStreamSynchronize(ctx->stream));
    return EFT_OK;
}
