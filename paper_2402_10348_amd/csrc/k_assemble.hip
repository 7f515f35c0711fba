// Element assembly of the unified momentum/mass system, eq. (PG_NS).
//
// Two kernels:
//   k_props    per node: generalized-alpha level values (Sec. 2.1.2),
//              phase-interpolated rho, mu (Sec. 2.1.1) and the mask of the
//              solids present;
//   k_ns_rows  row-owned assembly: a workgroup owns a set of consecutive block
//              rows; each (row, incident element) pair evaluates the element
//              at its quadrature points (Galerkin + SUPG/PSPG/LSIC with the
//              tau_m, tau_c formula and the Newtonian stress) and adds only
//              that row's residual and blocks into LDS accumulators; the
//              left-Cauchy-Green stress mu_L (B - I) of the solids present on
//              the element and its tangent through dB/dv (eq. (Bext) /
//              Appendix B) are queued per (pair, solid) and evaluated after
//              the fluid pass by all threads; the rows are written out once,
//              contiguously (no global atomics), with the unit rows of
//              Dirichlet dofs.
// The quadrature sums are factored: the sums over the points that do not
// depend on the row are shared by the row's residual and its blocks, so a
// 4x4 block costs a few dozen flops.
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
    double *va, *acc, *rho, *mu;
    uint64_t *smask;            // [N] bit s set where solid s has a non-zero fraction
};

// Fraction of the phase of an order parameter at n+alpha (reading 2: nodal
// clamp of (1 + phi)/2), from phi^n and the iterate.  Every kernel that needs
// a solid fraction evaluates this same expression, so they agree bit for bit.
__device__ __forceinline__ double phase_fraction(double fn, double f1, double alpha)
{
    const double fa = fn + alpha * (f1 - fn);
    return fmin(fmax(0.5 * (1.0 + fa), 0.0), 1.0);
}

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
    uint64_t sm = 0;
    for (int s = 0; s < a.n_s; ++s) {
        const int k = a.solid_ind[s];
        const double al = phase_fraction(a.l_phi[(int64_t)k * a.N + p], a.it_phi[(int64_t)k * a.N + p], a.alpha);
        if (al != 0.0) sm |= (uint64_t)1 << s;
    }
    a.smask[p] = sm;
    (void)NVv;
}

// ------------------------------------------------------ row-owned kernel --

// One workgroup owns a block of consecutive matrix rows.  Every (row node,
// incident element) pair is one thread: it evaluates the element (geometry,
// quadrature-point state, tau_m and tau_c) and adds that element's share of
// the row -- the residual of the row node and the blocks coupling it to the
// element's nodes -- into LDS accumulators.  Each element is thus evaluated
// once per node (4 times in 3D) instead of scattering 16 blocks with global
// atomics; the finished rows are written once, contiguously.  When the mesh
// allows it (at most 256 nodes per workgroup), the records of the nodes the
// workgroup's elements touch and its incidence words are first staged in LDS,
// so the pair loop makes no global loads.
struct RowArgs {
    int64_t N;                   // rows (nodes)
    int rpb, maxc;               // rows per workgroup, longest row (LDS layout)
    const int32_t *iptr, *ient;  // node -> incident (element << 2 | local node)
    const uint32_t *islot;       // per incidence entry: byte k = block slot, in the row, of local node (a + k) mod nn
    const int32_t *conn, *epos, *rowptr;
    const double *xyz, *va, *acc, *vp, *rho, *mu;
    int n_s;
    const double *as, *Ba, *muL;   // per-solid fraction and B at n+alpha ([n_s][N], [n_s][N][nv]), or null:
    const uint64_t *smask;         // [N] solids present at each node
    // with as = null the fractions and B at n+alpha of the present solids are
    // evaluated from phi^n, phi, B^n, B (solid s: order parameter solid_ind[s])
    const double *lphi, *iphi, *lB, *iB;
    const int32_t *solid_ind;
    double ct, alpha, kappa, dt, C_I, g0, g1, g2;
    double *R;
    float *J32;      // optional FP32 copy of the values
    uint16_t *J16;   // optional BF16 copy of the values
    const int32_t *col;      // block columns of the pattern
    const uint8_t *fmask;    // [N] free-dof bits: a Dirichlet dof's row is written as a unit row, residual 0
    // staged node records (or null): per workgroup its nodes wnode[wnptr[w] ..
    // wnptr[w + 1]) and per incidence entry the positions of the element's
    // nodes in that list (byte b: node (a + b) mod nn)
    const int32_t *wnptr, *wnode;
    const uint32_t *iloc;
    int maxnl, maxpw;        // most nodes, most incidence entries of a workgroup
};

// Staged node record in LDS: x, v and a at n+alpha, p, rho, mu, the solid
// mask (bits); an odd stride in doubles
template <int D> struct NodeRec {
    static constexpr int n = (3 * D + 4) | 1;
};

// Elastic stress mu_L (B - I) of solid sI on the element of one (row,
// element) pair (residual, added to rl), and its tangent through dB/dv, eq.
// (Bext), added to the row's blocks in LDS: with F = int alpha mu_L,
// W_b = int N_b alpha mu_L, M = int alpha mu_L B and D_k = (dB/dx_k) grad N_a,
// the residual gains (M - F I) grad N_a and block (a, b) gains
//   alpha kappa (-W_b D_k[i] + dN_a[k] (M grad N_b)_i + delta_ik grad N_a . M grad N_b).
// nd, dN: the element's nodes and shape gradients with the row node first;
// sl: the row's block slots of the element's nodes (same order).
constexpr int EQ_CAP = 2048;   // queued elastic (pair, solid) items per workgroup

template <int D>
__device__ __forceinline__ void elastic_pair(const RowArgs &a, const int (&nd)[D + 1], const double (&dN)[D + 1][D],
                                             double w, uint32_t sl, int lr, int sI, bool withJ, double *rl,
                                             double *accJ)
{
    constexpr int NN = D + 1, BS = D + 1, NQ = Rule<D>::NQ, NVv = NV<D>::v, BP = (BS * BS) | 1;
    constexpr double QA = Rule<D>::QA, QB = Rule<D>::QB, QD = QA - QB;
    const double(&da)[D] = dN[0];
    double asn[NN];
    double Bn[NN][NVv];
    if (a.as) {
#pragma unroll
        for (int b = 0; b < NN; ++b) {
            asn[b] = a.as[(int64_t)sI * a.N + nd[b]];
#pragma unroll
            for (int c = 0; c < NVv; ++c) Bn[b][c] = a.Ba[((int64_t)sI * a.N + nd[b]) * NVv + c];
        }
    } else {
        const int64_t ko = (int64_t)a.solid_ind[sI] * a.N;
#pragma unroll
        for (int b = 0; b < NN; ++b) {
            asn[b] = phase_fraction(a.lphi[ko + nd[b]], a.iphi[ko + nd[b]], a.alpha);
#pragma unroll
            for (int c = 0; c < NVv; ++c) {
                const int64_t o = ((int64_t)sI * a.N + nd[b]) * NVv + c;
                Bn[b][c] = a.lB[o] + a.alpha * (a.iB[o] - a.lB[o]);
            }
        }
    }
    const double muL = a.muL[sI];
    double sa = 0.0, sb[NVv];
#pragma unroll
    for (int c = 0; c < NVv; ++c) sb[c] = 0.0;
#pragma unroll
    for (int b = 0; b < NN; ++b) {
        sa += asn[b];
#pragma unroll
        for (int c = 0; c < NVv; ++c) sb[c] += Bn[b][c];
    }
    // Md = int alpha mu_L (B - I) (B - I formed before the product, as
    // mu_L may be large and B close to I), M = Md + F I
    double F = 0.0, Wbs[NN], Mv[NVv];
#pragma unroll
    for (int b = 0; b < NN; ++b) Wbs[b] = 0.0;
#pragma unroll
    for (int c = 0; c < NVv; ++c) Mv[c] = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double wf = w * (QB * sa + QD * asn[q]) * muL;
        F += wf;
#pragma unroll
        for (int b = 0; b < NN; ++b) Wbs[b] += wf * (b == q ? QA : QB);
#pragma unroll
        for (int c = 0; c < NVv; ++c) Mv[c] += wf * (QB * sb[c] + QD * Bn[q][c] - (c < D ? 1.0 : 0.0));
    }
    double M2[D][D];
    vfull<D>(Mv, M2);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double s2 = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) s2 += M2[i][j] * da[j];
        rl[i] += s2;
    }
    if (!withJ) return;
#pragma unroll
    for (int i = 0; i < D; ++i) M2[i][i] += F;
    double Dk[D][D];   // Dk[i][k] = ((dB/dx_k) grad N_a)_i
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
        double gf[D][D];
        vfull<D>(gk, gf);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double t = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) t += gf[i][j] * da[j];
            Dk[i][k] = t;
        }
    }
    const double ak = a.alpha * a.kappa;
#pragma unroll
    for (int ib = 0; ib < NN; ++ib) {
        const int slot = (sl >> (8 * ib)) & 0xff;
        double *blk = accJ + ((int64_t)lr * a.maxc + slot) * BP;
        double Mb[D], aMb = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double s2 = 0.0;
#pragma unroll
            for (int l = 0; l < D; ++l) s2 += M2[i][l] * dN[ib][l];
            Mb[i] = s2;
            aMb += da[i] * s2;
        }
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int k = 0; k < D; ++k)
                atomicAdd(blk + i * BS + k,
                          ak * (-Wbs[ib] * Dk[i][k] + da[k] * Mb[i] + (i == k ? aMb : 0.0)));
    }
}

// 1/x and 1/sqrt(x) for x > 0 from the hardware approximations refined by two
// Newton steps each (each step roughly doubles the correct bits: from the
// approximation's about 22 to beyond double precision), instead of the
// correctly rounded division and square root sequences: the results differ
// from those by an ulp or two
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-0.5 * x * y, y, 0.5);
    y = fma(y, e, y);
    e = fma(-0.5 * x * y, y, 0.5);
    return fma(y, e, y);
}

template <int D, typename TJ, bool ST>
__global__ __launch_bounds__(256, 2) void k_ns_rows(RowArgs a, TJ *__restrict__ Jv)
{
    extern __shared__ double lds[];
    constexpr int NN = D + 1, BS = D + 1, B2 = BS * BS, NQ = Rule<D>::NQ, NVv = NV<D>::v;
    // LDS strides padded to an odd number of doubles: with 4x4 blocks at a
    // 128-byte stride, entry (i, k) of every block would sit in one bank and
    // each atomic instruction would serialize over the wavefront
    constexpr int BP = B2 | 1, RP = BS | 1;
    const int64_t r0 = (int64_t)blockIdx.x * a.rpb;
    const int64_t r1 = r0 + a.rpb < a.N ? r0 + a.rpb : a.N;
    double *accJ = lds;                                 // [rpb][maxc][BP]
    double *accR = lds + (int64_t)a.rpb * a.maxc * BP;  // [rpb][RP]
    const int nacc = a.rpb * a.maxc * BP + a.rpb * RP;
    // the rows' incidence and block ranges, free-dof bits and, per block of
    // the workgroup's (contiguous) block range, its row
    int *istart = reinterpret_cast<int *>(lds + nacc);      // [rpb + 1]
    int *rstart = istart + (a.rpb + 1);                      // [rpb + 1]
    uint16_t *blkrow = reinterpret_cast<uint16_t *>(rstart + (a.rpb + 1));   // [rpb * maxc]
    uint8_t *fml = reinterpret_cast<uint8_t *>(blkrow + a.rpb * a.maxc);     // [rpb]
    // staged: the workgroup's node records, node ids and incidence words
    constexpr int NR = NodeRec<D>::n;
    double *ndat = lds + nacc + ((2 * (a.rpb + 1) * 4 + a.rpb * a.maxc * 2 + a.rpb + 7) / 8);   // [maxnl][NR]
    int *nid = reinterpret_cast<int *>(ndat + (ST ? a.maxnl * NR : 0));                     // [maxnl]
    uint32_t *pw = reinterpret_cast<uint32_t *>(nid + (ST ? a.maxnl : 0));                 // [maxpw][2]
    uint8_t *pla = reinterpret_cast<uint8_t *>(pw + (ST ? 2 * a.maxpw : 0));              // [maxpw]
    __shared__ int maxinc, eq_n;
    __shared__ uint32_t eq[EQ_CAP];   // queued (pair << 6 | solid) elastic work
    if (threadIdx.x == 0) maxinc = eq_n = 0;
    for (int t = threadIdx.x; t < nacc; t += blockDim.x) lds[t] = 0.0;
    const int nrow = (int)(r1 - r0);
    if (threadIdx.x <= nrow) {
        istart[threadIdx.x] = a.iptr[r0 + threadIdx.x];
        rstart[threadIdx.x] = a.rowptr[r0 + threadIdx.x];
    }
    if (threadIdx.x < nrow) fml[threadIdx.x] = a.fmask[r0 + threadIdx.x];
    if constexpr (ST) {
        // the records of every node the rows' elements touch, read once
        const int w0 = a.wnptr[blockIdx.x], nl = a.wnptr[blockIdx.x + 1] - w0;
        for (int t = threadIdx.x; t < nl; t += blockDim.x) {
            const int64_t n = a.wnode[w0 + t];
            double *rec = ndat + t * NR;
            nid[t] = (int)n;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                rec[i] = a.xyz[n * D + i];
                rec[D + i] = a.va[n * D + i];
                rec[2 * D + i] = a.acc[n * D + i];
            }
            rec[3 * D] = a.vp[n * BS + D];
            rec[3 * D + 1] = a.rho[n];
            rec[3 * D + 2] = a.mu[n];
            rec[3 * D + 3] = __longlong_as_double((long long)a.smask[n]);
        }
    }
    __syncthreads();
    if (threadIdx.x < nrow) {
        atomicMax(&maxinc, istart[threadIdx.x + 1] - istart[threadIdx.x]);
        for (int k = rstart[threadIdx.x]; k < rstart[threadIdx.x + 1]; ++k) blkrow[k - rstart[0]] = threadIdx.x;
    }
    if constexpr (ST) {
        const int i0 = istart[0], npw = istart[nrow] - i0;
        for (int t = threadIdx.x; t < npw; t += blockDim.x) {
            pw[2 * t] = a.iloc[i0 + t];
            pw[2 * t + 1] = a.islot[i0 + t];
            pla[t] = (uint8_t)(a.ient[i0 + t] & 3);
        }
    }
    __syncthreads();
    const double gv[3] = {a.g0, a.g1, a.g2};
    // (row, incident element) pairs are dealt row-interleaved: consecutive
    // lanes take different rows, so the LDS atomics of one wavefront rarely
    // hit the same block (all elements of a row add into its diagonal block)
    for (int k = threadIdx.x; k < nrow * maxinc; k += blockDim.x) {
        const int kr = k % nrow;
        const int ii = istart[kr] + k / nrow;
        if (ii >= istart[kr + 1]) continue;
        // the element's nodes rotated so that the row node comes first (local
        // node b is node (la + b) mod NN of the connectivity): every index
        // below is then a compile-time constant
        int nd[NN], la;
        uint32_t sl, lw = 0;
        double X[NN][D], v[NN][D], ac[NN][D], p[NN], rh[NN], mu[NN];
        uint64_t present = 0;   // solids present on the element
        if constexpr (ST) {
            // (the staged path keeps only the positions and reads the other
            // node values from LDS where it uses them)
            const int j = ii - istart[0];
            lw = pw[2 * j];
            sl = pw[2 * j + 1];
            la = pla[j];
#pragma unroll
            for (int b = 0; b < NN; ++b) {
                const int lb = (lw >> (8 * b)) & 0xff;
                const double *rec = ndat + lb * NR;
                nd[b] = nid[lb];
#pragma unroll
                for (int i = 0; i < D; ++i) X[b][i] = rec[i];
                present |= (uint64_t)__double_as_longlong(rec[3 * D + 3]);
            }
        } else {
            const int32_t ent = a.ient[ii];
            sl = a.islot[ii];
            const int64_t e = ent >> 2;
            la = ent & 3;
#pragma unroll
            for (int b = 0; b < NN; ++b) nd[b] = a.conn[e * NN + (la + b < NN ? la + b : la + b - NN)];
#pragma unroll
            for (int b = 0; b < NN; ++b) {
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
        }
        const int64_t row = nd[0];
        const int lr = (int)(row - r0);
        double dN[NN][D], G[D][D];
        const double vol = simplex_geom<D>(X, dN, G);
        // G = J^-T J^-1 belongs to the reference map with its origin at the
        // element's first node in the connectivity (it is not invariant under
        // a relabelling of the nodes): rebuild it as the sum of grad N grad N^T
        // over the other nodes; the rotation moved that node to local o0
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
        double GG = 0.0, trG = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            trG += G[i][i];
#pragma unroll
            for (int j = 0; j < D; ++j) GG += G[i][j] * G[i][j];
        }
        double L[D][D], gp[D], divv = 0.0;
        // staged: the node sums of rho, mu, p, v and a, with which a point
        // value is QB * sum + (QA - QB) * (value at the point's node)
        double Srh = 0.0, Smu = 0.0, Sp = 0.0, Sv[D], Sac[D];
        if constexpr (ST) {
#pragma unroll
            for (int i = 0; i < D; ++i) {
                Sv[i] = Sac[i] = gp[i] = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) L[i][j] = 0.0;
            }
#pragma unroll
            for (int b = 0; b < NN; ++b) {
                const double *rec = ndat + ((lw >> (8 * b)) & 0xff) * NR;
                const double pb = rec[3 * D];
                Sp += pb;
                Srh += rec[3 * D + 1];
                Smu += rec[3 * D + 2];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const double vb = rec[D + i];
                    Sv[i] += vb;
                    Sac[i] += rec[2 * D + i];
                    gp[i] += pb * dN[b][i];
#pragma unroll
                    for (int j = 0; j < D; ++j) L[i][j] += vb * dN[b][j];
                }
            }
        } else {
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
        }
#pragma unroll
        for (int i = 0; i < D; ++i) divv += L[i][i];
        const double(&da)[D] = dN[0];   // grad N of the row node
        const double w = vol * Rule<D>::WF;
        const double inv4dt2 = 4.0 / (a.dt * a.dt), rtrG = rcp_nr(trG);
        constexpr double QA = Rule<D>::QA, QB = Rule<D>::QB, QD = QA - QB;
        // Quadrature sums.  Element-level (the same for every row):
        //   P = int p, MU = int mu, Tc = int tau_c rho, Tp = int tau_m / rho,
        //   U = int tau_m v, Q2_b = int tau_m N_b;
        // row-level, with W_a = rho (N_a + tau_m u_a), u_a = v . grad N_a:
        //   Cs_b = int W_a N_b, V = int W_a v, Pa = int tau_m u_a and the residual.
        // The tangent sums of the unfactored form follow from them:
        //   int W_a (c_t N_b + alpha u_b) = c_t Cs_b + alpha V . grad N_b,
        //   int tau_m (c_t N_b + alpha u_b) = c_t Q2_b + alpha U . grad N_b.
        double P = 0.0, MU = 0.0, Tc = 0.0, Tp = 0.0, U[D], Q2s[NN], Cs[NN], V[D], Pa = 0.0, rl[BS];
#pragma unroll
        for (int i = 0; i < D; ++i) U[i] = V[i] = 0.0;
#pragma unroll
        for (int b = 0; b < NN; ++b) Q2s[b] = Cs[b] = 0.0;
#pragma unroll
        for (int i = 0; i < BS; ++i) rl[i] = 0.0;
        // not unrolled: one point's temporaries at a time keep the register
        // count (and so the occupancy) in check; q is uniform, so N_b(q) is a
        // scalar select
#pragma unroll 1
        for (int q = 0; q < NQ; ++q) {
            double rq = 0.0, mq = 0.0, pq = 0.0, vq[D], aq[D];
            if constexpr (ST) {
                const double *rec = ndat + ((lw >> (8 * q)) & 0xff) * NR;
                pq = QB * Sp + QD * rec[3 * D];
                rq = QB * Srh + QD * rec[3 * D + 1];
                mq = QB * Smu + QD * rec[3 * D + 2];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    vq[i] = QB * Sv[i] + QD * rec[D + i];
                    aq[i] = QB * Sac[i] + QD * rec[2 * D + i];
                }
            } else {
#pragma unroll
                for (int i = 0; i < D; ++i) vq[i] = aq[i] = 0.0;
#pragma unroll
                for (int b = 0; b < NN; ++b) {
                    const double Nb = b == q ? QA : QB;
                    rq += Nb * rh[b];
                    mq += Nb * mu[b];
                    pq += Nb * p[b];
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        vq[i] += Nb * v[b][i];
                        aq[i] += Nb * ac[b][i];
                    }
                }
            }
            double Rm[D], body[D], vGv = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                double s = 0.0, t = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    s += L[i][j] * vq[j];
                    t += G[i][j] * vq[j];
                }
                vGv += vq[i] * t;
                body[i] = aq[i] + s - gv[i];
                Rm[i] = rq * body[i] + gp[i];
            }
            const double ri = rcp_nr(rq), nu = mq * ri;
            const double Xq = inv4dt2 + vGv + a.C_I * nu * nu * GG;
            const double tau_m = rsqrt_nr(Xq), sq = Xq * tau_m, tau_c = sq * rtrG, TMq = w * tau_m;
            P += w * pq;
            MU += w * mq;
            Tc += w * tau_c * rq;
            Tp += TMq * ri;
#pragma unroll
            for (int i = 0; i < D; ++i) U[i] += TMq * vq[i];
#pragma unroll
            for (int b = 0; b < NN; ++b) Q2s[b] += TMq * (b == q ? QA : QB);
            // the row node's share
            const double Na = q == 0 ? QA : QB;
            double ua = 0.0, gR = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                ua += vq[j] * da[j];
                gR += da[j] * Rm[j];
            }
            const double tu = tau_m * ua, wNr = w * Na * rq;
#pragma unroll
            for (int i = 0; i < D; ++i) rl[i] += wNr * body[i] + w * tu * Rm[i];
            rl[D] += TMq * ri * gR;
            const double Wq = w * rq * (Na + tu);
#pragma unroll
            for (int b = 0; b < NN; ++b) Cs[b] += Wq * (b == q ? QA : QB);
#pragma unroll
            for (int i = 0; i < D; ++i) V[i] += Wq * vq[i];
            Pa += TMq * ua;
        }
        const double NI = w * (Rule<D>::QA + (NQ - 1) * Rule<D>::QB);   // int N_a
        // Galerkin pressure / viscous / LSIC terms of the residual, from the element sums
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) s += (L[i][j] + L[j][i]) * da[j];
            rl[i] += MU * s + (Tc * divv - P) * da[i];
        }
        rl[D] += NI * divv;
        // fluid (and pressure) blocks of the row: d(residual of the row node)/d(local node ib)
        if (Jv != nullptr) {
            const double al = a.alpha;
            double aL[D];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) s += da[j] * L[j][k];
                aL[k] = s;
            }
#pragma unroll
            for (int ib = 0; ib < NN; ++ib) {
                const double(&db)[D] = dN[ib];
                double gab = 0.0, Vb = 0.0, Ub = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    gab += da[j] * db[j];
                    Vb += V[j] * db[j];
                    Ub += U[j] * db[j];
                }
                const double Csb = Cs[ib], Q2 = Q2s[ib];
                const double A = a.ct * Csb + al * Vb, C = al * Csb, Q1 = a.ct * Q2 + al * Ub;
                const int slot = (sl >> (8 * ib)) & 0xff;
                double *blk = accJ + ((int64_t)lr * a.maxc + slot) * BP;
#pragma unroll
                for (int i = 0; i < D; ++i) {
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        double val = C * L[i][k] + al * MU * da[k] * db[i] + al * Tc * da[i] * db[k];
                        if (i == k) val += A + al * MU * gab;
                        atomicAdd(blk + i * BS + k, val);
                    }
                    atomicAdd(blk + i * BS + D, -da[i] * NI + Pa * db[i]);
                }
#pragma unroll
                for (int k = 0; k < D; ++k)
                    atomicAdd(blk + D * BS + k, al * db[k] * NI + da[k] * Q1 + al * aL[k] * Q2);
                atomicAdd(blk + D * BS + D, Tp * gab);
            }
        }
        // elastic stress of the solids present on the element: queued per
        // (pair, solid) for the dense pass below (a wavefront would otherwise
        // run the solid body for a few of its lanes), inline when the queue
        // is full
        if (a.n_s > 0) {
            if constexpr (!ST) {
#pragma unroll
                for (int b = 0; b < NN; ++b) present |= a.smask[nd[b]];
            }
            while (present) {   // in increasing solid order
                const int sI = __ffsll((unsigned long long)present) - 1;
                present &= present - 1;
                const int slot = atomicAdd(&eq_n, 1);
                if (slot < EQ_CAP) eq[slot] = ((uint32_t)k << 6) | (uint32_t)sI;
                else elastic_pair<D>(a, nd, dN, w, sl, lr, sI, Jv != nullptr, rl, accJ);
            }
        }
        // residual of the row node
#pragma unroll
        for (int i = 0; i < BS; ++i) atomicAdd(accR + lr * RP + i, rl[i]);
    }
    __syncthreads();
    // the queued elastic work, one (pair, solid) per thread
    const int nq = eq_n < EQ_CAP ? eq_n : EQ_CAP;
    for (int t = threadIdx.x; t < nq; t += blockDim.x) {
        const uint32_t item = eq[t];
        const int k = (int)(item >> 6), sI = (int)(item & 63);
        const int kr = k % nrow;
        const int ii = istart[kr] + k / nrow;
        int nd[NN];
        uint32_t sl;
        double X[NN][D];
        if constexpr (ST) {
            const int j = ii - istart[0];
            const uint32_t lw = pw[2 * j];
            sl = pw[2 * j + 1];
#pragma unroll
            for (int b = 0; b < NN; ++b) {
                const int lb = (lw >> (8 * b)) & 0xff;
                nd[b] = nid[lb];
#pragma unroll
                for (int i = 0; i < D; ++i) X[b][i] = ndat[lb * NR + i];
            }
        } else {
            const int32_t ent = a.ient[ii];
            sl = a.islot[ii];
            const int64_t e = ent >> 2;
            const int la = ent & 3;
#pragma unroll
            for (int b = 0; b < NN; ++b) {
                nd[b] = a.conn[e * NN + (la + b < NN ? la + b : la + b - NN)];
#pragma unroll
                for (int i = 0; i < D; ++i) X[b][i] = a.xyz[(int64_t)nd[b] * D + i];
            }
        }
        double dN[NN][D], G[D][D];
        const double w = simplex_geom<D>(X, dN, G) * Rule<D>::WF;
        double rl[D];
#pragma unroll
        for (int i = 0; i < D; ++i) rl[i] = 0.0;
        const int lr = (int)(nd[0] - r0);
        elastic_pair<D>(a, nd, dN, w, sl, lr, sI, Jv != nullptr, rl, accJ);
#pragma unroll
        for (int i = 0; i < D; ++i) atomicAdd(accR + lr * RP + i, rl[i]);
    }
    __syncthreads();
    // write-out, flat over the workgroup's rows: R, then the values of its
    // contiguous block range (coalesced), Dirichlet dofs as unit rows
    for (int t = threadIdx.x; t < nrow * BS; t += blockDim.x) {
        const int lr = t / BS, i = t - lr * BS;
        a.R[r0 * BS + t] = ((fml[lr] >> i) & 1) ? accR[lr * RP + i] : 0.0;
    }
    if (Jv == nullptr) return;
    const int kb0 = rstart[0];
    const int nval = (rstart[nrow] - kb0) * B2;
    for (int t = threadIdx.x; t < nval; t += blockDim.x) {
        const int kk = t / B2, e = t - kk * B2;
        const int lr = blkrow[kk];
        double v = accJ[((int64_t)lr * a.maxc + (kk - (rstart[lr] - kb0))) * BP + e];
        if (!((fml[lr] >> (e / BS)) & 1)) v = (a.col[kb0 + kk] == r0 + lr && e % (BS + 1) == 0) ? 1.0 : 0.0;
        const int64_t o = (int64_t)kb0 * B2 + t;
        Jv[o] = (TJ)v;
        if (a.J32) a.J32[o] = (float)v;
        if (a.J16) a.J16[o] = to_bf16_rne((float)v);
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

// ------------------------------------------------------ staged records --

// Node records staged per momentum-assembly workgroup (rows [w rpb, (w + 1)
// rpb)): the sorted nodes of the elements incident to its rows, and per
// incidence entry (element e, local node a) the positions in that list of
// nodes (a + b) mod nn, one byte each.  Returns false, with the outputs
// cleared, when a workgroup touches more than 256 nodes (the assembly then
// reads the node fields from the global arrays).
bool eft_ns_stage_build(int64_t N, int nn, const int32_t *conn, const std::vector<int32_t> &iptr,
                        const std::vector<int32_t> &ient, int rpb, std::vector<int32_t> &wnptr,
                        std::vector<int32_t> &wnode, std::vector<uint32_t> &iloc, int &maxnl, int &maxpw)
{
    const int64_t nw = (N + rpb - 1) / rpb;
    wnptr.assign(nw + 1, 0);
    wnode.clear();
    iloc.assign(ient.size(), 0);
    maxnl = maxpw = 0;
    std::vector<int64_t> seen(N, -1);   // workgroup that last listed the node
    std::vector<int32_t> pos(N, 0);     // its position in that list
    std::vector<int32_t> buf;
    for (int64_t w = 0; w < nw; ++w) {
        const int64_t r0 = w * rpb, r1 = std::min<int64_t>(N, r0 + rpb);
        buf.clear();
        for (int64_t t = iptr[r0]; t < iptr[r1]; ++t) {
            const int64_t e = ient[t] >> 2;
            for (int b = 0; b < nn; ++b) {
                const int32_t n = conn[e * nn + b];
                if (seen[n] != w) {
                    seen[n] = w;
                    buf.push_back(n);
                }
            }
        }
        if (buf.size() > 256) {
            wnptr.clear();
            wnode.clear();
            iloc.clear();
            maxnl = maxpw = 0;
            return false;
        }
        std::sort(buf.begin(), buf.end());
        for (size_t i = 0; i < buf.size(); ++i) pos[buf[i]] = (int32_t)i;
        for (int64_t t = iptr[r0]; t < iptr[r1]; ++t) {
            const int64_t e = ient[t] >> 2;
            const int a = ient[t] & 3;
            uint32_t word = 0;
            for (int b = 0; b < nn; ++b) word |= (uint32_t)pos[conn[e * nn + (a + b) % nn]] << (8 * b);
            iloc[t] = word;
        }
        wnode.insert(wnode.end(), buf.begin(), buf.end());
        wnptr[w + 1] = (int32_t)wnode.size();
        maxnl = std::max(maxnl, (int)buf.size());
        maxpw = std::max(maxpw, (int)(iptr[r1] - iptr[r0]));
    }
    return true;
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
    a.l_vp = lvl->vp;
    a.l_vdot = lvl->vdot;
    a.it_vp = it->vp;
    a.l_phi = lvl->phi;
    a.it_phi = it->phi;
    a.va = ctx->va;
    a.acc = ctx->acc;
    a.rho = ctx->rho;
    a.mu = ctx->mu;
    a.smask = ctx->smask;
    a.solid_ind = ctx->solid_ind_d;
    ctx->src_lphi = lvl->phi;
    ctx->src_iphi = it->phi;
    ctx->src_lB = lvl->B;
    ctx->src_iB = it->B;
    const int nb = eft_grid(ctx->N, 256);
    if (ctx->dim == 2)
        hipLaunchKernelGGL(k_props<2>, dim3(nb), dim3(256), 0, ctx->stream, a);
    else
        hipLaunchKernelGGL(k_props<3>, dim3(nb), dim3(256), 0, ctx->stream, a);
    EFT_HIP(hipGetLastError());
    return EFT_OK;
}


// Residual and Jacobian of the momentum/mass block at the iterate (the
// node fields va, acc, rho, mu and the solid mask must be current, see eft_props).
// Residual and Jacobian of the momentum/mass block on one mesh level (the
// node fields of the view must be current).
eft_status eft_ns_level(eft_ctx *ctx, const MeshView &M, const double *vp, double *R, eft_matrix *J, float *J32,
                        uint16_t *J16)
{
    GA ga = ga_of(ctx->par.rho_inf, ctx->par.dt);
    const int BS = ctx->bs;
    GA gq = ga;
    RowArgs a;
    a.N = M.N;
    a.rpb = M.rpb;
    a.maxc = M.maxc;
    a.iptr = M.iptr;
    a.ient = M.ient;
    a.islot = M.islot;
    a.conn = M.conn;
    a.epos = M.epos;
    a.rowptr = J ? J->rowptr : nullptr;
    a.col = J ? J->col : nullptr;
    a.fmask = M.fmask;
    a.wnptr = M.wnptr;
    a.wnode = M.wnode;
    a.iloc = M.iloc;
    a.maxnl = M.maxnl;
    a.maxpw = M.maxpw;
    const bool st = M.iloc != nullptr;
    if (!M.fmask) {
        ctx->err = "assembly without the free-dof mask";
        return EFT_EINVAL;
    }
    a.xyz = M.xyz;
    a.va = M.va;
    a.acc = M.acc;
    a.vp = vp;
    a.rho = M.rho;
    a.mu = M.mu;
    a.n_s = ctx->n_s;
    a.as = M.as;
    a.Ba = M.Ba;
    a.smask = M.smask;
    a.lphi = ctx->src_lphi;
    a.iphi = ctx->src_iphi;
    a.lB = ctx->src_lB;
    a.iB = ctx->src_iB;
    a.solid_ind = ctx->solid_ind_d;
    a.muL = ctx->phase_tab + 5 * EFT_MAX_PHASE;  // mu_L of each solid
    a.ct = gq.ct;
    a.alpha = gq.alpha;
    a.kappa = gq.kappa;
    a.dt = gq.dt;
    a.C_I = ctx->par.C_I;
    a.g0 = ctx->g[0];
    a.g1 = ctx->g[1];
    a.g2 = ctx->g[2];
    a.R = R;
    a.J32 = (J && !J->fp32) ? J32 : nullptr;
    a.J16 = J ? J16 : nullptr;
    if (!J) {
        // residual only: one row of accumulators suffices for the pattern-free path
        a.rowptr = ctx->J.rowptr;
    }
    const int nb = eft_grid(M.N, M.rpb);
    const size_t nrec = ctx->dim == 2 ? NodeRec<2>::n : NodeRec<3>::n;
    const size_t meta = ((size_t)(M.rpb + 1) * 2 * sizeof(int) + (size_t)M.rpb * M.maxc * sizeof(uint16_t) + M.rpb + 7) /
                        8 * 8;
    const size_t shm = (size_t)M.rpb * ((size_t)M.maxc * ((BS * BS) | 1) + (BS | 1)) * sizeof(double) + meta +
                       (st ? (size_t)M.maxnl * (nrec * sizeof(double) + sizeof(int)) + (size_t)M.maxpw * 9 : 0);
    // kernel-timing hook on the mesh level (not the coarse levels).
    // Algorithmic bytes: J (and its FP32 or BF16 copy when written) and R
    // written once; read once: the connectivity, the node state the element
    // evaluation needs (x, v and a at n+alpha, p, rho, mu and the solid mask:
    // 3d + 4 numbers) and the free-dof bits.  The solid fields of the present
    // solids are not counted (data-dependent; about 1% of the total on the
    // floe field).
    const bool fine = M.conn == ctx->conn;
    const int64_t slot = fine ? eft_kt_begin(ctx, EFT_KT_ASSEMBLE) : -1;
    const int d = ctx->dim;
    const double abytes =
        (J ? (double)J->nnzb * BS * BS * ((J->fp32 ? 4.0 : 8.0) + (a.J32 ? 4.0 : 0.0) + (a.J16 ? 2.0 : 0.0)) : 0.0) +
        (double)M.N * BS * 8.0 +
        (double)M.E * (d + 1) * 4.0 +
        (double)M.N * 8.0 * (3 * d + 4) + (double)M.N;
#define EFT_NS_LAUNCH(DD, TT, STG, JP) \
    hipLaunchKernelGGL((k_ns_rows<DD, TT, STG>), dim3(nb), dim3(256), shm, ctx->stream, a, JP)
    float *j32 = (J && J->fp32) ? J->val32 : nullptr;
    double *j64 = (J && !J->fp32) ? J->val : nullptr;
    if (ctx->dim == 2) {
        if (j32) { if (st) EFT_NS_LAUNCH(2, float, true, j32); else EFT_NS_LAUNCH(2, float, false, j32); }
        else if (st) EFT_NS_LAUNCH(2, double, true, j64);
        else EFT_NS_LAUNCH(2, double, false, j64);
    } else {
        if (j32) { if (st) EFT_NS_LAUNCH(3, float, true, j32); else EFT_NS_LAUNCH(3, float, false, j32); }
        else if (st) EFT_NS_LAUNCH(3, double, true, j64);
        else EFT_NS_LAUNCH(3, double, false, j64);
    }
#undef EFT_NS_LAUNCH
    EFT_HIP(hipGetLastError());
    eft_kt_end(ctx, slot, abytes, EFT_KT_ASSEMBLE);
    return EFT_OK;
}

// Residual and Jacobian of the momentum/mass block at the iterate (the node
// fields va, acc, rho, mu and the solid mask must be current, see eft_props); with a
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
    M.as = nullptr;   // (fractions and B at n+alpha from the arrays eft_props read)
    M.Ba = nullptr;
    M.smask = ctx->smask;
    M.n_dir = ctx->n_dir;
    M.dir_node = ctx->dir_node;
    M.dir_mask = ctx->dir_mask;
    M.fmask = ctx->fmask0;
    M.iptr = ctx->iptr;
    M.ient = ctx->ient;
    M.islot = ctx->islot;
    M.maxc = ctx->maxc;
    M.rpb = ctx->rpb_ns;
    M.wnptr = ctx->wnptr;
    M.wnode = ctx->wnode;
    M.iloc = ctx->iloc;
    M.maxnl = ctx->maxnl;
    M.maxpw = ctx->maxpw;
    // with the multigrid active, the assembly also writes the finest level's
    // FP32 copy of the values (no separate conversion pass over J)
    const bool mg = J && eft_mg_enabled(ctx, J);
    float *J32 = (mg && !ctx->par.mg_bf16 && !J->fp32) ? ctx->mg[0].A.val32 : nullptr;
    uint16_t *J16 = (mg && ctx->par.mg_bf16 && !J->fp32) ? ctx->mg[0].A.val16 : nullptr;
    EFT_TRY(eft_ns_level(ctx, M, it->vp, R, J, J32, J16));
    ctx->mg_f32_fresh = J32 != nullptr || J16 != nullptr;
    // (with mg_lag, inside a step past its first nonlinear iteration, the
    // coarse levels of the previous iteration are kept)
    if (mg) EFT_TRY(eft_mg_setup(ctx, it->vp, !(ctx->par.mg_lag && ctx->nl_k > 1 && ctx->mg_valid)));
    return EFT_OK;
}
