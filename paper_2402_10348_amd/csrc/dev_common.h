// Device helpers shared by the kernels: simplex geometry, the degree-2
// quadrature rule and wavefront/block reductions.
#pragma once

#include <hip/hip_runtime.h>

// Degree-2 simplex rules: triangle 3 points (2/3,1/6,1/6), weight |e|/3;
// tetrahedron 4 points (a,b,b,b) with a=(5+3 sqrt5)/20, b=(5-sqrt5)/20,
// weight |e|/4.  Point q has barycentric coordinate QA at node q and QB at the
// others.
template <int D> struct Rule;
template <> struct Rule<2> {
    static constexpr int NQ = 3;
    static constexpr double QA = 2.0 / 3.0;
    static constexpr double QB = 1.0 / 6.0;
    static constexpr double WF = 1.0 / 3.0;
};
template <> struct Rule<3> {
    static constexpr int NQ = 4;
    static constexpr double QA = 0.58541019662496845446;
    static constexpr double QB = 0.13819660112501051518;
    static constexpr double WF = 0.25;
};

template <int D> __device__ __forceinline__ double shape_at(int q, int a)
{
    return q == a ? Rule<D>::QA : Rule<D>::QB;
}

// Gradients of the P1 shape functions, contravariant metric G = J^-T J^-1 of
// the map from the unit right simplex, and |e|.  X[a][i] are node coordinates.
template <int D>
__device__ __forceinline__ double simplex_geom(const double (&X)[D + 1][D], double (&dN)[D + 1][D],
                                               double (&G)[D][D])
{
    double M[D][D];  // M[i][k] = dx_i / dxi_k
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int k = 0; k < D; ++k) M[i][k] = X[k + 1][i] - X[0][i];
    double inv[D][D];  // inv[k][i] = dxi_k / dx_i
    double det;
    if constexpr (D == 2) {
        det = M[0][0] * M[1][1] - M[0][1] * M[1][0];
        double r = 1.0 / det;
        inv[0][0] = M[1][1] * r;
        inv[0][1] = -M[0][1] * r;
        inv[1][0] = -M[1][0] * r;
        inv[1][1] = M[0][0] * r;
    } else {
        double c00 = M[1][1] * M[2][2] - M[1][2] * M[2][1];
        double c01 = M[1][2] * M[2][0] - M[1][0] * M[2][2];
        double c02 = M[1][0] * M[2][1] - M[1][1] * M[2][0];
        det = M[0][0] * c00 + M[0][1] * c01 + M[0][2] * c02;
        double r = 1.0 / det;
        inv[0][0] = c00 * r;
        inv[1][0] = c01 * r;
        inv[2][0] = c02 * r;
        inv[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) * r;
        inv[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) * r;
        inv[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) * r;
        inv[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) * r;
        inv[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) * r;
        inv[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) * r;
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            dN[k + 1][i] = inv[k][i];
            s += inv[k][i];
        }
        dN[0][i] = -s;
    }
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) s += inv[k][i] * inv[k][j];
            G[i][j] = s;
        }
    return fabs(det) * (D == 2 ? 0.5 : (1.0 / 6.0));
}

// Voigt component c -> (i, j): [11,22,33,12,23,13] (3D), [11,22,12] (2D)
template <int D> __device__ __forceinline__ void vpair(int c, int &i, int &j)
{
    if constexpr (D == 3) {
        const int I[6] = {0, 1, 2, 0, 1, 0}, J[6] = {0, 1, 2, 1, 2, 2};
        i = I[c];
        j = J[c];
    } else {
        const int I[3] = {0, 1, 0}, J[3] = {0, 1, 1};
        i = I[c];
        j = J[c];
    }
}

template <int D> struct NV {
    static constexpr int v = D == 3 ? 6 : 3;
};

template <int D> __device__ __forceinline__ void vfull(const double *b, double (&M)[D][D])
{
#pragma unroll
    for (int c = 0; c < NV<D>::v; ++c) {
        int i, j;
        vpair<D>(c, i, j);
        M[i][j] = b[c];
        M[j][i] = b[c];
    }
}

// ---------------------------------------------------------- reductions ----

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// BF16 bit pattern of f, round to nearest even (the upper half of the FP32
// pattern after adding the rounding bias).
__device__ __forceinline__ uint16_t to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Sum over a block of BLOCK threads; result valid in thread 0.
template <int BLOCK> __device__ __forceinline__ double block_sum(double v, double *lds)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) s += lds[w];
    }
    __syncthreads();
    return s;
}
