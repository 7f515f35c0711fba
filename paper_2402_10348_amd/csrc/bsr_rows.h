// Block-row products of a BSR matrix with square bs x bs blocks, shared by
// the Krylov SpMV and the multigrid smoother/residual kernels.
//
// One 64-wide wavefront owns R consecutive block rows.  Lane l = bs*j + r
// (j < 64/bs) holds scalar row r of block k0 + j (+ 64/bs, + 2*64/bs, ... for
// long rows) of each of them: it loads that row's bs contiguous values with
// vector loads, gathers the bs entries of x under the block's column and
// accumulates the dot product.  A whole block row of the 3D momentum matrix
// (<= 15 blocks of 4x4) is then a single pass whose value loads cover one
// contiguous run of the value array, and the R rows' passes are issued
// together, so every load of a wavefront is in flight at once; partial sums
// over j are combined with a shuffle tree over strides bs, 2 bs, 4 bs, ...
//
// Blocks are stored row-major (value (i, c) of block k at k*bs*bs + i*bs + c)
// and the value array starts 256-byte aligned.
//
// For narrow values (FP32, BF16) a second layout is faster: one block per
// lane (bsr_block_dot).  There a lane's loads are a whole block, and x under
// the block's column is gathered once per block instead of once per scalar
// row, which halves the gather requests that bound the layout above when
// the values are half as wide as x.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

typedef double eft_d2 __attribute__((ext_vector_type(2)));
typedef float eft_f2 __attribute__((ext_vector_type(2)));
typedef float eft_f4 __attribute__((ext_vector_type(4)));

// Index of the wavefront in its workgroup, as a wave-uniform value (so that
// loads indexed by it, such as the row pointers, go through the scalar unit).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// One load, plain or non-temporal (streamed: not kept in the caches).
template <bool NT, typename T> __device__ __forceinline__ T ld_hint(const T *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// bs consecutive values starting at p, with the widest aligned vector loads
// the offset allows.
template <int BS, typename T, bool NT> struct RowLoad;

template <int BS, bool NT> struct RowLoad<BS, double, NT> {
    static __device__ __forceinline__ void get(const double *p, double (&v)[BS])
    {
        if constexpr (BS % 2 == 0) {
#pragma unroll
            for (int q = 0; q < BS / 2; ++q) {
                const eft_d2 t = ld_hint<NT>(reinterpret_cast<const eft_d2 *>(p) + q);
                v[2 * q] = t.x;
                v[2 * q + 1] = t.y;
            }
        } else {
#pragma unroll
            for (int q = 0; q < BS; ++q) v[q] = ld_hint<NT>(p + q);
        }
    }
};

template <int BS, bool NT> struct RowLoad<BS, float, NT> {
    static __device__ __forceinline__ void get(const float *p, double (&v)[BS])
    {
        if constexpr (BS % 4 == 0) {
#pragma unroll
            for (int q = 0; q < BS / 4; ++q) {
                const eft_f4 t = ld_hint<NT>(reinterpret_cast<const eft_f4 *>(p) + q);
                v[4 * q] = t.x;
                v[4 * q + 1] = t.y;
                v[4 * q + 2] = t.z;
                v[4 * q + 3] = t.w;
            }
        } else if constexpr (BS % 2 == 0) {
#pragma unroll
            for (int q = 0; q < BS / 2; ++q) {
                const eft_f2 t = ld_hint<NT>(reinterpret_cast<const eft_f2 *>(p) + q);
                v[2 * q] = t.x;
                v[2 * q + 1] = t.y;
            }
        } else {
#pragma unroll
            for (int q = 0; q < BS; ++q) v[q] = ld_hint<NT>(p + q);
        }
    }
};

// BF16 value (the upper half of an FP32 bit pattern)
struct eft_bf16 {
    uint16_t v;
};

__device__ __forceinline__ double bf16_to_double(uint32_t bits16) { return (double)__uint_as_float(bits16 << 16); }

template <int BS, bool NT> struct RowLoad<BS, eft_bf16, NT> {
    static __device__ __forceinline__ void get(const eft_bf16 *p, double (&v)[BS])
    {
        typedef uint32_t u2 __attribute__((ext_vector_type(2)));
        if constexpr (BS % 4 == 0) {
#pragma unroll
            for (int q = 0; q < BS / 4; ++q) {
                const u2 t = ld_hint<NT>(reinterpret_cast<const u2 *>(p) + q);
                v[4 * q] = bf16_to_double(t.x & 0xFFFFu);
                v[4 * q + 1] = bf16_to_double(t.x >> 16);
                v[4 * q + 2] = bf16_to_double(t.y & 0xFFFFu);
                v[4 * q + 3] = bf16_to_double(t.y >> 16);
            }
        } else {
#pragma unroll
            for (int q = 0; q < BS; ++q) v[q] = bf16_to_double(p[q].v);
        }
    }
};

// bs entries of x under block column c (cached loads: x is re-read by every
// row that couples to c); x in FP64 or FP32.
template <int BS, typename TX = double>
__device__ __forceinline__ void x_get(const TX *__restrict__ x, int64_t c, double (&v)[BS])
{
    const TX *p = x + c * BS;
    if constexpr (sizeof(TX) == 4) {
        if constexpr (BS % 4 == 0) {
#pragma unroll
            for (int q = 0; q < BS / 4; ++q) {
                const eft_f4 t = reinterpret_cast<const eft_f4 *>(p)[q];
                v[4 * q] = t.x;
                v[4 * q + 1] = t.y;
                v[4 * q + 2] = t.z;
                v[4 * q + 3] = t.w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < BS; ++q) v[q] = p[q];
        }
    } else if constexpr (BS % 2 == 0) {
#pragma unroll
        for (int q = 0; q < BS / 2; ++q) {
            const eft_d2 t = reinterpret_cast<const eft_d2 *>(p)[q];
            v[2 * q] = t.x;
            v[2 * q + 1] = t.y;
        }
    } else {
#pragma unroll
        for (int q = 0; q < BS; ++q) v[q] = p[q];
    }
}

// (A x) of the block rows with extents [k0[q], k1[q]), q < R: the result for
// scalar row r of row q ends in acc[q] of lane r (lanes 0..bs-1); other
// lanes hold partial sums.  The first pass of every row is
// unrolled across the R rows so that all their loads are in flight together.
// Block extents [k0, k1) of wave-uniform rows (rows >= n get an empty
// extent; rowptr has n + 1 entries).  The loads go through the scalar unit.
template <int R>
__device__ __forceinline__ void row_extents(const int64_t (&row)[R], int64_t n, const int32_t *__restrict__ rowptr,
                                            int (&k0)[R], int (&k1)[R])
{
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int64_t a = row[q] < n ? row[q] : n, b = row[q] + 1 < n ? row[q] + 1 : n;
        k0[q] = rowptr[a];
        k1[q] = rowptr[b];
    }
}

template <int BS, typename TV, int R, bool NT>
__device__ __forceinline__ void bsr_rows_dot(const int (&k0)[R], const int (&k1)[R],
                                             const int32_t *__restrict__ col, const TV *__restrict__ val,
                                             const double *__restrict__ x, int lane, double (&acc)[R])
{
    constexpr int J = 64 / BS;
    const int j = lane / BS, r = lane - j * BS;
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = 0.0;
    if (j < J) {
        double v[R][BS], xv[R][BS];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int k = k0[q] + j;
            const bool ok = k < k1[q];
            const int c = ok ? col[k] : 0;
            if (ok) {
                RowLoad<BS, TV, NT>::get(val + (int64_t)k * (BS * BS) + r * BS, v[q]);
            } else {
#pragma unroll
                for (int e = 0; e < BS; ++e) v[q][e] = 0.0;
            }
            x_get<BS>(x, c, xv[q]);
        }
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int e = 0; e < BS; ++e) acc[q] += v[q][e] * xv[q][e];
#pragma unroll
        for (int q = 0; q < R; ++q)
            for (int k = k0[q] + j + J; k < k1[q]; k += J) {
                const int c = col[k];
                double vv[BS], xx[BS];
                RowLoad<BS, TV, NT>::get(val + (int64_t)k * (BS * BS) + r * BS, vv);
                x_get<BS>(x, c, xx);
#pragma unroll
                for (int e = 0; e < BS; ++e) acc[q] += vv[e] * xx[e];
            }
    }
#pragma unroll
    for (int s = 1; s < J; s <<= 1)
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const double o = __shfl_down(acc[q], s * BS, 64);
            if (j + s < J) acc[q] += o;
        }
}

// ---------------------------------------------------------------------------
// One block per lane.  The wavefront is split into segments of SEG lanes, one
// block row per segment (64 / SEG consecutive rows per wavefront); lane j of a
// segment takes blocks k0 + j, k0 + j + SEG, ... of its row whole, gathers the
// bs entries of x once per block and accumulates all bs outputs.  A butterfly
// over the segment leaves the row's product in every lane of the segment.

// Lanes per segment: the 3D Kuhn pattern has <= 15 blocks per row, the 2D one
// <= 7 (longer rows take further passes).
template <int BS> struct BlockSeg {
    static constexpr int SEG = BS <= 3 ? 8 : 16;
    static constexpr int RPW = 64 / SEG;   // rows per wavefront
};

// Extents [k0, k1) of row row0 + q (q = the lane's segment) from the RPW + 1
// wave-uniform row pointers at row0 (scalar loads; rows >= n are empty).
template <int RPW>
__device__ __forceinline__ void seg_extents(int64_t row0, int64_t n, const int32_t *__restrict__ rowptr, int q,
                                            int &k0, int &k1)
{
    int rp[RPW + 1];
#pragma unroll
    for (int t = 0; t <= RPW; ++t) rp[t] = rowptr[row0 + t < n ? row0 + t : n];
    k0 = rp[0];
    k1 = rp[1];
#pragma unroll
    for (int t = 1; t < RPW; ++t)
        if (q == t) {
            k0 = rp[t];
            k1 = rp[t + 1];
        }
}

template <int BS, typename TV, int SEG, typename TX>
__device__ __forceinline__ void bsr_block_dot(int k0, int k1, const int32_t *__restrict__ col,
                                              const TV *__restrict__ val, const TX *__restrict__ x, int j,
                                              double (&acc)[BS])
{
#pragma unroll
    for (int i = 0; i < BS; ++i) acc[i] = 0.0;
    for (int k = k0 + j; k < k1; k += SEG) {
        const int c = col[k];
        double v[BS][BS], xx[BS];
#pragma unroll
        for (int i = 0; i < BS; ++i) RowLoad<BS, TV, false>::get(val + (int64_t)k * (BS * BS) + i * BS, v[i]);
        x_get<BS>(x, c, xx);
#pragma unroll
        for (int i = 0; i < BS; ++i)
#pragma unroll
            for (int e = 0; e < BS; ++e) acc[i] += v[i][e] * xx[e];
    }
#pragma unroll
    for (int s = SEG / 2; s > 0; s >>= 1)
#pragma unroll
        for (int i = 0; i < BS; ++i) acc[i] += __shfl_xor(acc[i], s, 64);
}

// A whole bs x bs block (row-major at p) into v, with the widest loads its
// alignment allows: a 4x4 BF16 block (32 bytes, 32-byte aligned) is two
// 16-byte loads.
template <int BS, typename TV> __device__ __forceinline__ void block_get(const TV *__restrict__ p, double (&v)[BS][BS])
{
    if constexpr (BS == 4 && sizeof(TV) == 2) {
        typedef uint32_t u4 __attribute__((ext_vector_type(4)));
        const u4 lo = reinterpret_cast<const u4 *>(p)[0], hi = reinterpret_cast<const u4 *>(p)[1];
        const uint32_t w[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            v[t / 2][2 * (t % 2)] = bf16_to_double(w[t] & 0xFFFFu);
            v[t / 2][2 * (t % 2) + 1] = bf16_to_double(w[t] >> 16);
        }
    } else {
#pragma unroll
        for (int i = 0; i < BS; ++i) RowLoad<BS, TV, false>::get(p + i * BS, v[i]);
    }
}

// The same product for a pattern in stencil form: every column of row r is r
// + soff[s] for the set bits s of the row's mask m (soff ascending, at most
// SEG offsets), so lane j of the segment takes stencil slot j: its block is
// the popcount of the mask below j past the row's first block, its column is
// row + soff_j.  No column index is read, and the x gather does not wait for
// one.
template <int BS, typename TV, int SEG, typename TX>
__device__ __forceinline__ void bsr_stencil_dot(int k0, uint32_t m, int64_t row, int soff_j,
                                                const TV *__restrict__ val, const TX *__restrict__ x, int j,
                                                double (&acc)[BS])
{
#pragma unroll
    for (int i = 0; i < BS; ++i) acc[i] = 0.0;
    if ((m >> j) & 1u) {
        const int k = k0 + __popc(m & ((1u << j) - 1u));
        double v[BS][BS], xx[BS];
        block_get<BS, TV>(val + (int64_t)k * (BS * BS), v);
        x_get<BS>(x, row + soff_j, xx);
#pragma unroll
        for (int i = 0; i < BS; ++i)
#pragma unroll
            for (int e = 0; e < BS; ++e) acc[i] += v[i][e] * xx[e];
    }
#pragma unroll
    for (int s = SEG / 2; s > 0; s >>= 1)
#pragma unroll
        for (int i = 0; i < BS; ++i) acc[i] += __shfl_xor(acc[i], s, 64);
}

// bsr_rows_dot for a pattern in stencil form (wave-uniform rows row[q] with
// masks m[q]; soff_j = the offset of stencil slot j = lane / bs, 0 past the
// slots): lane bs*j + r takes scalar row r of the block at slot j, so no
// column index is read.  MAXS: the slots (at most 64 / bs).
template <int BS, typename TV, int R, int MAXS>
__device__ __forceinline__ void bsr_rows_stencil_dot(const int (&k0)[R], const uint32_t (&m)[R],
                                                     const int64_t (&row)[R], int soff_j,
                                                     const TV *__restrict__ val, const double *__restrict__ x,
                                                     int lane, double (&acc)[R])
{
    static_assert(MAXS * BS <= 64, "one slot per group of bs lanes");
    const int j = lane / BS, r = lane - j * BS;
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = 0.0;
    if (j < MAXS) {
        double v[R][BS], xv[R][BS];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const bool ok = (m[q] >> j) & 1u;
            const int k = k0[q] + __popc(m[q] & ((1u << j) - 1u));
            if (ok) {
                RowLoad<BS, TV, false>::get(val + (int64_t)k * (BS * BS) + r * BS, v[q]);
            } else {
#pragma unroll
                for (int e = 0; e < BS; ++e) v[q][e] = 0.0;
            }
            x_get<BS>(x, ok ? row[q] + soff_j : 0, xv[q]);
        }
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int e = 0; e < BS; ++e) acc[q] += v[q][e] * xv[q][e];
    }
#pragma unroll
    for (int s = 1; s < MAXS; s <<= 1)
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const double o = __shfl_down(acc[q], s * BS, 64);
            if (j + s < MAXS) acc[q] += o;
        }
}
