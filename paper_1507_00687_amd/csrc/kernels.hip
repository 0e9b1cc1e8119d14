// Device kernels for gfx950 (CDNA4): scaling-vector reductions, the fused leaf-product
// GEMM (S/T formation folded into the tile loads, MFMA leaf product) and the W-combination.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "devtypes.h"
#include "launch.h"

namespace fastmm {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;  // 4 wave64 per work-group
constexpr int kXcds = 8;       // MI355X: 8 XCDs, work-groups dispatched round-robin

template <typename T>
struct Mfma;
// D(16x16) += A(16x4) B(4x16) with lane l holding A[l%16][l/16] and B[l/16][l%16].
// Row of accumulator element v in lane l (column l%16): (l/16) + 4v for the f64 form,
// 4(l/16) + v for the f32 form (checked on the device).
template <>
struct Mfma<double> {
    typedef d4_t acc_t;
    __device__ static inline acc_t op(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
    typedef f4_t acc_t;
    __device__ static inline acc_t op(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

__device__ inline double ldexp_t(double x, int e) { return ldexp(x, e); }
__device__ inline float ldexp_t(float x, int e) { return ldexpf(x, e); }

// Block id remap so that consecutive logical tiles land on the same XCD (each XCD has its
// own L2): hardware places block b on XCD b % 8.  Bijective for any grid size.
__device__ inline int64_t xcd_remap(int64_t b, int64_t G) {
    const int64_t x = b % kXcds, j = b / kXcds;
    const int64_t per = G / kXcds, rem = G % kXcds;
    const int64_t base = (x < rem) ? x * (per + 1) : rem * (per + 1) + (x - rem) * per;
    return base + j;
}

template <typename T>
struct LeafArgs {
    const T *A;
    const T *B;
    T *out;
    int64_t lda, ldb, ldo;
    int64_t m, k, n;
    int64_t mb, kb, nb;
    int64_t leaf_stride;
    int tiles_m, tiles_n;
    const LeafEntry *leaves;
    const SrcEntry *asrc;
    const SrcEntry *bsrc;
    ScaleExps sc;
};

// One BMxBN tile of one leaf product.  2x2 waves, each owning a (BM/2)x(BN/2) sub-tile made
// of 16x16 MFMA blocks.  Per K step of BK: every thread forms BM*BK/256 elements of the S
// tile as the sequential sum over the leaf's A sources of coef * (scaled) element, and the
// same for T, stores them to LDS (k-major), then the waves run BK/4 MFMA steps.
template <typename T, int BM, int BN, int BK, bool TA, bool TB, bool SCALED, bool DIRECT>
__global__ __launch_bounds__(kThreads) void leaf_kernel(LeafArgs<T> p) {
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int EA = BM * BK / kThreads, EB = BK * BN / kThreads;
    static_assert(EA * kThreads == BM * BK && EB * kThreads == BK * BN, "tile/threads");
    __shared__ T As[BK][BM + 1];
    __shared__ T Bs[BK][BN + 1];

    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t tiles = (int64_t)p.tiles_m * p.tiles_n;
    const int64_t bid = xcd_remap(blockIdx.x, gridDim.x);
    const int leaf = (int)(bid / tiles);
    const int64_t rem = bid - (int64_t)leaf * tiles;
    const int64_t tm = rem / p.tiles_n, tn = rem - tm * p.tiles_n;
    const LeafEntry le = p.leaves[leaf];

    typename Mfma<T>::acc_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = typename Mfma<T>::acc_t{};

    for (int64_t k0 = 0; k0 < p.kb; k0 += BK) {
        T ra[EA], rb[EB];
        // ---- S tile: sum_src coef * A'(src block)
#pragma unroll
        for (int s = 0; s < EA; ++s) ra[s] = T(0);
        for (int q = 0; q < le.a_count; ++q) {
            const SrcEntry se = p.asrc[le.a_begin + q];
            const T c = (T)se.coef;
#pragma unroll
            for (int s = 0; s < EA; ++s) {
                const int e = t + kThreads * s;
                const int row = TA ? (e % BM) : (e / BK);
                const int kk = TA ? (e / BM) : (e % BK);
                const int64_t x = tm * BM + row, y = k0 + kk;
                const int64_t gr = (int64_t)se.br * p.mb + x, gc = (int64_t)se.bc * p.kb + y;
                T v = T(0);
                if (x < p.mb && y < p.kb && gr < p.m && gc < p.k) {
                    v = TA ? p.A[gc * p.lda + gr] : p.A[gr * p.lda + gc];
                    if (SCALED) v = ldexp_t(v, p.sc.ep[gc] - p.sc.ea[gr]);
                }
                const T term = c * v;
                ra[s] = (q == 0) ? term : ra[s] + term;
            }
        }
        // ---- T tile: sum_src coef * B'(src block)
#pragma unroll
        for (int s = 0; s < EB; ++s) rb[s] = T(0);
        for (int q = 0; q < le.b_count; ++q) {
            const SrcEntry se = p.bsrc[le.b_begin + q];
            const T c = (T)se.coef;
#pragma unroll
            for (int s = 0; s < EB; ++s) {
                const int e = t + kThreads * s;
                const int kk = TB ? (e % BK) : (e / BN);
                const int col = TB ? (e / BK) : (e % BN);
                const int64_t y = k0 + kk, z = tn * BN + col;
                const int64_t gr = (int64_t)se.br * p.kb + y, gc = (int64_t)se.bc * p.nb + z;
                T v = T(0);
                if (y < p.kb && z < p.nb && gr < p.k && gc < p.n) {
                    v = TB ? p.B[gc * p.ldb + gr] : p.B[gr * p.ldb + gc];
                    if (SCALED) v = ldexp_t(v, -p.sc.ep[gr] - p.sc.eb[gc]);
                }
                const T term = c * v;
                rb[s] = (q == 0) ? term : rb[s] + term;
            }
        }
#pragma unroll
        for (int s = 0; s < EA; ++s) {
            const int e = t + kThreads * s;
            const int row = TA ? (e % BM) : (e / BK);
            const int kk = TA ? (e / BM) : (e % BK);
            As[kk][row] = ra[s];
        }
#pragma unroll
        for (int s = 0; s < EB; ++s) {
            const int e = t + kThreads * s;
            const int kk = TB ? (e % BK) : (e / BN);
            const int col = TB ? (e / BK) : (e % BN);
            Bs[kk][col] = rb[s];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            T a[TM], b[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) a[i] = As[ks + (lane >> 4)][wm * WM + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < TN; ++j) b[j] = Bs[ks + (lane >> 4)][wn * WN + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = Mfma<T>::op(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }

    // ---- epilogue
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = tm * BM + wm * WM + i * 16 + Mfma<T>::row(lane, v);
                const int64_t col = tn * BN + wn * WN + j * 16 + (lane & 15);
                T val = acc[i][j][v];
                if (DIRECT) {
                    if (row < p.m && col < p.n) {
                        if (SCALED) val = ldexp_t(val, p.sc.ea[row] + p.sc.eb[col]);
                        p.out[row * p.ldo + col] = val;
                    }
                } else {
                    if (row < p.mb && col < p.nb) p.out[(int64_t)leaf * p.leaf_stride + row * p.ldo + col] = val;
                }
            }
}

template <typename T>
struct CombineArgs {
    const T *M;
    int64_t leaf_stride;
    T *C;
    int64_t ldc, m, n, mb, nb;
    int NB;
    const BlockDests *bdest;
    const DestEntry *dest;
    ScaleExps sc;
    int64_t zM = 0, zC = 0;  // combine_level_kernel: offsets of work-group layer z in M and C
};

// C(i, j) = 2^(ea_i + eb_j) * sum_q coef_q * M_{leaf_q}(i mod mb, j mod nb), summed in list
// order.  A thread owns VEC consecutive columns (x, y .. y+VEC-1) of the leaf-block grid and
// writes that position of every output block in turn, so the products it reads for one block
// are re-read for the next from cache, not HBM: each product element leaves HBM once.  VEC > 1
// only when the block width, n, ldc and the pointers allow 16-byte accesses (so the VEC
// columns never straddle C's edge); every element of C is written once.
template <typename T, int VEC>
struct VecOf;
template <>
struct VecOf<float, 4> {
    typedef float4 t;
};
template <>
struct VecOf<double, 2> {
    typedef double2 t;
};
template <>
struct VecOf<float, 2> {
    typedef float2 t;
};

// VEC consecutive int32 exponents in one load (the exponent vectors are 16-byte aligned and
// VEC divides the column index wherever VEC > 1).
template <int VEC>
__device__ inline void load_exps(const int32_t *e, int (&out)[VEC]) {
    if constexpr (VEC == 4) {
        const int4 t = *reinterpret_cast<const int4 *>(e);
        out[0] = t.x, out[1] = t.y, out[2] = t.z, out[3] = t.w;
    } else if constexpr (VEC == 2) {
        const int2 t = *reinterpret_cast<const int2 *>(e);
        out[0] = t.x, out[1] = t.y;
    } else {
        out[0] = e[0];
    }
}

template <typename T, bool SCALED, int VEC>
__global__ __launch_bounds__(kThreads) void combine_kernel(CombineArgs<T> p) {
    const int64_t y = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * VEC;
    if (y >= p.nb) return;
    const int64_t nP = (p.m + p.mb - 1) / p.mb, nS = (p.n + p.nb - 1) / p.nb;
    for (int64_t x = blockIdx.y; x < p.mb; x += gridDim.y) {
        for (int64_t P = blockIdx.z; P < nP; P += gridDim.z) {  // block rows spread over z when positions are few
            const int64_t row = P * p.mb + x;
            if (row >= p.m) break;
            for (int64_t S = 0; S < nS; ++S) {
                const int64_t col = S * p.nb + y;
                if (col >= p.n) break;
                const BlockDests bd = p.bdest[P * p.NB + S];
                T acc[VEC];
                // contributions in groups of up to 4: the group's loads are issued together,
                // then added in list order
                for (int q0 = 0; q0 < bd.count; q0 += 4) {
                    const int nq = bd.count - q0 < 4 ? bd.count - q0 : 4;
                    DestEntry de[4];
                    T v[4][VEC];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (u >= nq) break;
                        de[u] = p.dest[bd.begin + q0 + u];
                        const T *src = p.M + (int64_t)de[u].leaf * p.leaf_stride + x * p.nb + y;
                        if constexpr (VEC == 1) {
                            v[u][0] = *src;
                        } else {
                            const typename VecOf<T, VEC>::t w = *reinterpret_cast<const typename VecOf<T, VEC>::t *>(src);
                            const T *ws = reinterpret_cast<const T *>(&w);
#pragma unroll
                            for (int e = 0; e < VEC; ++e) v[u][e] = ws[e];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (u >= nq) break;
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            const T term = (T)de[u].coef * v[u][e];
                            acc[e] = (q0 + u == 0) ? term : acc[e] + term;
                        }
                    }
                }
                if (bd.count == 0) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) acc[e] = T(0);
                }
                if (SCALED) {
                    int eb[VEC];
                    load_exps<VEC>(p.sc.eb + col, eb);
                    const int ea = p.sc.ea[row];
#pragma unroll
                    for (int e = 0; e < VEC; ++e) acc[e] = ldexp_t(acc[e], ea + eb[e]);
                }
                T *dst = p.C + row * p.ldc + col;
                if constexpr (VEC == 1) {
                    *dst = acc[0];
                } else {
                    typename VecOf<T, VEC>::t w;
                    T *ws = reinterpret_cast<T *>(&w);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) ws[e] = acc[e];
                    *reinterpret_cast<typename VecOf<T, VEC>::t *>(dst) = w;
                }
            }
        }
    }
}

template <typename T>
struct Combine2Args {
    const T *M;
    int64_t leaf_stride;
    T *C;
    int64_t ldc, m, n, mb, nb;
    int R1, R2;
    float w1[4][8], w2[4][8];
    ScaleExps sc;
};

// The W-combination of two levels of <2,K0,2> rules, level by level as the recursion of eq.
// (2) sums it: for each first-level product r1 the thread forms the four second-level sums
// N(p2) = sum_r2 w2[p2][r2] M_(r1,r2), then adds w1[p1][r1] N(p2) to output block (p1, p2);
// both sums in increasing product order, zero coefficients skipped.  A thread owns VEC
// consecutive columns of one row of the leaf-block grid and keeps all 16 output blocks of that
// position in registers, so each product element is read once.
template <typename T, bool SCALED, int VEC>
__global__ __launch_bounds__(kThreads) void combine2_kernel(Combine2Args<T> p) {
    const int64_t y = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * VEC;
    if (y >= p.nb) return;
    for (int64_t x = blockIdx.y; x < p.mb; x += gridDim.y) {
        T acc[4][4][VEC];
        bool seen[4] = {false, false, false, false};
        for (int r1 = 0; r1 < p.R1; ++r1) {
            T mv[8][VEC];
#pragma unroll
            for (int r2 = 0; r2 < 8; ++r2) {
                if (r2 < p.R2) {
                    const T *src = p.M + (int64_t)(r1 * p.R2 + r2) * p.leaf_stride + x * p.nb + y;
                    if constexpr (VEC == 1) {
                        mv[r2][0] = *src;
                    } else {
                        const typename VecOf<T, VEC>::t w = *reinterpret_cast<const typename VecOf<T, VEC>::t *>(src);
                        const T *ws = reinterpret_cast<const T *>(&w);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) mv[r2][e] = ws[e];
                    }
                }
            }
            T nsum[4][VEC];
#pragma unroll
            for (int p2 = 0; p2 < 4; ++p2) {
                bool first = true;
#pragma unroll
                for (int r2 = 0; r2 < 8; ++r2) {
                    const float w = r2 < p.R2 ? p.w2[p2][r2] : 0.f;
                    if (w != 0.f) {
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            const T term = (T)w * mv[r2][e];
                            nsum[p2][e] = first ? term : nsum[p2][e] + term;
                        }
                        first = false;
                    }
                }
                if (first) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) nsum[p2][e] = T(0);
                }
            }
#pragma unroll
            for (int p1 = 0; p1 < 4; ++p1) {
                const float w = p.w1[p1][r1];
                if (w != 0.f) {
#pragma unroll
                    for (int p2 = 0; p2 < 4; ++p2)
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            const T term = (T)w * nsum[p2][e];
                            acc[p1][p2][e] = seen[p1] ? acc[p1][p2][e] + term : term;
                        }
                    seen[p1] = true;
                }
            }
        }
#pragma unroll
        for (int p1 = 0; p1 < 4; ++p1)
#pragma unroll
            for (int p2 = 0; p2 < 4; ++p2) {
                const int64_t row = (2 * (p1 >> 1) + (p2 >> 1)) * p.mb + x;
                const int64_t col = (2 * (p1 & 1) + (p2 & 1)) * p.nb + y;
                if (row >= p.m || col >= p.n) continue;
                T out[VEC];
                int eb[VEC];
                if (SCALED) load_exps<VEC>(p.sc.eb + col, eb);
                const int ea = SCALED ? p.sc.ea[row] : 0;
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    out[e] = seen[p1] ? acc[p1][p2][e] : T(0);
                    if (SCALED) out[e] = ldexp_t(out[e], ea + eb[e]);
                }
                T *dst = p.C + row * p.ldc + col;
                if constexpr (VEC == 1) {
                    *dst = out[0];
                } else {
                    typename VecOf<T, VEC>::t w;
                    T *ws = reinterpret_cast<T *>(&w);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) ws[e] = out[e];
                    *reinterpret_cast<typename VecOf<T, VEC>::t *>(dst) = w;
                }
            }
    }
}

// One level of a <2,K0,2> rule: C_p = sum_r w1[p][r] M_r for the four output blocks, products
// in increasing order (the order of the destination lists), each product element read once.
template <typename T, bool SCALED, int VEC>
__global__ __launch_bounds__(kThreads) void combine1_kernel(Combine2Args<T> p) {
    const int64_t y = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * VEC;
    if (y >= p.nb) return;
    for (int64_t x = blockIdx.y; x < p.mb; x += gridDim.y) {
        T mv[8][VEC];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (r < p.R1) {
                const T *src = p.M + (int64_t)r * p.leaf_stride + x * p.nb + y;
                if constexpr (VEC == 1) {
                    mv[r][0] = *src;
                } else {
                    const typename VecOf<T, VEC>::t w = *reinterpret_cast<const typename VecOf<T, VEC>::t *>(src);
                    const T *ws = reinterpret_cast<const T *>(&w);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) mv[r][e] = ws[e];
                }
            }
        }
#pragma unroll
        for (int p1 = 0; p1 < 4; ++p1) {
            const int64_t row = (p1 >> 1) * p.mb + x, col = (p1 & 1) * p.nb + y;
            if (row >= p.m || col >= p.n) continue;
            T acc[VEC];
            bool first = true;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const float w = r < p.R1 ? p.w1[p1][r] : 0.f;
                if (w != 0.f) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const T term = (T)w * mv[r][e];
                        acc[e] = first ? term : acc[e] + term;
                    }
                    first = false;
                }
            }
            int eb[VEC];
            if (SCALED) load_exps<VEC>(p.sc.eb + col, eb);
            const int ea = SCALED ? p.sc.ea[row] : 0;
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                if (first) acc[e] = T(0);
                if (SCALED) acc[e] = ldexp_t(acc[e], ea + eb[e]);
            }
            T *dst = p.C + row * p.ldc + col;
            if constexpr (VEC == 1) {
                *dst = acc[0];
            } else {
                typename VecOf<T, VEC>::t w;
                T *ws = reinterpret_cast<T *>(&w);
#pragma unroll
                for (int e = 0; e < VEC; ++e) ws[e] = acc[e];
                *reinterpret_cast<typename VecOf<T, VEC>::t *>(dst) = w;
            }
        }
    }
}

// One level of any rule with at most 16 output blocks (M0 N0 <= 16) and at most 64 products,
// from the destination lists: C_p = sum_r W[p][r] M_r in list order.  The lists are expanded
// into a dense W in LDS; a thread streams the products of its position (VEC columns of one row
// of the leaf-block grid), each read once, four loads in flight, into the output blocks it
// keeps in registers.
constexpr int kCombineMaxBlocks = 16, kCombineMaxProducts = 64;

template <typename T, bool SCALED, int VEC, int NBT>
__global__ __launch_bounds__(kThreads) void combine_level_kernel(CombineArgs<T> p, int nblocks, int nprod) {
    __shared__ float wt[kCombineMaxProducts][kCombineMaxBlocks];
    for (int i = threadIdx.x; i < kCombineMaxProducts * kCombineMaxBlocks; i += kThreads)
        wt[i / kCombineMaxBlocks][i % kCombineMaxBlocks] = 0.f;
    __syncthreads();
    for (int b = threadIdx.x; b < nblocks; b += kThreads) {
        const BlockDests bd = p.bdest[b];
        for (int q = 0; q < bd.count; ++q) {
            const DestEntry de = p.dest[bd.begin + q];
            wt[de.leaf][b] = de.coef;
        }
    }
    __syncthreads();
    const int64_t y = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * VEC;
    if (y >= p.nb) return;
    const T *M = p.M + (int64_t)blockIdx.z * p.zM;
    T *C = p.C + (int64_t)blockIdx.z * p.zC;
    for (int64_t x = blockIdx.y; x < p.mb; x += gridDim.y) {
        T acc[kCombineMaxBlocks][VEC];
        bool seen[kCombineMaxBlocks];
#pragma unroll
        for (int b = 0; b < kCombineMaxBlocks; ++b) seen[b] = false;
        for (int r0 = 0; r0 < nprod; r0 += 4) {
            T mv[4][VEC];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (r0 + u < nprod) {
                    const T *src = M + (int64_t)(r0 + u) * p.leaf_stride + x * p.nb + y;
                    if constexpr (VEC == 1) {
                        mv[u][0] = *src;
                    } else {
                        const typename VecOf<T, VEC>::t w = *reinterpret_cast<const typename VecOf<T, VEC>::t *>(src);
                        const T *ws = reinterpret_cast<const T *>(&w);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) mv[u][e] = ws[e];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
                for (int b = 0; b < kCombineMaxBlocks; ++b) {
                    const float w = r0 + u < nprod ? wt[r0 + u][b] : 0.f;
                    if (w != 0.f) {
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            const T term = (T)w * mv[u][e];
                            acc[b][e] = seen[b] ? acc[b][e] + term : term;
                        }
                        seen[b] = true;
                    }
                }
            }
        }
        // With the block-grid width NBT known at compile time, the scaling exponents of the
        // thread's NBT columns and 16 / NBT rows are loaded once, not once per output block
        // (per-block loads doubled the time of the scaled second level of <4,2,4>).
        constexpr int NR = NBT > 0 ? (kCombineMaxBlocks + NBT - 1) / NBT : 1, NC = NBT > 0 ? NBT : 1;
        int ea_r[NR], eb_c[NC][VEC];
        if constexpr (SCALED && NBT > 0) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const int64_t row = r * p.mb + x;
                ea_r[r] = (r * NBT < nblocks && row < p.m) ? p.sc.ea[row] : 0;
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int64_t col = c * p.nb + y;
                if (col < p.n) {
                    load_exps<VEC>(p.sc.eb + col, eb_c[c]);
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) eb_c[c][e] = 0;
                }
            }
        }
        const int nbw = NBT > 0 ? NBT : p.NB;
#pragma unroll
        for (int b = 0; b < kCombineMaxBlocks; ++b) {
            const int64_t row = (b / nbw) * p.mb + x, col = (b % nbw) * p.nb + y;
            if (b >= nblocks || row >= p.m || col >= p.n) continue;
            int eb[VEC], ea = 0;
            if constexpr (SCALED) {
                if constexpr (NBT > 0) {
                    ea = ea_r[b / NBT];
#pragma unroll
                    for (int e = 0; e < VEC; ++e) eb[e] = eb_c[b % NBT][e];
                } else {
                    load_exps<VEC>(p.sc.eb + col, eb);
                    ea = p.sc.ea[row];
                }
            }
            T out[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                out[e] = seen[b] ? acc[b][e] : T(0);
                if (SCALED) out[e] = ldexp_t(out[e], ea + eb[e]);
            }
            T *dst = C + row * p.ldc + col;
            if constexpr (VEC == 1) {
                *dst = out[0];
            } else {
                typename VecOf<T, VEC>::t w;
                T *ws = reinterpret_cast<T *>(&w);
#pragma unroll
                for (int e = 0; e < VEC; ++e) ws[e] = out[e];
                *reinterpret_cast<typename VecOf<T, VEC>::t *>(dst) = w;
            }
        }
    }
}

template <typename T>
struct NodeDenseArgs {
    const T *X;
    int64_t ld_r, ld_c, R, K, rb, cb;
    const LeafEntry *nodes;
    const SrcEntry *src;
    int b_side;
    const int32_t *e_r, *e_c;
    int s_r, s_c;
    T *Y;
    int64_t y_stride, y_ld;
};

// Node operands of the first recursion level written out (eq. (2)): node q is the sum over
// its source list of coef * block (br, bc) of op(X), each element scaled first.  One thread
// per column of the node block, rows strided over blockIdx.y, node q = blockIdx.z.
template <typename T, bool SCALED, int VEC>
__global__ __launch_bounds__(kThreads) void node_dense_kernel(NodeDenseArgs<T> p) {
    const int q = blockIdx.z;
    const LeafEntry le = p.nodes[q];
    const int begin = p.b_side ? le.b_begin : le.a_begin;
    const int count = p.b_side ? le.b_count : le.a_count;
    const int64_t col = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * VEC;  // VEC columns
    if (col >= p.cb) return;
    T *Y = p.Y + (int64_t)q * p.y_stride;
    for (int64_t row = blockIdx.y; row < p.rb; row += gridDim.y) {
        T acc[VEC];
        for (int j = 0; j < count; ++j) {
            const SrcEntry se = p.src[begin + j];
            const int64_t gr = (int64_t)se.br * p.rb + row, gc = (int64_t)se.bc * p.cb + col;
            T v[VEC];
            bool whole = false;
            if constexpr (VEC > 1) {
                whole = gr < p.R && gc + VEC <= p.K;
                if (whole) {  // the whole group inside op(X): one 16-byte load
                    const typename VecOf<T, VEC>::t w = *reinterpret_cast<const typename VecOf<T, VEC>::t *>(
                        p.X + gr * p.ld_r + gc);
                    const T *ws = reinterpret_cast<const T *>(&w);
                    int ec[VEC];
                    if (SCALED) load_exps<VEC>(p.e_c + gc, ec);
                    const int er = SCALED ? p.s_r * p.e_r[gr] : 0;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) v[e] = SCALED ? ldexp_t(ws[e], er + p.s_c * ec[e]) : ws[e];
                }
            }
            if (!whole) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    v[e] = T(0);
                    if (gr < p.R && gc + e < p.K) {
                        v[e] = p.X[gr * p.ld_r + (gc + e) * p.ld_c];
                        if (SCALED) v[e] = ldexp_t(v[e], p.s_r * p.e_r[gr] + p.s_c * p.e_c[gc + e]);
                    }
                }
            }
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const T term = (T)se.coef * v[e];
                acc[e] = j == 0 ? term : acc[e] + term;
            }
        }
        if (count == 0) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[e] = T(0);
        }
        if constexpr (VEC == 1) {
            Y[row * p.y_ld + col] = acc[0];
        } else {
            typename VecOf<T, VEC>::t w;
            T *ws = reinterpret_cast<T *>(&w);
#pragma unroll
            for (int e = 0; e < VEC; ++e) ws[e] = acc[e];
            *reinterpret_cast<typename VecOf<T, VEC>::t *>(Y + row * p.y_ld + col) = w;
        }
    }
}

// 16-byte accesses when op(X) has contiguous, 16-byte aligned rows and the node blocks hold
// whole groups (the planner's leaf blocks are multiples of 8 elements).
template <typename T>
hipError_t node_dense_go(const NodeDense &f, int nodes, hipStream_t s) {
    NodeDenseArgs<T> a;
    a.X = (const T *)f.X;
    a.ld_r = f.ld_r, a.ld_c = f.ld_c, a.R = f.R, a.K = f.K, a.rb = f.rb, a.cb = f.cb;
    a.nodes = f.nodes, a.src = f.src, a.b_side = f.b_side;
    a.e_r = f.e_r, a.e_c = f.e_c, a.s_r = f.s_r, a.s_c = f.s_c;
    a.Y = (T *)f.Y, a.y_stride = f.y_stride, a.y_ld = f.y_ld;
    constexpr int VEC = 16 / (int)sizeof(T);
    const bool vec = f.ld_c == 1 && (uintptr_t)f.X % 16 == 0 && f.ld_r % VEC == 0 && f.cb % VEC == 0 &&
                     f.y_ld % VEC == 0 && f.y_stride % VEC == 0 && (uintptr_t)f.Y % 16 == 0 &&
                     (f.e_c == nullptr || (uintptr_t)f.e_c % 16 == 0);
    const int per = vec ? VEC : 1;
    const int64_t gx = (f.cb / per + kThreads - 1) / kThreads;
    dim3 grid((unsigned)gx, (unsigned)std::min<int64_t>(f.rb, 1024), (unsigned)nodes);
    if (vec) {
        if (f.e_r) hipLaunchKernelGGL((node_dense_kernel<T, true, VEC>), grid, dim3(kThreads), 0, s, a);
        else hipLaunchKernelGGL((node_dense_kernel<T, false, VEC>), grid, dim3(kThreads), 0, s, a);
    } else {
        if (f.e_r) hipLaunchKernelGGL((node_dense_kernel<T, true, 1>), grid, dim3(kThreads), 0, s, a);
        else hipLaunchKernelGGL((node_dense_kernel<T, false, 1>), grid, dim3(kThreads), 0, s, a);
    }
    return hipGetLastError();
}

__global__ void fill_i32_kernel(int32_t *p, int64_t count, int32_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

template <typename T>
__global__ void zero_kernel(T *C, int64_t ldc, int64_t m, int64_t n) {
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= n) return;
    for (int64_t row = blockIdx.y; row < m; row += gridDim.y) C[row * ldc + col] = T(0);
}

// ------------------------------------------------------------------ scaling reductions
template <typename T>
struct Bits;
template <>
struct Bits<double> {
    typedef unsigned long long u;
    __device__ static u of(double x) { return (u)__double_as_longlong(x); }
};
template <>
struct Bits<float> {
    typedef unsigned int u;
    __device__ static u of(float x) { return (u)__float_as_uint(x); }
};

// max that keeps NaN once seen (so a NaN row/column gets the neutral factor 1)
template <typename T>
__device__ inline T nanmax(T a, T b) {
    return (b > a || b != b) ? b : a;
}

// 16-byte loads of VEC elements (VEC = 1: plain loads) and of the matching VEC exponents.
template <typename T, int VEC>
struct Vec {
    typedef T v_t __attribute__((ext_vector_type(VEC)));
    typedef int e_t __attribute__((ext_vector_type(VEC)));
    __device__ static v_t load(const T *p) { return *reinterpret_cast<const v_t *>(p); }
    __device__ static e_t exps(const int32_t *p) { return *reinterpret_cast<const e_t *>(p); }
};
template <typename T>
struct Vec<T, 1> {
    typedef T v_t;
    typedef int e_t;
    __device__ static v_t load(const T *p) { return *p; }
    __device__ static e_t exps(const int32_t *p) { return *p; }
};
template <typename V>
__device__ inline auto lane_of(const V &v, int j) {
    if constexpr (std::is_arithmetic<V>::value) return v;
    else return v[j];
}

// out[r] = max_c |X(r,c)| * 2^(sr*er[r] + sc*ec[c]) over a stored row-major R x C matrix
// whose rows are contiguous.  One wave per row; each lane takes VEC consecutive elements per
// load (rows 16-byte aligned when VEC > 1), four loads in flight, the tail element-wise.
template <typename T, int VEC>
__global__ __launch_bounds__(kThreads) void rowmax_kernel(const T *X, int64_t ld, int64_t R, int64_t C,
                                                           const int32_t *er, int sr, const int32_t *ec, int sc,
                                                           T *out) {
    typedef Vec<T, VEC> V;
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (r >= R) return;
    const int rexp = sr * er[r];
    const T *row = X + r * ld;
    T mx[4] = {T(0), T(0), T(0), T(0)};
    const int64_t Cv = C / VEC * VEC, step = 64 * VEC;
    int64_t c = (int64_t)lane * VEC;
    for (; c + 3 * step < Cv; c += 4 * step) {
        typename V::v_t x[4];
        typename V::e_t e[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = V::load(row + c + u * step), e[u] = V::exps(ec + c + u * step);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                const T xv = lane_of(x[u], j);
                const int ev = lane_of(e[u], j);
                mx[u] = nanmax(mx[u], ldexp_t(fabs(xv), rexp + sc * ev));
            }
    }
    for (; c < Cv; c += step) {
        const typename V::v_t x = V::load(row + c);
        const typename V::e_t e = V::exps(ec + c);
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const T xv = lane_of(x, j);
            const int ev = lane_of(e, j);
            mx[0] = nanmax(mx[0], ldexp_t(fabs(xv), rexp + sc * ev));
        }
    }
    for (int64_t t = Cv + lane; t < C; t += 64) mx[1] = nanmax(mx[1], ldexp_t(fabs(row[t]), rexp + sc * ec[t]));
    T m = nanmax(nanmax(mx[0], mx[1]), nanmax(mx[2], mx[3]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = nanmax(m, (T)__shfl_xor(m, off, 64));
    if (lane == 0) out[r] = m;
}

// out[c] = max_r |X(r,c)| * 2^(sr*er[r] + sc*ec[c]).  A work-group covers 64 VEC columns
// (16-byte loads when VEC > 1: rows 16-byte aligned) and a chunk of rows; each of its four
// waves takes every fourth row of the chunk, so a wave reads whole 64 VEC-column row
// segments.  The waves' maxima meet in LDS and one atomic max per column (on the IEEE bit
// pattern: order-independent, so the result is deterministic) merges the work-groups.  `out`
// must start at +0.
template <typename T, int VEC>
__global__ __launch_bounds__(kThreads) void colmax_kernel(const T *X, int64_t ld, int64_t R, int64_t C,
                                                           const int32_t *er, int sr, const int32_t *ec, int sc,
                                                           int64_t rows_per_block, T *out) {
    typedef Vec<T, VEC> V;
    constexpr int kGroups = kThreads / 64;
    __shared__ T part[kGroups][64 * VEC];
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int64_t c0 = ((int64_t)blockIdx.x * 64 + lane) * VEC;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_block;
    const int64_t r1 = r0 + rows_per_block < R ? r0 + rows_per_block : R;
    T mx[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) mx[j] = T(0);
    if (c0 + VEC <= C) {
        const typename V::e_t ce = V::exps(ec + c0);
        int64_t r = r0 + grp;
        for (; r + 3 * kGroups < r1; r += 4 * kGroups) {
            typename V::v_t x[4];
            int e[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                x[u] = V::load(X + (r + u * kGroups) * ld + c0), e[u] = sr * er[r + u * kGroups];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int j = 0; j < VEC; ++j)
                    mx[j] = nanmax(mx[j], ldexp_t(fabs(lane_of(x[u], j)), e[u] + sc * lane_of(ce, j)));
        }
        for (; r < r1; r += kGroups) {
            const typename V::v_t x = V::load(X + r * ld + c0);
            const int e = sr * er[r];
#pragma unroll
            for (int j = 0; j < VEC; ++j) mx[j] = nanmax(mx[j], ldexp_t(fabs(lane_of(x, j)), e + sc * lane_of(ce, j)));
        }
    } else {
        for (int j = 0; j < VEC && c0 + j < C; ++j) {
            const int cexp = sc * ec[c0 + j];
            for (int64_t r = r0 + grp; r < r1; r += kGroups)
                mx[j] = nanmax(mx[j], ldexp_t(fabs(X[r * ld + c0 + j]), cexp + sr * er[r]));
        }
    }
#pragma unroll
    for (int j = 0; j < VEC; ++j) part[grp][lane * VEC + j] = mx[j];
    __syncthreads();
    if (grp == 0) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            T m = part[0][lane * VEC + j];
#pragma unroll
            for (int g = 1; g < kGroups; ++g) m = nanmax(m, part[g][lane * VEC + j]);
            if (c0 + j < C) atomicMax(reinterpret_cast<typename Bits<T>::u *>(out + c0 + j), Bits<T>::of(m));
        }
    }
}

template <typename T>
__global__ void zero_elems_kernel(T *p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = T(0);
}

template <typename T>
__device__ inline bool finite_pos(T x) {
    return x > T(0) && x < T(INFINITY);  // false for NaN
}

// Smallest e with x <= 2^e, for finite x > 0.
template <typename T>
__device__ inline int ceil_log2(T x) {
    int e;
    const T f = frexp(x, &e);
    return (f == T(0.5)) ? e - 1 : e;
}

// Nearest integer to log2(x), for finite x > 0.  With x = f 2^e, f in [1/2, 1): e when
// f > 2^-1/2, else e - 1.  2^-1/2 is irrational, so no f equals it: comparing with the double
// just above it decides exactly (also for float f, whose values are doubles).
template <typename T>
__device__ inline int nearest_log2(T x) {
    int e;
    const T f = frexp(x, &e);
    return ((double)f >= 0x1.6a09e667f3bcdp-1) ? e : e - 1;
}

// Nearest integer to log2(b/a)/2, ties to even, for finite a, b > 0 (exact: mantissas of b
// and a compared directly).
template <typename T>
__device__ inline int half_log2_ratio(T b, T a) {
    int eb, ea;
    const T fb = frexp(b, &eb), fa = frexp(a, &ea);
    const int d = eb - ea;
    if ((d & 1) == 0) return d / 2;  // d even: log2(b/a) in (d-1, d+1)
    const int lo = (d - 1) >> 1, hi = lo + 1;
    if (fb < fa) return lo;
    if (fb > fa) return hi;
    return (lo & 1) == 0 ? lo : hi;
}

// O-step finalisation: e[i] += ceil_log2(max[i]) (or nearest_log2) where the max is finite
// and positive.  Stopping test (tau > 0): fail unless every unrounded factor max[i] >= thr.
template <typename T>
__global__ void o_finalize_kernel(const T *mx, int64_t count, int32_t *e, const int32_t *flags, int32_t *fail,
                                  int test, double thr, int nearest) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (flags[0] != 0 || i >= count) return;  // flags[0]: iteration already stopped
    const T v = mx[i];
    if (finite_pos(v)) {
        e[i] += nearest ? nearest_log2(v) : ceil_log2(v);
        if (test && (double)v < thr) atomicOr(fail, 1);
    }
}

// I-step finalisation: e[k] += nearest integer to log2(bmax/amax)/2.  Stopping test: fail
// unless every unrounded factor sqrt(bmax/amax) lies in [lo, hi].
template <typename T>
__global__ void i_finalize_kernel(const T *amax, const T *bmax, int64_t count, int32_t *e, const int32_t *flags,
                                  int32_t *fail, int test, double lo, double hi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (flags[0] != 0 || i >= count) return;
    const T a = amax[i], b = bmax[i];
    if (finite_pos(a) && finite_pos(b)) {
        e[i] += half_log2_ratio(b, a);
        if (test) {
            const double pe = sqrt((double)b / (double)a);
            if (pe < lo || pe > hi) atomicOr(fail, 1);
        }
    }
}

// After a tested step: stop the iteration if no factor failed; reset the fail flag.
__global__ void stop_update_kernel(int32_t *flags) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (flags[0] == 0 && flags[1] == 0) flags[0] = 1;
        flags[1] = 0;
    }
}

template <typename T, int BM, int BN, int BK, bool TA, bool TB>
hipError_t leaf_go(const LeafLaunch &L, hipStream_t s) {
    LeafArgs<T> a;
    a.A = (const T *)L.A;
    a.B = (const T *)L.B;
    a.out = (T *)L.out;
    a.lda = L.lda, a.ldb = L.ldb, a.ldo = L.ldo;
    a.m = L.m, a.k = L.k, a.n = L.n;
    a.mb = L.mb, a.kb = L.kb, a.nb = L.nb;
    a.leaf_stride = L.leaf_stride;
    a.tiles_m = (int)((L.mb + BM - 1) / BM);
    a.tiles_n = (int)((L.nb + BN - 1) / BN);
    a.leaves = L.leaves, a.asrc = L.asrc, a.bsrc = L.bsrc;
    a.sc = L.sc;
    const int64_t blocks = (int64_t)a.tiles_m * a.tiles_n * L.nleaves;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const bool scaled = L.sc.ea != nullptr;
    dim3 grid((unsigned)blocks), block(kThreads);
    if (L.direct) {
        if (scaled) hipLaunchKernelGGL((leaf_kernel<T, BM, BN, BK, TA, TB, true, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((leaf_kernel<T, BM, BN, BK, TA, TB, false, true>), grid, block, 0, s, a);
    } else {
        if (scaled) hipLaunchKernelGGL((leaf_kernel<T, BM, BN, BK, TA, TB, true, false>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((leaf_kernel<T, BM, BN, BK, TA, TB, false, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

template <typename T, int BM, int BN, int BK>
hipError_t leaf_trans(const LeafLaunch &L, hipStream_t s) {
    if (L.transA) {
        if (L.transB) return leaf_go<T, BM, BN, BK, true, true>(L, s);
        return leaf_go<T, BM, BN, BK, true, false>(L, s);
    }
    if (L.transB) return leaf_go<T, BM, BN, BK, false, true>(L, s);
    return leaf_go<T, BM, BN, BK, false, false>(L, s);
}

template <typename T>
hipError_t combine2_go(const CombineLaunch &L, hipStream_t s) {
    Combine2Args<T> a;
    a.M = (const T *)L.M;
    a.leaf_stride = L.leaf_stride;
    a.C = (T *)L.C;
    a.ldc = L.ldc, a.m = L.m, a.n = L.n, a.mb = L.mb, a.nb = L.nb;
    a.R1 = L.R1, a.R2 = L.R2;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 8; ++j) a.w1[i][j] = L.w1[i][j], a.w2[i][j] = L.w2[i][j];
    a.sc = L.sc;
    if (L.R1 < 1 || L.R1 > 8 || (L.kron == 2 && (L.R2 < 1 || L.R2 > 8))) return hipErrorInvalidValue;
    constexpr int VEC = 16 / (int)sizeof(T), VEC2 = 2;
    const bool vec = L.nb % VEC == 0 && L.n % VEC == 0 && L.ldc % VEC == 0 && (uintptr_t)L.C % 16 == 0 &&
                     (uintptr_t)L.M % 16 == 0 && L.leaf_stride % VEC == 0;
    const int per = vec ? VEC : 1;
    const int64_t cols = (L.nb + per - 1) / per;
    dim3 grid((unsigned)((cols + kThreads - 1) / kThreads), (unsigned)(L.mb < 65535 ? L.mb : 65535));
    const bool sc = L.sc.ea != nullptr;
    if (L.kron == 1) {
        if (vec) {
            if (sc) hipLaunchKernelGGL((combine1_kernel<T, true, VEC>), grid, dim3(kThreads), 0, s, a);
            else hipLaunchKernelGGL((combine1_kernel<T, false, VEC>), grid, dim3(kThreads), 0, s, a);
        } else {
            if (sc) hipLaunchKernelGGL((combine1_kernel<T, true, 1>), grid, dim3(kThreads), 0, s, a);
            else hipLaunchKernelGGL((combine1_kernel<T, false, 1>), grid, dim3(kThreads), 0, s, a);
        }
    } else if (vec) {
        // two-element vectors: for FP32 half the registers of 16-byte ones (the 16 output
        // blocks' sums are live), so twice the waves in flight (n=16384: 1.42 -> 0.85 ms); for
        // FP64 16 bytes, 14 % faster than one element (n=8192: 0.50 -> 0.43 ms)
        const dim3 grid2((unsigned)((L.nb / VEC2 + kThreads - 1) / kThreads), grid.y);
        if (sc) hipLaunchKernelGGL((combine2_kernel<T, true, VEC2>), grid2, dim3(kThreads), 0, s, a);
        else hipLaunchKernelGGL((combine2_kernel<T, false, VEC2>), grid2, dim3(kThreads), 0, s, a);
    } else {
        if (sc) hipLaunchKernelGGL((combine2_kernel<T, true, 1>), grid, dim3(kThreads), 0, s, a);
        else hipLaunchKernelGGL((combine2_kernel<T, false, 1>), grid, dim3(kThreads), 0, s, a);
    }
    return hipGetLastError();
}

// One level of the lists in `a` over nz layers (layer z reads M + z zM, writes C + z zC), with
// 16-byte vectors where the shapes allow (16 output blocks' sums are live per thread; 8-byte
// vectors ran 12-14 % slower for FP32 and 1.8x for FP64, whose 8-byte form is one element).
template <typename T>
hipError_t combine_level_launch(const CombineArgs<T> &a, int nblocks, int nprod, int nz, hipStream_t s) {
    if (nblocks < 1 || nblocks > kCombineMaxBlocks || nprod < 1 || nprod > kCombineMaxProducts || a.NB < 1 ||
        nz < 1 || nz > 65535)
        return hipErrorInvalidValue;
    constexpr int VEC = 16 / (int)sizeof(T);
    const bool vec = VEC > 1 && a.nb % VEC == 0 && a.n % VEC == 0 && a.ldc % VEC == 0 && (uintptr_t)a.C % 8 == 0 &&
                     (uintptr_t)a.M % 8 == 0 && a.leaf_stride % VEC == 0 && a.zM % VEC == 0 && a.zC % VEC == 0;
    const int per = vec ? VEC : 1;
    const int64_t cols = (a.nb + per - 1) / per;
    dim3 grid((unsigned)((cols + kThreads - 1) / kThreads), (unsigned)(a.mb < 65535 ? a.mb : 65535), (unsigned)nz);
    const bool sc = a.sc.ea != nullptr;
    if (vec && sc && a.NB == 4) {
        hipLaunchKernelGGL((combine_level_kernel<T, true, VEC, 4>), grid, dim3(kThreads), 0, s, a, nblocks, nprod);
    } else if (vec) {
        if (sc) hipLaunchKernelGGL((combine_level_kernel<T, true, VEC, 0>), grid, dim3(kThreads), 0, s, a, nblocks, nprod);
        else hipLaunchKernelGGL((combine_level_kernel<T, false, VEC, 0>), grid, dim3(kThreads), 0, s, a, nblocks, nprod);
    } else {
        if (sc) hipLaunchKernelGGL((combine_level_kernel<T, true, 1, 0>), grid, dim3(kThreads), 0, s, a, nblocks, nprod);
        else hipLaunchKernelGGL((combine_level_kernel<T, false, 1, 0>), grid, dim3(kThreads), 0, s, a, nblocks, nprod);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t combine_level_go(const CombineLaunch &L, hipStream_t s) {
    CombineArgs<T> a;
    a.M = (const T *)L.M;
    a.leaf_stride = L.leaf_stride;
    a.C = (T *)L.C;
    a.ldc = L.ldc, a.m = L.m, a.n = L.n, a.mb = L.mb, a.nb = L.nb;
    a.NB = L.NB;
    a.bdest = L.bdest, a.dest = L.dest, a.sc = L.sc;
    return combine_level_launch<T>(a, L.R2, L.R1, 1, s);  // R2 output blocks, R1 products
}

// Two levels of one rule, level by level (kron = 4): the R children of every first-level node
// summed into the node's product (M0 mb x N0 nb, in L.nodes), then the R node products into C
// with the scaling factors; each product element is read once per level.
template <typename T>
hipError_t combine_two_go(const CombineLaunch &L, hipStream_t s) {
    const int R = L.R1, nblocks = L.M0 * L.N0;
    const int64_t nm = (int64_t)L.M0 * L.mb, nn = (int64_t)L.N0 * L.nb, node = nm * nn;
    CombineArgs<T> a;
    a.M = (const T *)L.M, a.leaf_stride = L.leaf_stride;
    a.C = (T *)L.nodes, a.ldc = nn, a.m = nm, a.n = nn, a.mb = L.mb, a.nb = L.nb;
    a.NB = L.N0, a.bdest = L.bdest1, a.dest = L.dest1, a.sc = ScaleExps{nullptr, nullptr, nullptr};
    a.zM = (int64_t)R * L.leaf_stride, a.zC = node;
    hipError_t e = combine_level_launch<T>(a, nblocks, R, R, s);
    if (e != hipSuccess) return e;
    CombineArgs<T> b;
    b.M = (const T *)L.nodes, b.leaf_stride = node;
    b.C = (T *)L.C, b.ldc = L.ldc, b.m = L.m, b.n = L.n, b.mb = nm, b.nb = nn;
    b.NB = L.N0, b.bdest = L.bdest1, b.dest = L.dest1, b.sc = L.sc;
    return combine_level_launch<T>(b, nblocks, R, 1, s);
}

template <typename T>
hipError_t combine_go(const CombineLaunch &L, hipStream_t s) {
    if (L.kron == 3) {
        if (L.m <= 0 || L.n <= 0) return hipSuccess;
        if (L.mb <= 0 || L.nb <= 0) return hipErrorInvalidValue;
        return combine_level_go<T>(L, s);
    }
    if (L.kron == 4) {
        if (L.m <= 0 || L.n <= 0) return hipSuccess;
        if (L.mb <= 0 || L.nb <= 0 || !L.nodes || !L.bdest1 || !L.dest1) return hipErrorInvalidValue;
        return combine_two_go<T>(L, s);
    }
    if (L.kron) {
        if (L.m <= 0 || L.n <= 0) return hipSuccess;
        if (L.mb <= 0 || L.nb <= 0) return hipErrorInvalidValue;
        return combine2_go<T>(L, s);
    }
    CombineArgs<T> a;
    a.M = (const T *)L.M;
    a.leaf_stride = L.leaf_stride;
    a.C = (T *)L.C;
    a.ldc = L.ldc, a.m = L.m, a.n = L.n, a.mb = L.mb, a.nb = L.nb;
    a.NB = L.NB;
    a.bdest = L.bdest, a.dest = L.dest, a.sc = L.sc;
    if (L.m <= 0 || L.n <= 0) return hipSuccess;
    constexpr int VEC = 16 / (int)sizeof(T);
    const bool vec = L.nb % VEC == 0 && L.n % VEC == 0 && L.ldc % VEC == 0 && (uintptr_t)L.C % 16 == 0 &&
                     (uintptr_t)L.M % 16 == 0 && L.leaf_stride % VEC == 0;
    if (L.mb <= 0 || L.nb <= 0) return hipErrorInvalidValue;
    const int per = vec ? VEC : 1;
    const int64_t cols = (L.nb + per - 1) / per;  // threads span one leaf block; each visits every block
    // with few positions (small leaf blocks, many output blocks) the output block rows are
    // spread over gridDim.z, for about 4M threads in flight
    const int64_t nP = (L.m + L.mb - 1) / L.mb, threads = cols * L.mb;
    const int64_t z = std::max<int64_t>(1, std::min<int64_t>(nP, ((int64_t)1 << 22) / std::max<int64_t>(threads, 1)));
    dim3 grid((unsigned)((cols + kThreads - 1) / kThreads), (unsigned)(L.mb < 65535 ? L.mb : 65535),
              (unsigned)std::min<int64_t>(z, 65535));
    const bool sc = L.sc.ea != nullptr;
    if (vec) {
        if (sc) hipLaunchKernelGGL((combine_kernel<T, true, VEC>), grid, dim3(kThreads), 0, s, a);
        else hipLaunchKernelGGL((combine_kernel<T, false, VEC>), grid, dim3(kThreads), 0, s, a);
    } else {
        if (sc) hipLaunchKernelGGL((combine_kernel<T, true, 1>), grid, dim3(kThreads), 0, s, a);
        else hipLaunchKernelGGL((combine_kernel<T, false, 1>), grid, dim3(kThreads), 0, s, a);
    }
    return hipGetLastError();
}

inline unsigned grid1d(int64_t count, int per) {
    int64_t g = (count + per - 1) / per;
    if (g < 1) g = 1;
    if (g > 65535) g = 65535;
    return (unsigned)g;
}

// Elements per 16-byte load for a stored row-major matrix: 16 / sizeof(T) when every row
// starts 16-byte aligned, else 1.
template <typename T>
constexpr int kVec = 16 / (int)sizeof(T);
template <typename T>
bool rows_aligned(const T *X, int64_t ld) {
    return ((uintptr_t)X % 16) == 0 && ld % kVec<T> == 0;
}

template <typename T>
void launch_rowmax(const T *X, int64_t ld, int64_t R, int64_t C, const int32_t *er, int sr, const int32_t *ec,
                   int sc, T *out, hipStream_t s) {
    const dim3 grid((unsigned)((R + 3) / 4));
    if (rows_aligned(X, ld))
        hipLaunchKernelGGL((rowmax_kernel<T, kVec<T>>), grid, dim3(kThreads), 0, s, X, ld, R, C, er, sr, ec, sc, out);
    else
        hipLaunchKernelGGL((rowmax_kernel<T, 1>), grid, dim3(kThreads), 0, s, X, ld, R, C, er, sr, ec, sc, out);
}

// Column maxima of a stored R x C matrix: about 2048 work-groups of at least 32 rows.
template <typename T>
void launch_colmax(const T *X, int64_t ld, int64_t R, int64_t C, const int32_t *er, int sr, const int32_t *ec,
                   int sc, T *out, hipStream_t s) {
    hipLaunchKernelGGL(zero_elems_kernel<T>, dim3(grid1d(C, kThreads)), dim3(kThreads), 0, s, out, C);
    if (R <= 0) return;  // empty columns: maxima 0
    const int vec = rows_aligned(X, ld) ? kVec<T> : 1;
    const int64_t gx = (C + 64 * vec - 1) / (64 * vec);
    int64_t rpb = std::max<int64_t>(32, (R * gx + 2047) / 2048);
    const int64_t gy = std::min<int64_t>((R + rpb - 1) / rpb, 65535);
    rpb = (R + gy - 1) / gy;
    const dim3 grid((unsigned)gx, (unsigned)gy);
    if (vec > 1)
        hipLaunchKernelGGL((colmax_kernel<T, kVec<T>>), grid, dim3(kThreads), 0, s, X, ld, R, C, er, sr, ec, sc, rpb,
                           out);
    else
        hipLaunchKernelGGL((colmax_kernel<T, 1>), grid, dim3(kThreads), 0, s, X, ld, R, C, er, sr, ec, sc, rpb, out);
}

// Logical reductions over op(X) where op(X) is R x C; the stored matrix is row-major with
// contiguous rows (trans == 0) or op(X) = stored^T (trans != 0).
template <typename T>
hipError_t reduce_rows(const T *X, int64_t ld, int trans, int64_t R, int64_t C, const int32_t *er, int sr,
                       const int32_t *ec, int sc, T *out, hipStream_t s) {
    if (R <= 0) return hipSuccess;
    if (!trans) launch_rowmax<T>(X, ld, R, C, er, sr, ec, sc, out, s);
    else launch_colmax<T>(X, ld, C, R, ec, sc, er, sr, out, s);  // rows of op(X): columns of the stored C x R
    return hipGetLastError();
}

template <typename T>
hipError_t reduce_cols(const T *X, int64_t ld, int trans, int64_t R, int64_t C, const int32_t *er, int sr,
                       const int32_t *ec, int sc, T *out, hipStream_t s) {
    if (C <= 0) return hipSuccess;
    if (!trans) launch_colmax<T>(X, ld, R, C, er, sr, ec, sc, out, s);
    else launch_rowmax<T>(X, ld, C, R, ec, sc, er, sr, out, s);
    return hipGetLastError();
}

template <typename T>
hipError_t scale_step_t(const ScaleStep &S, hipStream_t s) {
    const T *A = (const T *)S.A;
    const T *B = (const T *)S.B;
    T *mA = (T *)S.maxA;
    T *mB = (T *)S.maxB;
    hipError_t err;
    // Note: the reductions run even after an early stop; the finalisers are guarded by the
    // stop flag, so the exponents no longer change.
    if (S.kind == 'O') {
        // rows of A' = diag(2^-ea) A diag(2^ep): max over k of |A_ik| 2^(ep_k - ea_i)
        err = reduce_rows<T>(A, S.lda, S.transA, S.m, S.k, S.ea, -1, S.ep, +1, mA, s);
        if (err != hipSuccess) return err;
        // columns of B' = diag(2^-ep) B diag(2^-eb)
        err = reduce_cols<T>(B, S.ldb, S.transB, S.k, S.n, S.ep, -1, S.eb, -1, mB, s);
        if (err != hipSuccess) return err;
        const double thr = S.test ? std::pow(1.0 + S.tau, -0.5) : 0.0;
        hipLaunchKernelGGL(o_finalize_kernel<T>, dim3(grid1d(S.m, kThreads)), dim3(kThreads), 0, s, mA, S.m,
                           S.ea, S.flags, S.flags + 1, S.test, thr, S.o_nearest);
        hipLaunchKernelGGL(o_finalize_kernel<T>, dim3(grid1d(S.n, kThreads)), dim3(kThreads), 0, s, mB, S.n,
                           S.eb, S.flags, S.flags + 1, S.test, thr, S.o_nearest);
    } else {
        // columns of A' and rows of B'
        err = reduce_cols<T>(A, S.lda, S.transA, S.m, S.k, S.ea, -1, S.ep, +1, mA, s);
        if (err != hipSuccess) return err;
        err = reduce_rows<T>(B, S.ldb, S.transB, S.k, S.n, S.ep, -1, S.eb, -1, mB, s);
        if (err != hipSuccess) return err;
        const double lo = S.test ? std::pow(1.0 + S.tau, -0.25) : 0.0;
        const double hi = S.test ? std::pow(1.0 + S.tau, 0.25) : 0.0;
        hipLaunchKernelGGL(i_finalize_kernel<T>, dim3(grid1d(S.k, kThreads)), dim3(kThreads), 0, s, mA, mB, S.k,
                           S.ep, S.flags, S.flags + 1, S.test, lo, hi);
    }
    if (S.test) hipLaunchKernelGGL(stop_update_kernel, dim3(1), dim3(64), 0, s, S.flags);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_leaf(const LeafLaunch &L, hipStream_t s) {
    if (!L.transA && !L.transB) return launch_leaf_pipelined(L, s);
    if (L.elem == Elem::F64) return leaf_trans<double, 64, 64, 16>(L, s);
    return leaf_trans<float, 128, 128, 16>(L, s);
}

hipError_t launch_combine(const CombineLaunch &L, hipStream_t s) {
    if (L.elem == Elem::F64) return combine_go<double>(L, s);
    return combine_go<float>(L, s);
}

hipError_t launch_node_dense(const NodeDense &f, int nodes, hipStream_t s) {
    if (nodes <= 0 || f.rb <= 0 || f.cb <= 0) return hipSuccess;
    if (nodes > 65535 || (f.cb + kThreads - 1) / kThreads > 0x7fffffff) return hipErrorInvalidValue;
    if (f.elem == Elem::F64) return node_dense_go<double>(f, nodes, s);
    return node_dense_go<float>(f, nodes, s);
}

hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t value, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid1d(count, kThreads)), dim3(kThreads), 0, s, p, count, value);
    return hipGetLastError();
}

hipError_t launch_zero_elems(Elem e, void *C, int64_t ldc, int64_t m, int64_t n, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + kThreads - 1) / kThreads), (unsigned)(m < 65535 ? m : 65535));
    if (e == Elem::F64) hipLaunchKernelGGL(zero_kernel<double>, grid, dim3(kThreads), 0, s, (double *)C, ldc, m, n);
    else hipLaunchKernelGGL(zero_kernel<float>, grid, dim3(kThreads), 0, s, (float *)C, ldc, m, n);
    return hipGetLastError();
}

hipError_t launch_scale_step(const ScaleStep &S, hipStream_t s) {
    if (S.elem == Elem::F64) return scale_step_t<double>(S, s);
    return scale_step_t<float>(S, s);
}

}  // namespace fastmm
