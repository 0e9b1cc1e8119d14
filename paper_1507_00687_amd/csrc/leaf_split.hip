// Split-precision fused leaf-product kernel: FP32 operands, leaf products on the bf16 / fp16
// matrix cores (v_mfma_f32_16x16x32_bf16 / _f16) with FP32 accumulation.
//
// Each S_r / T_r tile element is formed in FP32 from the leaf's source blocks (coefficients and
// scaling exponents applied in registers, as in the FP32 kernel), then split into limbs
// x = x_1 + x_2 (+ x_3) with x_1 = round(x), x_2 = round(x - x_1), ... (round to nearest even
// in bf16 or fp16; every residual is exact in FP32).  The leaf product is the sum of the limb
// products of total order <= 2 that the precision form keeps: 1 product (one limb), 3 products
// x1 y1 + x1 y2 + x2 y1 (two limbs), 6 products x1y1 + x1y2 + x2y1 + x1y3 + x2y2 + x3y1 (three
// limbs).  Both operands are read with k contiguous: A as stored (m x k) and B through a
// transposed copy (n x k) made by transpose_kernel, so the 8-element k fragments that the
// packed MFMA operands need are single 16-byte LDS reads.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "devtypes.h"
#include "fastmm.h"
#include "launch.h"

namespace fastmm {
namespace {

constexpr int kNT = 256;
constexpr int kXcd = 8;

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef short s8v __attribute__((ext_vector_type(8)));
typedef short s4v __attribute__((ext_vector_type(4)));

// Limb format: BF16 or FP16, stored in LDS as 16-bit patterns.
template <bool HALF>
struct Limb;
template <>
struct Limb<false> {
    typedef __bf16 t;
    __device__ static short bits(float x, float &back) {
        const __bf16 h = (__bf16)x;  // round to nearest even
        back = (float)h;
        return __builtin_bit_cast(short, h);
    }
    // D(16x16) += A(16x32) B(32x16): lane l supplies A[l%16][8(l/16) .. 8(l/16)+7] and
    // B[8(l/16) .. 8(l/16)+7][l%16]; accumulator element v of lane l is D[4(l/16)+v][l%16].
    __device__ static f4v mma(s8v a, s8v b, f4v c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a), __builtin_bit_cast(bf8v, b), c,
                                                       0, 0, 0);
    }
};
template <>
struct Limb<true> {
    typedef _Float16 t;
    __device__ static short bits(float x, float &back) {
        const _Float16 h = (_Float16)x;
        back = (float)h;
        return __builtin_bit_cast(short, h);
    }
    __device__ static f4v mma(s8v a, s8v b, f4v c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8v, a), __builtin_bit_cast(h8v, b), c, 0,
                                                      0, 0);
    }
};

struct SArgs {
    const float *A;   // m x k, row-major (lda)
    const float *Bt;  // n x k, row-major (ldbt): the transpose of B
    float *out;
    int64_t lda, ldbt, ldo;
    int64_t m, k, n;
    int64_t mb, kb, nb;
    int64_t leaf_stride;
    int tiles_m, tiles_n;
    const LeafEntry *leaves;
    const SrcEntry *asrc;
    const SrcEntry *bsrc;
    ScaleExps sc;
    int vec_a, vec_b;
};

__device__ inline int64_t remap_xcd(int64_t b, int64_t G) {
    const int64_t x = b % kXcd, j = b / kXcd;
    const int64_t per = G / kXcd, rem = G % kXcd;
    return ((x < rem) ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + j;
}

// NL limbs of format HALF; NP = number of limb products kept (1, 3 or 6).
template <bool HALF, int NL, bool SCALED, bool DIRECT>
__global__ __launch_bounds__(kNT, 1) void fmm_leaf_split(SArgs p) {
    typedef Limb<HALF> LB;
    constexpr int BM = 128, BN = 128, BK = 32, VEC = 4;
    constexpr int TPR = BK / VEC, RPP = kNT / TPR, NPASS = BM / RPP;  // 8 threads/row, 32 rows/pass
    constexpr int LDS_S = BK + 8;                                       // 80-byte rows: b128 reads conflict-free
    constexpr int WM = 64, WN = 64, TM = WM / 16, TN = WN / 16;
    static_assert(BM == BN, "square tile");

    __shared__ __attribute__((aligned(16))) short As[2][NL][BM * LDS_S];
    __shared__ __attribute__((aligned(16))) short Bs[2][NL][BN * LDS_S];

    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t tiles = (int64_t)p.tiles_m * p.tiles_n;
    const int bid = __builtin_amdgcn_readfirstlane((int)remap_xcd(blockIdx.x, gridDim.x));
    const int leaf = __builtin_amdgcn_readfirstlane((int)(bid / tiles));
    const int rem = __builtin_amdgcn_readfirstlane((int)(bid - (int64_t)leaf * tiles));
    // Grouped tile order: 8 tile-rows at a time, column by column inside the group, so the
    // work-groups resident on one XCD share A row panels and B column panels in its L2.
    const int grp = rem / (8 * p.tiles_n);
    const int gsz = min(8, p.tiles_m - grp * 8);
    const int gidx = rem - grp * 8 * p.tiles_n;
    const int64_t tm = __builtin_amdgcn_readfirstlane(grp * 8 + gidx % gsz);
    const int64_t tn = __builtin_amdgcn_readfirstlane(gidx / gsz);
    LeafEntry le = p.leaves[leaf];
    le.a_begin = __builtin_amdgcn_readfirstlane(le.a_begin);
    le.a_count = __builtin_amdgcn_readfirstlane(le.a_count);
    le.b_begin = __builtin_amdgcn_readfirstlane(le.b_begin);
    le.b_count = __builtin_amdgcn_readfirstlane(le.b_count);

    const int rr = t / TPR, kc = (t % TPR) * VEC;  // row within pass, k offset

    // Part of one source block of A (rows of S) or of B^T (rows of T^T) at K offset k0.
    //   A:  operand row = br*mb + tm*BM + r  (< m),  column = bc*kb + k0 + kc (< k)
    //   Bt: operand row = bc*nb + tn*BN + r  (< n),  column = br*kb + k0 + kc (< k)
    auto load_src = [&](bool isA, const SrcEntry &se, int64_t k0, float (&v)[NPASS][VEC]) {
        const float *base = isA ? p.A : p.Bt;
        const int64_t ld = isA ? p.lda : p.ldbt;
        const int64_t rows_blk = isA ? p.mb : p.nb, rows_all = isA ? p.m : p.n;
        const int64_t t0 = isA ? tm : tn;
        const int64_t row0 = (int64_t)(isA ? se.br : se.bc) * rows_blk + t0 * BM;
        const int64_t col0 = (int64_t)(isA ? se.bc : se.br) * p.kb + k0 + kc;
        const bool full = (isA ? p.vec_a : p.vec_b) && (k0 + BK <= p.kb) &&
                          ((int64_t)(isA ? se.bc : se.br) * p.kb + k0 + BK <= p.k);
        if (full) {
#pragma unroll
            for (int ps = 0; ps < NPASS; ++ps) {
                const int r = ps * RPP + rr;
                const bool rok = (t0 * BM + r < rows_blk) && (row0 + r < rows_all);
                const float *src = rok ? base + (row0 + r) * ld + col0 : base;
                const float4 x = *reinterpret_cast<const float4 *>(__builtin_assume_aligned(src, 16));
                v[ps][0] = rok ? x.x : 0.f, v[ps][1] = rok ? x.y : 0.f;
                v[ps][2] = rok ? x.z : 0.f, v[ps][3] = rok ? x.w : 0.f;
            }
        } else {
#pragma unroll
            for (int ps = 0; ps < NPASS; ++ps) {
                const int r = ps * RPP + rr;
                const bool rok = (t0 * BM + r < rows_blk) && (row0 + r < rows_all);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const bool ok = rok && (k0 + kc + e < p.kb) && (col0 + e < p.k);
                    const float x = *(ok ? base + (row0 + r) * ld + col0 + e : base);
                    v[ps][e] = ok ? x : 0.f;
                }
            }
        }
        if (SCALED) {
            // A' = diag(2^-ea) A diag(2^ep);  B'^T = diag(2^-eb) B^T diag(2^-ep)
#pragma unroll
            for (int ps = 0; ps < NPASS; ++ps) {
                const int r = ps * RPP + rr;
                const bool rok = (t0 * BM + r < rows_blk) && (row0 + r < rows_all);
                const int er = isA ? p.sc.ea[rok ? row0 + r : 0] : p.sc.eb[rok ? row0 + r : 0];
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const bool cok = col0 + e < p.k;
                    const int ec = p.sc.ep[cok ? col0 + e : 0];
                    v[ps][e] = ldexpf(v[ps][e], isA ? ec - er : -ec - er);
                }
            }
        }
    };

    float sa[NPASS][VEC], sb[NPASS][VEC];
    float xa0[NPASS][VEC], xb0[NPASS][VEC], xa1[NPASS][VEC], xb1[NPASS][VEC];

    auto prefetch = [&](int64_t k0) {
        load_src(true, p.asrc[le.a_begin], k0, xa0);
        if (le.a_count > 1) load_src(true, p.asrc[le.a_begin + 1], k0, xa1);
        load_src(false, p.bsrc[le.b_begin], k0, xb0);
        if (le.b_count > 1) load_src(false, p.bsrc[le.b_begin + 1], k0, xb1);
    };
    auto finish = [&](int64_t k0) {
        const float ca0 = p.asrc[le.a_begin].coef, cb0 = p.bsrc[le.b_begin].coef;
#pragma unroll
        for (int i = 0; i < NPASS; ++i)
#pragma unroll
            for (int e = 0; e < VEC; ++e) sa[i][e] = ca0 * xa0[i][e], sb[i][e] = cb0 * xb0[i][e];
        if (le.a_count > 1) {
            const float c = p.asrc[le.a_begin + 1].coef;
#pragma unroll
            for (int i = 0; i < NPASS; ++i)
#pragma unroll
                for (int e = 0; e < VEC; ++e) sa[i][e] = sa[i][e] + c * xa1[i][e];
        }
        if (le.b_count > 1) {
            const float c = p.bsrc[le.b_begin + 1].coef;
#pragma unroll
            for (int i = 0; i < NPASS; ++i)
#pragma unroll
                for (int e = 0; e < VEC; ++e) sb[i][e] = sb[i][e] + c * xb1[i][e];
        }
        for (int q = 2; q < le.a_count; ++q) {
            const SrcEntry se = p.asrc[le.a_begin + q];
            load_src(true, se, k0, xa0);
#pragma unroll
            for (int i = 0; i < NPASS; ++i)
#pragma unroll
                for (int e = 0; e < VEC; ++e) sa[i][e] = sa[i][e] + se.coef * xa0[i][e];
        }
        for (int q = 2; q < le.b_count; ++q) {
            const SrcEntry se = p.bsrc[le.b_begin + q];
            load_src(false, se, k0, xb0);
#pragma unroll
            for (int i = 0; i < NPASS; ++i)
#pragma unroll
                for (int e = 0; e < VEC; ++e) sb[i][e] = sb[i][e] + se.coef * xb0[i][e];
        }
    };
    // Split the formed S/T values into limbs and write them to LDS stage s.
    auto store = [&](int s) {
#pragma unroll
        for (int ps = 0; ps < NPASS; ++ps) {
            s4v la[NL], lb[NL];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                float ra = sa[ps][e], rb = sb[ps][e];
#pragma unroll
                for (int l = 0; l < NL; ++l) {
                    float ba, bb;
                    la[l][e] = LB::bits(ra, ba);
                    lb[l][e] = LB::bits(rb, bb);
                    ra = ra - ba;  // exact: the residual of a round-to-nearest is representable
                    rb = rb - bb;
                }
            }
            const int off = (ps * RPP + rr) * LDS_S + kc;
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                *reinterpret_cast<s4v *>(&As[s][l][off]) = la[l];
                *reinterpret_cast<s4v *>(&Bs[s][l][off]) = lb[l];
            }
        }
    };

    f4v acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};

    const int64_t nk = (p.kb + BK - 1) / BK;
    prefetch(0);
    finish(0);
    store(0);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        const bool more = kt + 1 < nk;
        if (more) prefetch((kt + 1) * BK);
        const int fo = (lane >> 4) * 8;  // k offset of this lane's 8-element fragment
        s8v a[NL][TM], b[NL][TN];
#pragma unroll
        for (int l = 0; l < NL; ++l) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
                a[l][i] = *reinterpret_cast<const s8v *>(&As[cur][l][(wm * WM + i * 16 + (lane & 15)) * LDS_S + fo]);
#pragma unroll
            for (int j = 0; j < TN; ++j)
                b[l][j] = *reinterpret_cast<const s8v *>(&Bs[cur][l][(wn * WN + j * 16 + (lane & 15)) * LDS_S + fo]);
        }
        // Limb products, smallest terms first: (NL=2) x2y1, x1y2, x1y1;
        // (NL=3) x3y1, x2y2, x1y3, x2y1, x1y2, x1y1.
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                if constexpr (NL == 3) {
                    acc[i][j] = LB::mma(a[2][i], b[0][j], acc[i][j]);
                    acc[i][j] = LB::mma(a[1][i], b[1][j], acc[i][j]);
                    acc[i][j] = LB::mma(a[0][i], b[2][j], acc[i][j]);
                }
                if constexpr (NL >= 2) {
                    acc[i][j] = LB::mma(a[1][i], b[0][j], acc[i][j]);
                    acc[i][j] = LB::mma(a[0][i], b[1][j], acc[i][j]);
                }
            }
        if (more) {
            finish((kt + 1) * BK);
            store(cur ^ 1);
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = LB::mma(a[0][i], b[0][j], acc[i][j]);
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = tm * BM + wm * WM + i * 16 + 4 * (lane >> 4) + v;
                const int64_t col = tn * BN + wn * WN + j * 16 + (lane & 15);
                float val = acc[i][j][v];
                if (DIRECT) {
                    if (row < p.m && col < p.n) {
                        if (SCALED) val = ldexpf(val, p.sc.ea[row] + p.sc.eb[col]);
                        p.out[row * p.ldo + col] = val;
                    }
                } else {
                    if (row < p.mb && col < p.nb) p.out[(int64_t)leaf * p.leaf_stride + row * p.ldo + col] = val;
                }
            }
}

// out (C x R, row-major ldo) = in^T where in is R x C row-major (ldi); 32x32 tiles via LDS.
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T *in, int64_t ldi, int64_t R, int64_t C, T *out,
                                                        int64_t ldo) {
    __shared__ T tile[32][33];
    const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
#pragma unroll
    for (int i = 0; i < 32; i += 8) {
        const int64_t r = r0 + ty + i, c = c0 + tx;
        if (r < R && c < C) tile[ty + i][tx] = in[r * ldi + c];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 32; i += 8) {
        const int64_t c = c0 + ty + i, r = r0 + tx;
        if (r < R && c < C) out[c * ldo + r] = tile[tx][ty + i];
    }
}

template <bool HALF, int NL>
hipError_t split_go(const SArgs &a, int64_t blocks, bool scaled, bool direct, hipStream_t s) {
    dim3 grid((unsigned)blocks), block(kNT);
    if (direct) {
        if (scaled) hipLaunchKernelGGL((fmm_leaf_split<HALF, NL, true, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((fmm_leaf_split<HALF, NL, false, true>), grid, block, 0, s, a);
    } else {
        if (scaled) hipLaunchKernelGGL((fmm_leaf_split<HALF, NL, true, false>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((fmm_leaf_split<HALF, NL, false, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_transpose_f32(const float *in, int64_t ldi, int64_t R, int64_t C, float *out, int64_t ldo,
                                hipStream_t s) {
    if (R <= 0 || C <= 0) return hipSuccess;
    if ((C + 31) / 32 > 0x7fffffffLL || (R + 31) / 32 > 65535) return hipErrorInvalidValue;
    dim3 grid((unsigned)((C + 31) / 32), (unsigned)((R + 31) / 32));
    hipLaunchKernelGGL(transpose_kernel<float>, grid, dim3(256), 0, s, in, ldi, R, C, out, ldo);
    return hipGetLastError();
}

hipError_t launch_transpose(Elem e, const void *in, int64_t ldi, int64_t R, int64_t C, void *out, int64_t ldo,
                            hipStream_t s) {
    if (e == Elem::F32) return launch_transpose_f32((const float *)in, ldi, R, C, (float *)out, ldo, s);
    if (R <= 0 || C <= 0) return hipSuccess;
    if ((C + 31) / 32 > 0x7fffffffLL || (R + 31) / 32 > 65535) return hipErrorInvalidValue;
    dim3 grid((unsigned)((C + 31) / 32), (unsigned)((R + 31) / 32));
    hipLaunchKernelGGL(transpose_kernel<double>, grid, dim3(256), 0, s, (const double *)in, ldi, R, C,
                       (double *)out, ldo);
    return hipGetLastError();
}

hipError_t launch_leaf_split(const LeafLaunch &L, const float *Bt, int64_t ldbt, hipStream_t s) {
    SArgs a;
    a.A = (const float *)L.A;
    a.Bt = Bt;
    a.out = (float *)L.out;
    a.lda = L.lda, a.ldbt = ldbt, a.ldo = L.ldo;
    a.m = L.m, a.k = L.k, a.n = L.n;
    a.mb = L.mb, a.kb = L.kb, a.nb = L.nb;
    a.leaf_stride = L.leaf_stride;
    a.tiles_m = (int)((L.mb + 127) / 128);
    a.tiles_n = (int)((L.nb + 127) / 128);
    a.leaves = L.leaves, a.asrc = L.asrc, a.bsrc = L.bsrc;
    a.sc = L.sc;
    a.vec_a = ((uintptr_t)L.A % 16 == 0) && (L.lda % 4 == 0) && (L.kb % 4 == 0);
    a.vec_b = ((uintptr_t)Bt % 16 == 0) && (ldbt % 4 == 0) && (L.kb % 4 == 0);
    const int64_t blocks = (int64_t)a.tiles_m * a.tiles_n * L.nleaves;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const bool scaled = L.sc.ea != nullptr, direct = L.direct != 0;
    switch (L.prec) {
        case FASTMM_BF16: return split_go<false, 1>(a, blocks, scaled, direct, s);
        case FASTMM_F16: return split_go<true, 1>(a, blocks, scaled, direct, s);
        case FASTMM_BF16X3: return split_go<false, 2>(a, blocks, scaled, direct, s);
        case FASTMM_F16X3: return split_go<true, 2>(a, blocks, scaled, direct, s);
        case FASTMM_BF16X6: return split_go<false, 3>(a, blocks, scaled, direct, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace fastmm
