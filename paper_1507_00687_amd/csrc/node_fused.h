// Fused one-level kernel for <2,2,2;7> rules with coefficients in {0, +1, -1} (Strassen's rule,
// Winograd's variant, their cyclic rotations and the transposes of those), FP64 and FP32 on
// MFMA.  The kernel template; node_fused.hip and node_fused_t.hip instantiate it for their sign
// patterns (two translation units, compiled in parallel).
//
// The innermost recursion level is done entirely inside one launch.  A work-group owns one
// 64x64 (FP32) or 64x32 (FP64) tile position (tm, tn) of the four output sub-blocks of one node
// of the recursion tree (the node is the whole problem at depth 1; at depth L it is one of the
// R^(L-1) products of the outer levels).  Per K stage it loads the matching tiles of the node's
// four A sub-blocks and four B sub-blocks into LDS once -- one source block per node operand:
// the operands themselves at depth 1, the node operands written by the outer levels' formation
// from depth 2 -- and then, for every product r, forms the
// MFMA fragments of S_r = sum_i u_ir A_i and T_r = sum_j v_jr B_j (eq. (1)) from those LDS
// tiles and accumulates M_r = S_r T_r in registers.  The epilogue forms C_k = sum_r w_kr M_r
// (eq. (1)) and writes each element of the node's output once: into C with the outside-scaling
// factors at depth 1, else into the node's workspace slot for the outer W-combination.  Each
// loaded tile serves all seven products, and the seven M_r never reach memory.  Scaled plans
// hand the kernel operands already scaled (one copy pass before the launch); the kernel applies
// only the output factors 2^(ea_i + eb_j).
//
// The sign pattern of the rule is a template argument (bit s*7+r of the P / N masks marks
// coefficient +1 / -1 in row s, column r), so every fragment sum is straight-line code.
// Single indices follow eq. (1): A and B sub-blocks column-major, C sub-blocks row-major.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "devtypes.h"
#include "launch.h"

namespace fastmm {
namespace {

typedef double nd4 __attribute__((ext_vector_type(4)));
typedef float nf4 __attribute__((ext_vector_type(4)));
constexpr int kNT = 256;
constexpr int kXcds = 8;

template <typename T>
struct NCore;
template <>
struct NCore<double> {
    typedef nd4 acc_t;
    typedef double2 vec_t;
    static constexpr int VEC = 2, OCC = 1, BK = 16, TN = 2;
    __device__ static acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // output row (inside the 16x16 block) of accumulator element v of `lane`
    __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
    __device__ static double scale(double x, int e) { return ldexp(x, e); }
};
template <>
struct NCore<float> {
    typedef nf4 acc_t;
    typedef float4 vec_t;
    static constexpr int VEC = 4, OCC = 2, BK = 16, TN = 2;
    __device__ static acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
    __device__ static float scale(float x, int e) { return ldexpf(x, e); }
};

template <typename T>
struct NArgs {
    const T *A;
    const T *B;
    T *out;
    int64_t lda, ldb, ldo;
    int64_t m, k, n;
    int64_t mb, kb, nb;  // sub-block sizes (the leaf block of the full recursion)
    int tiles_m, tiles_n;
    const LeafEntry *outer;  // per node: its one A and one B source (blocks of 2mb x 2kb, 2kb x 2nb),
                             // coefficient 1
    const SrcEntry *asrc;
    const SrcEntry *bsrc;
    int64_t node_stride;  // elements between node products in the workspace
    ScaleExps sc;
    int vec_a, vec_b;  // 16-byte loads allowed (alignment of pointers, ld and block sizes)
    int small_ld;      // a 64-row tile of A and a BK-row tile of B span < 2^31 bytes
};

// Coefficient of row s, column r of a {0, +1, -1} pattern.
template <uint32_t P, uint32_t N>
__device__ constexpr int cf(int s, int r) {
    return ((P >> (s * 7 + r)) & 1u) ? 1 : (((N >> (s * 7 + r)) & 1u) ? -1 : 0);
}

// sum_s c_sr e[s] in ascending s: the first term is +-e, the others are added or subtracted.
template <uint32_t P, uint32_t N, typename T>
__device__ __forceinline__ T psum(int r, const T (&e)[4]) {
    T a = T(0);
    bool first = true;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int c = cf<P, N>(s, r);
        if (c == 0) continue;
        if (first) a = (c > 0) ? e[s] : -e[s];
        else a = (c > 0) ? a + e[s] : a - e[s];
        first = false;
    }
    return a;
}

// A wave-uniform 64-bit value, kept in scalar registers.
__device__ __forceinline__ int64_t uniform64(int64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ inline int64_t xcd_remap(int64_t b, int64_t G) {
    const int64_t x = b % kXcds, j = b / kXcds;
    const int64_t per = G / kXcds, rem = G % kXcds;
    return ((x < rem) ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + j;
}

template <typename T, bool SCALED, uint32_t UP, uint32_t UN, uint32_t VP, uint32_t VN, uint32_t WP,
          uint32_t WN>
__global__ __launch_bounds__(kNT, NCore<T>::OCC) void fmm_node222(NArgs<T> p) {
    typedef NCore<T> C;
    typedef typename C::vec_t vec_t;
    constexpr int TM = 2, TN = C::TN;  // 16x16 MFMA blocks per wave and product
    constexpr int BM = 32 * TM, BN = 32 * TN, BK = C::BK, VEC = C::VEC;
    constexpr int KPL = BK / 4;  // consecutive k per lane group and stage
    constexpr int TPRA = BK / VEC, RPPA = kNT / TPRA, NPA = BM / RPPA;  // A: threads/row, rows/pass
    // B is loaded in VEC x VEC blocks (VEC k-rows by VEC columns) and stored transposed, one
    // 16-byte LDS write per column; consecutive lanes take consecutive k-blocks, which keeps
    // both the global reads (whole row segments) and the LDS writes free of conflicts.
    constexpr int KBV = BK / VEC, CBV = BN / VEC, NBT = 4 * KBV * CBV / kNT;  // B: blocks per thread
    // LDS tiles are k-contiguous for both operands (B stored transposed).  FP32: rows of 16
    // floats (64 bytes, four 16-byte chunks); row r is kept at row q = r ^ ((r / 4) mod 4) (a
    // permutation inside each aligned group of four rows) with its chunk c at chunk
    // c ^ ((q / 2) mod 4).  Measured with SQ_LDS_BANK_CONFLICT on MI355X, this layout is free of
    // bank conflicts for the three access patterns here: the 16-row fragment reads (one chunk per
    // 16 lanes), the row-major A writes (four lanes per row) and the transposed B writes (rows
    // c, c + 4, c + 8, ... of one column offset); without the row permutation the B writes take
    // two extra cycles each, and with padded rows the reads take one.  FP64: rows padded to a
    // 16-byte multiple that spreads consecutive rows over the banks.  lidx(r, k): element (row r,
    // k) for k a multiple of VEC.
    constexpr bool SWZ = sizeof(T) == 4;
    constexpr int LDS_K = SWZ ? BK : BK + 16 / (int)sizeof(T);
    auto lidx = [](int r, int k) {
        if constexpr (SWZ) {
            const int q = r ^ ((r >> 2) & 3);
            return q * LDS_K + (((k / VEC) ^ ((q >> 1) & 3)) * VEC);
        } else {
            return r * LDS_K + k;
        }
    };
    // lidx(r16 + r, k) = lbase(r16) + lidx(r, k) for r16 a multiple of 16: the lane parts are
    // computed once, the rest is a constant offset.
    auto lbase = [](int r16) { return r16 * LDS_K; };
    static_assert((LDS_K * sizeof(T)) % 16 == 0 && KPL % VEC == 0, "row alignment");

    // one stage's A and B tiles side by side
    struct Stage {
        __attribute__((aligned(16))) T a[4][BM * LDS_K];
        __attribute__((aligned(16))) T b[4][BN * LDS_K];
    };
    __shared__ Stage stg[2];

    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t tiles = (int64_t)p.tiles_m * p.tiles_n;
    const int bid = __builtin_amdgcn_readfirstlane((int)xcd_remap(blockIdx.x, gridDim.x));
    const int node = __builtin_amdgcn_readfirstlane((int)(bid / tiles));
    const int rem = __builtin_amdgcn_readfirstlane((int)(bid - (int64_t)node * tiles));
    // grouped order: 8 tile rows per group, so consecutive work-groups share B panels
    const int grp = rem / (8 * p.tiles_n);
    const int gsz = min(8, p.tiles_m - grp * 8);
    const int gidx = rem - grp * 8 * p.tiles_n;
    const int64_t tm = __builtin_amdgcn_readfirstlane(grp * 8 + gidx % gsz);
    const int64_t tn = __builtin_amdgcn_readfirstlane(gidx / gsz);
    // The node's one A source and one B source (coefficient 1): block row / column of the node
    // operand in the stacked or plain operand.
    const LeafEntry le = p.outer[node];
    const SrcEntry sa = p.asrc[le.a_begin], sbs = p.bsrc[le.b_begin];
    const int64_t abr = __builtin_amdgcn_readfirstlane(sa.br), abc = __builtin_amdgcn_readfirstlane(sa.bc);
    const int64_t bbr = __builtin_amdgcn_readfirstlane(sbs.br), bbc = __builtin_amdgcn_readfirstlane(sbs.bc);

    const int ra = t / TPRA, ka = (t % TPRA) * VEC;   // A: row within pass, k offset
    int sB[NBT], kB[NBT], cB[NBT];  // B: the thread's blocks (sub-block, k offset, column offset)
#pragma unroll
    for (int u = 0; u < NBT; ++u) {
        const int idx = t + kNT * u, b = idx % (KBV * CBV);
        sB[u] = idx / (KBV * CBV), kB[u] = (b % KBV) * VEC, cB[u] = (b / KBV) * VEC;
    }
    const int64_t mb2 = 2 * p.mb, kb2 = 2 * p.kb, nb2 = 2 * p.nb;
    // first row and column of the work-group's tile in sub-block s4 (A: s4 = p + 2q for
    // sub-block (p, q); B likewise), k offset 0; uniform, recomputed where used
    auto rowA = [&](int s4) { return abr * mb2 + (s4 & 1) * p.mb + tm * BM; };
    auto colA = [&](int s4) { return abc * kb2 + (s4 >> 1) * p.kb; };
    auto rowB = [&](int s4) { return bbr * kb2 + (s4 & 1) * p.kb; };
    auto colB = [&](int s4) { return bbc * nb2 + (s4 >> 1) * p.nb + tn * BN; };

    // Stages with k0 + BK <= kfast read whole tiles with vector loads and no bounds checks:
    // every tile of this work-group lies inside its sub-block and inside the operand.
    int64_t kfast = (p.vec_a && p.vec_b && p.small_ld && tm * BM + BM <= p.mb && tn * BN + BN <= p.nb) ? p.kb : 0;
    if (rowA(1) + BM > p.m || colB(2) + BN > p.n) kfast = 0;  // the last sub-block row / column
    kfast = min(kfast, min(p.k - colA(2), p.k - rowB(1)));
    kfast = __builtin_amdgcn_readfirstlane(kfast);
    // byte offsets of the thread's vectors inside a tile (the same for every sub-block and K
    // stage)
    uint32_t voA[NPA], voB[NBT];
#pragma unroll
    for (int pa = 0; pa < NPA; ++pa) voA[pa] = (uint32_t)(((pa * RPPA + ra) * p.lda + ka) * sizeof(T));
#pragma unroll
    for (int u = 0; u < NBT; ++u) voB[u] = (uint32_t)((kB[u] * p.ldb + cB[u]) * sizeof(T));

    // The thread's part of the A tiles of the four node sub-blocks at K offset k0, zero outside
    // A and the sub-block.
    auto load_a_one = [&](int64_t k0, T (&v)[4][NPA][VEC]) {
        const bool fast = k0 + BK <= kfast;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int64_t row0 = rowA(s4), cbase = colA(s4) + k0;
            if (fast) {
                const char *base = reinterpret_cast<const char *>(p.A + uniform64(row0 * p.lda + cbase));
#pragma unroll
                for (int pa = 0; pa < NPA; ++pa) {
                    const vec_t w = *reinterpret_cast<const vec_t *>(__builtin_assume_aligned(base + voA[pa], 16));
                    const T *ws = reinterpret_cast<const T *>(&w);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) v[s4][pa][e] = ws[e];
                }
            } else {
#pragma unroll
                for (int pa = 0; pa < NPA; ++pa) {
                    const int r = pa * RPPA + ra;
                    const bool rok = (tm * BM + r < p.mb) && (row0 + r < p.m);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const bool ok = rok && (k0 + ka + e < p.kb) && (cbase + ka + e < p.k);
                        const T y = *(ok ? p.A + (row0 + r) * p.lda + cbase + ka + e : p.A);
                        v[s4][pa][e] = ok ? y : T(0);
                    }
                }
            }
        }
    };
    // The thread's B blocks at K offset k0, zero outside B and the sub-block.
    auto load_b_one = [&](int64_t k0, T (&v)[NBT][VEC][VEC]) {
        const bool fast = k0 + BK <= kfast;
#pragma unroll
        for (int u = 0; u < NBT; ++u) {
            const int sb = sB[u];
            const int64_t row0 = rowB(sb) + k0, cbase = colB(sb);  // k-row of block row 0, tile column 0
            if (fast) {
                const char *base = reinterpret_cast<const char *>(p.B + uniform64(row0 * p.ldb + cbase)) + voB[u];
#pragma unroll
                for (int vr = 0; vr < VEC; ++vr) {
                    const vec_t w = *reinterpret_cast<const vec_t *>(
                        __builtin_assume_aligned(base + (size_t)vr * p.ldb * sizeof(T), 16));
                    const T *ws = reinterpret_cast<const T *>(&w);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) v[u][vr][e] = ws[e];
                }
            } else {
#pragma unroll
                for (int vr = 0; vr < VEC; ++vr) {
                    const int kr = kB[u] + vr;
                    const bool rok = (k0 + kr < p.kb) && (row0 + kr < p.k);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const int cc = cB[u] + e;
                        const bool ok = rok && (tn * BN + cc < p.nb) && (cbase + cc < p.n);
                        const T y = *(ok ? p.B + (row0 + kr) * p.ldb + cbase + cc : p.B);
                        v[u][vr][e] = ok ? y : T(0);
                    }
                }
            }
        }
    };
    // FP64 keeps the source-list form of the load stage (table entries read per stage): with the
    // tile origins kept across the loop, as in the FP32 form, its register budget (224 AGPR
    // accumulators) spills (measured 10-19 % slower); for FP32 the origins in scalar registers and
    // no per-stage table reads took the kernel from 0.61 to 0.72 of the FP32 peak.
    // Stages with k0 + BK <= kfast read whole tiles with vector loads and no bounds checks:
    // every source tile of this work-group lies inside its sub-block and inside the operand.
    int64_t kfast_l = (p.vec_a && p.vec_b && p.small_ld && tm * BM + BM <= p.mb && tn * BN + BN <= p.nb) ? p.kb : 0;
    for (int q = 0; q < le.a_count && kfast_l > 0; ++q) {
        const SrcEntry se = p.asrc[le.a_begin + q];
        for (int s = 0; s < 4; ++s) {
            if ((int64_t)se.br * mb2 + (s & 1) * p.mb + tm * BM + BM > p.m) kfast_l = 0;
            kfast_l = min(kfast_l, p.k - ((int64_t)se.bc * kb2 + (s >> 1) * p.kb));
        }
    }
    for (int q = 0; q < le.b_count && kfast_l > 0; ++q) {
        const SrcEntry se = p.bsrc[le.b_begin + q];
        for (int s = 0; s < 4; ++s) {
            if ((int64_t)se.bc * nb2 + (s >> 1) * p.nb + tn * BN + BN > p.n) kfast_l = 0;
            kfast_l = min(kfast_l, p.k - ((int64_t)se.br * kb2 + (s & 1) * p.kb));
        }
    }
    kfast_l = __builtin_amdgcn_readfirstlane(kfast_l);
    // byte offsets of the thread's vectors inside a tile (the same for every source, sub-block
    // and K stage)

    // The thread's part of the A tiles of the four node sub-blocks at K offset k0: the sum over
    // the node's sources of coef * A, zero outside A and the sub-block.
    auto load_a_list = [&](int64_t k0, T (&v)[4][NPA][VEC]) {
        const bool fast = k0 + BK <= kfast_l;
        for (int q = 0; q < le.a_count; ++q) {
            const SrcEntry se = p.asrc[le.a_begin + q];
            const T c = (T)se.coef;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int64_t row0 = (int64_t)se.br * mb2 + (s & 1) * p.mb + tm * BM;
                const int64_t cbase = (int64_t)se.bc * kb2 + (s >> 1) * p.kb + k0;
                T x[NPA][VEC];
                if (fast) {
                    const char *base = reinterpret_cast<const char *>(p.A + row0 * p.lda + cbase);
#pragma unroll
                    for (int pa = 0; pa < NPA; ++pa) {
                        const vec_t w = *reinterpret_cast<const vec_t *>(__builtin_assume_aligned(base + voA[pa], 16));
                        const T *ws = reinterpret_cast<const T *>(&w);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) x[pa][e] = ws[e];
                    }
                } else {
#pragma unroll
                    for (int pa = 0; pa < NPA; ++pa) {
                        const int r = pa * RPPA + ra;
                        const bool rok = (tm * BM + r < p.mb) && (row0 + r < p.m);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            const bool ok = rok && (k0 + ka + e < p.kb) && (cbase + ka + e < p.k);
                            const T y = *(ok ? p.A + (row0 + r) * p.lda + cbase + ka + e : p.A);
                            x[pa][e] = ok ? y : T(0);
                        }
                    }
                }
#pragma unroll
                for (int pa = 0; pa < NPA; ++pa)
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        v[s][pa][e] = (q == 0) ? c * x[pa][e] : v[s][pa][e] + c * x[pa][e];
            }
        }
    };
    // The thread's B blocks at K offset k0: the sum over the node's sources of coef * B, zero
    // outside B and the sub-block.
    auto load_b_list = [&](int64_t k0, T (&v)[NBT][VEC][VEC]) {
        const bool fast = k0 + BK <= kfast_l;
        for (int q = 0; q < le.b_count; ++q) {
            const SrcEntry se = p.bsrc[le.b_begin + q];
            const T c = (T)se.coef;
#pragma unroll
            for (int u = 0; u < NBT; ++u) {
                const int sb = sB[u];
                const int64_t row0 = (int64_t)se.br * kb2 + (sb & 1) * p.kb + k0;        // k-row of block row 0
                const int64_t cbase = (int64_t)se.bc * nb2 + (sb >> 1) * p.nb + tn * BN;  // column of tile column 0
                T x[VEC][VEC];
                if (fast) {
                    const char *base = reinterpret_cast<const char *>(p.B + row0 * p.ldb + cbase) + voB[u];
#pragma unroll
                    for (int vr = 0; vr < VEC; ++vr) {
                        const vec_t w = *reinterpret_cast<const vec_t *>(
                            __builtin_assume_aligned(base + (size_t)vr * p.ldb * sizeof(T), 16));
                        const T *ws = reinterpret_cast<const T *>(&w);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) x[vr][e] = ws[e];
                    }
                } else {
#pragma unroll
                    for (int vr = 0; vr < VEC; ++vr) {
                        const int kr = kB[u] + vr;
                        const bool rok = (k0 + kr < p.kb) && (row0 + kr < p.k);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            const int cc = cB[u] + e;
                            const bool ok = rok && (tn * BN + cc < p.nb) && (cbase + cc < p.n);
                            const T y = *(ok ? p.B + (row0 + kr) * p.ldb + cbase + cc : p.B);
                            x[vr][e] = ok ? y : T(0);
                        }
                    }
                }
#pragma unroll
                for (int vr = 0; vr < VEC; ++vr)
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        v[u][vr][e] = (q == 0) ? c * x[vr][e] : v[u][vr][e] + c * x[vr][e];
            }
        }
    };
    auto load_a = [&](int64_t k0, T (&v)[4][NPA][VEC]) {
        if constexpr (SWZ) load_a_one(k0, v);
        else load_a_list(k0, v);
    };
    auto load_b = [&](int64_t k0, T (&v)[NBT][VEC][VEC]) {
        if constexpr (SWZ) load_b_one(k0, v);
        else load_b_list(k0, v);
    };
    static_assert(RPPA % 16 == 0, "pass rows");
    const int sto_a = lidx(ra, ka);
    int sto_b[NBT][VEC];
#pragma unroll
    for (int u = 0; u < NBT; ++u)
#pragma unroll
        for (int e = 0; e < VEC; ++e) sto_b[u][e] = lidx(cB[u] + e, kB[u]);
    auto store = [&](int st, const T (&va)[4][NPA][VEC], const T (&vb)[NBT][VEC][VEC]) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int pa = 0; pa < NPA; ++pa) {
                vec_t x;
                T *xs = reinterpret_cast<T *>(&x);
#pragma unroll
                for (int e = 0; e < VEC; ++e) xs[e] = va[s][pa][e];
                *reinterpret_cast<vec_t *>(&stg[st].a[s][lbase(pa * RPPA) + sto_a]) = x;
            }
        }
#pragma unroll
        for (int u = 0; u < NBT; ++u)
#pragma unroll
            for (int e = 0; e < VEC; ++e) {  // column cB + e, k-rows kB .. kB + VEC - 1
                vec_t x;
                T *xs = reinterpret_cast<T *>(&x);
#pragma unroll
                for (int vr = 0; vr < VEC; ++vr) xs[vr] = vb[u][vr][e];
                *reinterpret_cast<vec_t *>(&stg[st].b[sB[u]][sto_b[u][e]]) = x;
            }
    };

    typename C::acc_t acc[7][TM][TN];
#pragma unroll
    for (int r = 0; r < 7; ++r)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[r][i][j] = typename C::acc_t{};

    T va[4][NPA][VEC], vb[NBT][VEC][VEC];
    const int64_t nk = (p.kb + BK - 1) / BK;
    load_a(0, va);
    load_b(0, vb);
    store(0, va, vb);
    __syncthreads();
    // MFMA step j of a stage takes k = KPL g + j from lane group g = lane / 16, so each lane's
    // operands for the KPL steps are KPL consecutive k of one tile row: 16-byte LDS reads.
    const int g4 = KPL * (lane >> 4), l16 = lane & 15;
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        const bool more = kt + 1 < nk;
        if (more) {  // next stage's global loads overlap this stage's MFMA work
            load_a((kt + 1) * BK, va);
            load_b((kt + 1) * BK, vb);
        }
#pragma unroll
        for (int jh = 0; jh < KPL / VEC; ++jh) {
            const int rdo = lidx(l16, g4 + jh * VEC);
            T ea[TM][4][VEC], eb[TN][4][VEC];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const vec_t w = *reinterpret_cast<const vec_t *>(
                        &stg[cur].a[s][lbase(wm * 16 * TM + i * 16) + rdo]);
                    const T *ws = reinterpret_cast<const T *>(&w);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) ea[i][s][e] = ws[e];
                }
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const vec_t w = *reinterpret_cast<const vec_t *>(
                        &stg[cur].b[s][lbase(wn * 16 * TN + j * 16) + rdo]);
                    const T *ws = reinterpret_cast<const T *>(&w);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) eb[j][s][e] = ws[e];
                }
            }
#pragma unroll
            for (int e = 0; e < VEC; ++e)
#pragma unroll
                for (int r = 0; r < 7; ++r) {
                    T a[TM], b[TN];
#pragma unroll
                    for (int i = 0; i < TM; ++i) {
                        const T x[4] = {ea[i][0][e], ea[i][1][e], ea[i][2][e], ea[i][3][e]};
                        a[i] = psum<UP, UN>(r, x);
                    }
#pragma unroll
                    for (int j = 0; j < TN; ++j) {
                        const T x[4] = {eb[j][0][e], eb[j][1][e], eb[j][2][e], eb[j][3][e]};
                        b[j] = psum<VP, VN>(r, x);
                    }
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j) acc[r][i][j] = C::mma(a[i], b[j], acc[r][i][j]);
                }
        }
        if (more) store(cur ^ 1, va, vb);  // the other buffer was last read before the previous barrier
        __syncthreads();
    }

    // C_k = sum_r w_kr M_r for the four output sub-blocks (k row-major), each element written once.
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
        const int64_t rsub = (kc >> 1) * p.mb, csub = (kc & 1) * p.nb;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    T mr[7];
#pragma unroll
                    for (int r = 0; r < 7; ++r) mr[r] = acc[r][i][j][v];
                    T val = T(0);
                    bool first = true;
#pragma unroll
                    for (int r = 0; r < 7; ++r) {
                        const int c = cf<WP, WN>(kc, r);
                        if (c == 0) continue;
                        if (first) val = (c > 0) ? mr[r] : -mr[r];
                        else val = (c > 0) ? val + mr[r] : val - mr[r];
                        first = false;
                    }
                    const int64_t lr = tm * BM + wm * 16 * TM + i * 16 + C::row(lane, v);  // inside the sub-block
                    const int64_t lc = tn * BN + wn * 16 * TN + j * 16 + (lane & 15);
                    if (lr >= p.mb || lc >= p.nb) continue;
                    const int64_t row = rsub + lr, col = csub + lc;  // inside the node's output
                    if (p.node_stride == 0) {  // depth 1: the node is the whole product
                        if (row < p.m && col < p.n) {
                            if (SCALED) val = C::scale(val, p.sc.ea[row] + p.sc.eb[col]);
                            p.out[row * p.ldo + col] = val;
                        }
                    } else {
                        p.out[(int64_t)node * p.node_stride + row * nb2 + col] = val;
                    }
                }
    }
}

// Launch of the compiled pattern (UP .. WN); scaled: the depth-1 output takes 2^(ea_i + eb_j).
template <typename T, uint32_t UP, uint32_t UN, uint32_t VP, uint32_t VN, uint32_t WP, uint32_t WN>
hipError_t node_launch(const NArgs<T> &a, unsigned blocks, bool scaled, hipStream_t s) {
    if (scaled)
        hipLaunchKernelGGL((fmm_node222<T, true, UP, UN, VP, VN, WP, WN>), dim3(blocks), dim3(kNT), 0, s, a);
    else
        hipLaunchKernelGGL((fmm_node222<T, false, UP, UN, VP, VN, WP, WN>), dim3(blocks), dim3(kNT), 0, s, a);
    return hipGetLastError();
}

// Kernel arguments of a launch; blocks = 0 when there is nothing to do, -1 when the grid is too
// large.
template <typename T>
NArgs<T> node_args(const NodeLaunch &L, int64_t &blocks) {
    NArgs<T> a;
    a.A = (const T *)L.A;
    a.B = (const T *)L.B;
    a.out = (T *)L.out;
    a.lda = L.lda, a.ldb = L.ldb, a.ldo = L.ldo;
    a.m = L.m, a.k = L.k, a.n = L.n;
    a.mb = L.mb, a.kb = L.kb, a.nb = L.nb;
    constexpr int BN = 32 * NCore<T>::TN;
    a.tiles_m = (int)((L.mb + 63) / 64);
    a.tiles_n = (int)((L.nb + BN - 1) / BN);
    a.outer = L.outer, a.asrc = L.asrc, a.bsrc = L.bsrc;
    a.node_stride = L.node_stride;
    a.sc = L.sc;
    constexpr int VEC = NCore<T>::VEC;
    a.vec_a = ((uintptr_t)L.A % 16 == 0) && (L.lda % VEC == 0) && (L.kb % VEC == 0);
    a.vec_b = ((uintptr_t)L.B % 16 == 0) && (L.ldb % VEC == 0) && (L.nb % VEC == 0);
    a.small_ld = (64 * (L.lda + 8) * (int64_t)sizeof(T) < (int64_t(1) << 31)) &&
                 (16 * (L.ldb + 8) * (int64_t)sizeof(T) < (int64_t(1) << 31));
    blocks = (int64_t)a.tiles_m * a.tiles_n * L.nnodes;
    if (blocks > 0x7fffffffLL) blocks = -1;
    return a;
}

// Launch for the patterns listed by PATTERNS(X) (X(up, un, vp, vn, wp, wn) per pattern); sets
// *found to whether the plan's masks are among them.
#define FASTMM_NODE_DISPATCH(PATTERNS)                                                                   \
    template <typename T>                                                                              \
    hipError_t node_go(const NodeLaunch &L, hipStream_t s, bool *found) {                              \
        *found = false;                                                                                \
        const uint32_t *m = L.masks;                                                                   \
        int64_t blocks = 0;                                                                            \
        const NArgs<T> a = node_args<T>(L, blocks);                                                    \
        const bool scaled = L.sc.ea != nullptr;                                                        \
        PATTERNS(FASTMM_NODE_TRY)                                                                      \
        return hipErrorInvalidValue;                                                                   \
    }                                                                                                  \
    bool node_match(const uint32_t m[6]) {                                                             \
        PATTERNS(FASTMM_NODE_MATCH)                                                                    \
        return false;                                                                                  \
    }
#define FASTMM_NODE_TRY(up, un, vp, vn, wp, wn)                                                          \
    if (m[0] == up && m[1] == un && m[2] == vp && m[3] == vn && m[4] == wp && m[5] == wn) {             \
        *found = true;                                                                                 \
        if (blocks == 0) return hipSuccess;                                                            \
        if (blocks < 0) return hipErrorInvalidValue;                                                   \
        return node_launch<T, up, un, vp, vn, wp, wn>(a, (unsigned)blocks, scaled, s);                 \
    }
#define FASTMM_NODE_MATCH(up, un, vp, vn, wp, wn)                                                        \
    if (m[0] == up && m[1] == un && m[2] == vp && m[3] == vn && m[4] == wp && m[5] == wn) return true;

}  // namespace
}  // namespace fastmm
