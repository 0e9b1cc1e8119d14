// Fused one-level kernel for <2,2,2;7> rules with coefficients in {0, +1, -1} (Strassen's rule,
// Winograd's variant and their cyclic rotations), FP64 and FP32 on MFMA.
//
// The innermost recursion level is done entirely inside one launch.  A work-group owns one
// 64x64 tile position (tm, tn) of the four output sub-blocks of one node of the recursion tree
// (the node is the whole problem at depth 1; at depth L it is one of the R^(L-1) products of the
// outer levels).  Per K stage it loads the matching tiles of the node's four A sub-blocks and
// four B sub-blocks into LDS once -- each node operand being the sum of its outer-level sources,
// formed while loading with the scaling exponents applied -- and then, for every product r,
// forms the MFMA fragments of S_r = sum_i u_ir A_i and T_r = sum_j v_jr B_j (eq. (1)) from
// those LDS tiles and accumulates M_r = S_r T_r in registers.  The epilogue forms
// C_k = sum_r w_kr M_r (eq. (1)) and writes each element of the node's output once: into C with
// the outside-scaling factors at depth 1, else into the node's workspace slot for the outer
// W-combination.  Each loaded tile serves all seven products, and the seven M_r never reach
// memory.
//
// The sign pattern of the rule is a template argument (bit s*7+r of the P / N masks marks
// coefficient +1 / -1 in row s, column r), so every fragment sum is straight-line code.
// Single indices follow eq. (1): A and B sub-blocks column-major, C sub-blocks row-major.
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
    static constexpr int VEC = 2, OCC = 1;
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
    static constexpr int VEC = 4, OCC = 2;
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
    const LeafEntry *outer;  // per node: its operand sources (blocks of 2mb x 2kb, 2kb x 2nb)
    const SrcEntry *asrc;
    const SrcEntry *bsrc;
    int64_t node_stride;  // elements between node products in the workspace
    ScaleExps sc;
    int vec_a, vec_b;  // 16-byte loads allowed (alignment of pointers, ld and block sizes)
    int small_ld;      // 64 rows of A and 16 rows of B span < 2^31 bytes
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

__device__ inline int64_t xcd_remap(int64_t b, int64_t G) {
    const int64_t x = b % kXcds, j = b / kXcds;
    const int64_t per = G / kXcds, rem = G % kXcds;
    return ((x < rem) ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + j;
}

template <typename T, bool SCALED, uint32_t UP, uint32_t UN, uint32_t VP, uint32_t VN, uint32_t WP, uint32_t WN>
__global__ __launch_bounds__(kNT, NCore<T>::OCC) void fmm_node222(NArgs<T> p) {
    typedef NCore<T> C;
    typedef typename C::vec_t vec_t;
    constexpr int BM = 64, BN = 64, BK = 16, VEC = C::VEC;
    constexpr int TPRA = BK / VEC, RPPA = kNT / TPRA, NPA = BM / RPPA;  // A: threads/row, rows/pass
    constexpr int TPRB = BN / VEC, KPPB = kNT / TPRB, NPB = BK / KPPB;  // B: threads/k-row, k-rows/pass
    constexpr int LDA_S = BK + 1, LDB_S = BN + 16;
    constexpr int TM = 2, TN = 2;  // 16x16 MFMA blocks per wave and product (wave tile 32x32)
    static_assert(NPA * RPPA == BM && NPB * KPPB == BK, "tile shape");

    __shared__ T As[2][4][BM * LDA_S];
    __shared__ __attribute__((aligned(16))) T Bs[2][4][BK * LDB_S];

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
    LeafEntry le = p.outer[node];
    le.a_begin = __builtin_amdgcn_readfirstlane(le.a_begin);
    le.a_count = __builtin_amdgcn_readfirstlane(le.a_count);
    le.b_begin = __builtin_amdgcn_readfirstlane(le.b_begin);
    le.b_count = __builtin_amdgcn_readfirstlane(le.b_count);

    const int ra = t / TPRA, ka = (t % TPRA) * VEC;   // A: row within pass, k offset
    const int kbr = t / TPRB, cb = (t % TPRB) * VEC;  // B: k-row within pass, column offset
    const int64_t mb2 = 2 * p.mb, kb2 = 2 * p.kb, nb2 = 2 * p.nb;
    const bool a_rows_in = tm * BM + BM <= p.mb;
    const bool b_cols_in = tn * BN + BN <= p.nb;
    // byte offsets of the thread's vectors inside an interior tile (independent of the source,
    // the sub-block and the K stage)
    uint32_t voA[NPA], voB[NPB];
#pragma unroll
    for (int pa = 0; pa < NPA; ++pa) voA[pa] = (uint32_t)(((pa * RPPA + ra) * p.lda + ka) * sizeof(T));
#pragma unroll
    for (int pb = 0; pb < NPB; ++pb) voB[pb] = (uint32_t)(((pb * KPPB + kbr) * p.ldb + cb) * sizeof(T));

    // The thread's part of the A tiles of the four node sub-blocks at K offset k0: the sum over
    // the node's sources of coef * 2^(ep_col - ea_row) * A, zero outside A and the sub-block.
    auto load_a = [&](int64_t k0, T (&v)[4][NPA][VEC]) {
        const bool k_in = k0 + BK <= p.kb;
        for (int q = 0; q < le.a_count; ++q) {
            const SrcEntry se = p.asrc[le.a_begin + q];
            const T c = (T)se.coef;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int64_t row0 = (int64_t)se.br * mb2 + (s & 1) * p.mb + tm * BM;
                const int64_t cbase = (int64_t)se.bc * kb2 + (s >> 1) * p.kb + k0;
                T x[NPA][VEC];
                if (p.vec_a && p.small_ld && k_in && a_rows_in && cbase + BK <= p.k && row0 + BM <= p.m) {
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
                if (SCALED) {
#pragma unroll
                    for (int pa = 0; pa < NPA; ++pa) {
                        const int64_t row = row0 + pa * RPPA + ra;
                        const int er = p.sc.ea[row < p.m ? row : 0];
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            const int64_t col = cbase + ka + e;
                            x[pa][e] = C::scale(x[pa][e], p.sc.ep[col < p.k ? col : 0] - er);
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
    // Likewise for B: 2^(-ep_row - eb_col) * B.
    auto load_b = [&](int64_t k0, T (&v)[4][NPB][VEC]) {
        const bool k_in = k0 + BK <= p.kb;
        for (int q = 0; q < le.b_count; ++q) {
            const SrcEntry se = p.bsrc[le.b_begin + q];
            const T c = (T)se.coef;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int64_t row0 = (int64_t)se.br * kb2 + (s & 1) * p.kb + k0;
                const int64_t cbase = (int64_t)se.bc * nb2 + (s >> 1) * p.nb + tn * BN;
                T x[NPB][VEC];
                if (p.vec_b && p.small_ld && k_in && b_cols_in && cbase + BN <= p.n && row0 + BK <= p.k) {
                    const char *base = reinterpret_cast<const char *>(p.B + row0 * p.ldb + cbase);
#pragma unroll
                    for (int pb = 0; pb < NPB; ++pb) {
                        const vec_t w = *reinterpret_cast<const vec_t *>(__builtin_assume_aligned(base + voB[pb], 16));
                        const T *ws = reinterpret_cast<const T *>(&w);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) x[pb][e] = ws[e];
                    }
                } else {
#pragma unroll
                    for (int pb = 0; pb < NPB; ++pb) {
                        const int kr = pb * KPPB + kbr;
                        const bool rok = (k0 + kr < p.kb) && (row0 + kr < p.k);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            const bool ok = rok && (tn * BN + cb + e < p.nb) && (cbase + cb + e < p.n);
                            const T y = *(ok ? p.B + (row0 + kr) * p.ldb + cbase + cb + e : p.B);
                            x[pb][e] = ok ? y : T(0);
                        }
                    }
                }
                if (SCALED) {
#pragma unroll
                    for (int pb = 0; pb < NPB; ++pb) {
                        const int64_t row = row0 + pb * KPPB + kbr;
                        const int er = p.sc.ep[row < p.k ? row : 0];
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            const int64_t col = cbase + cb + e;
                            x[pb][e] = C::scale(x[pb][e], -er - p.sc.eb[col < p.n ? col : 0]);
                        }
                    }
                }
#pragma unroll
                for (int pb = 0; pb < NPB; ++pb)
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        v[s][pb][e] = (q == 0) ? c * x[pb][e] : v[s][pb][e] + c * x[pb][e];
            }
        }
    };
    auto store = [&](int st, const T (&va)[4][NPA][VEC], const T (&vb)[4][NPB][VEC]) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int pa = 0; pa < NPA; ++pa)
#pragma unroll
                for (int e = 0; e < VEC; ++e) As[st][s][(pa * RPPA + ra) * LDA_S + ka + e] = va[s][pa][e];
#pragma unroll
            for (int pb = 0; pb < NPB; ++pb) {
                vec_t x;
                T *xs = reinterpret_cast<T *>(&x);
#pragma unroll
                for (int e = 0; e < VEC; ++e) xs[e] = vb[s][pb][e];
                *reinterpret_cast<vec_t *>(&Bs[st][s][(pb * KPPB + kbr) * LDB_S + cb]) = x;
            }
        }
    };

    typename C::acc_t acc[7][TM][TN];
#pragma unroll
    for (int r = 0; r < 7; ++r)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[r][i][j] = typename C::acc_t{};

    T va[4][NPA][VEC], vb[4][NPB][VEC];
    const int64_t nk = (p.kb + BK - 1) / BK;
    load_a(0, va);
    load_b(0, vb);
    store(0, va, vb);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        const bool more = kt + 1 < nk;
        if (more) {  // next stage's global loads overlap this stage's MFMA work
            load_a((kt + 1) * BK, va);
            load_b((kt + 1) * BK, vb);
        }
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            T ea[TM][4], eb[TN][4];  // this lane's element of each sub-block tile, per 16-block
#pragma unroll
            for (int s = 0; s < 4; ++s) {
#pragma unroll
                for (int i = 0; i < TM; ++i)
                    ea[i][s] = As[cur][s][(wm * 32 + i * 16 + (lane & 15)) * LDA_S + ks + (lane >> 4)];
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    eb[j][s] = Bs[cur][s][(ks + (lane >> 4)) * LDB_S + wn * 32 + j * 16 + (lane & 15)];
            }
#pragma unroll
            for (int r = 0; r < 7; ++r) {
                T a[TM], b[TN];
#pragma unroll
                for (int i = 0; i < TM; ++i) a[i] = psum<UP, UN>(r, ea[i]);
#pragma unroll
                for (int j = 0; j < TN; ++j) b[j] = psum<VP, VN>(r, eb[j]);
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
                    const int64_t lr = tm * BM + wm * 32 + i * 16 + C::row(lane, v);  // inside the sub-block
                    const int64_t lc = tn * BN + wn * 32 + j * 16 + (lane & 15);
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

// The sign patterns with a compiled kernel: Strassen's rule, Winograd's variant and the two
// cyclic rotations of each, as the rule registry holds them ((U+, U-, V+, V-, W+, W-) masks).
// A rule is matched against them coefficient by coefficient, so a pattern is only ever used
// for a rule that equals it.
#define FASTMM_NODE222_PATTERNS(X)                                                     \
    X(0x1741115u, 0x8000020u, 0xa292423u, 0x0800008u, 0x4a28a49u, 0x0400010u)          \
    X(0x4a28a49u, 0x0400010u, 0x1741115u, 0x8000020u, 0xa292423u, 0x0800008u)          \
    X(0xa292423u, 0x0800008u, 0x4a28a49u, 0x0400010u, 0x1741115u, 0x8000020u)          \
    X(0x7019845u, 0x0802220u, 0xd840129u, 0x01a0410u, 0xe385a83u, 0x0020000u)          \
    X(0xe385a83u, 0x0020000u, 0x7019845u, 0x0802220u, 0xd840129u, 0x01a0410u)          \
    X(0xd840129u, 0x01a0410u, 0xe385a83u, 0x0020000u, 0x7019845u, 0x0802220u)

template <typename T, uint32_t UP, uint32_t UN, uint32_t VP, uint32_t VN, uint32_t WP, uint32_t WN>
hipError_t node_launch(const NArgs<T> &a, unsigned blocks, bool scaled, hipStream_t s) {
    if (scaled)
        hipLaunchKernelGGL((fmm_node222<T, true, UP, UN, VP, VN, WP, WN>), dim3(blocks), dim3(kNT), 0, s, a);
    else
        hipLaunchKernelGGL((fmm_node222<T, false, UP, UN, VP, VN, WP, WN>), dim3(blocks), dim3(kNT), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t node_go(const NodeLaunch &L, hipStream_t s) {
    NArgs<T> a;
    a.A = (const T *)L.A;
    a.B = (const T *)L.B;
    a.out = (T *)L.out;
    a.lda = L.lda, a.ldb = L.ldb, a.ldo = L.ldo;
    a.m = L.m, a.k = L.k, a.n = L.n;
    a.mb = L.mb, a.kb = L.kb, a.nb = L.nb;
    a.tiles_m = (int)((L.mb + 63) / 64);
    a.tiles_n = (int)((L.nb + 63) / 64);
    a.outer = L.outer, a.asrc = L.asrc, a.bsrc = L.bsrc;
    a.node_stride = L.node_stride;
    a.sc = L.sc;
    constexpr int VEC = NCore<T>::VEC;
    a.vec_a = ((uintptr_t)L.A % 16 == 0) && (L.lda % VEC == 0) && (L.kb % VEC == 0);
    a.vec_b = ((uintptr_t)L.B % 16 == 0) && (L.ldb % VEC == 0) && (L.nb % VEC == 0);
    a.small_ld = (64 * (L.lda + 8) * (int64_t)sizeof(T) < (int64_t(1) << 31)) &&
                 (16 * (L.ldb + 8) * (int64_t)sizeof(T) < (int64_t(1) << 31));
    const int64_t blocks = (int64_t)a.tiles_m * a.tiles_n * L.nnodes;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const bool scaled = L.sc.ea != nullptr;
    const uint32_t *m = L.masks;
#define FASTMM_NODE_TRY(up, un, vp, vn, wp, wn)                                                        \
    if (m[0] == up && m[1] == un && m[2] == vp && m[3] == vn && m[4] == wp && m[5] == wn)             \
        return node_launch<T, up, un, vp, vn, wp, wn>(a, (unsigned)blocks, scaled, s);
    FASTMM_NODE222_PATTERNS(FASTMM_NODE_TRY)
#undef FASTMM_NODE_TRY
    return hipErrorInvalidValue;
}

}  // namespace

bool node222_supported(const uint32_t masks[6]) {
#define FASTMM_NODE_MATCH(up, un, vp, vn, wp, wn)                                                           \
    if (masks[0] == up && masks[1] == un && masks[2] == vp && masks[3] == vn && masks[4] == wp && masks[5] == wn) \
        return true;
    FASTMM_NODE222_PATTERNS(FASTMM_NODE_MATCH)
#undef FASTMM_NODE_MATCH
    return false;
}

hipError_t launch_node222(const NodeLaunch &L, hipStream_t s) {
    if (L.elem == Elem::F64) return node_go<double>(L, s);
    return node_go<float>(L, s);
}

}  // namespace fastmm
