// Pipelined fused leaf-product kernel for row-major (non-transposed) operands: FP64 via
// v_mfma_f64_16x16x4f64 and FP32 via v_mfma_f32_16x16x4f32.
//
// Each work-group computes one 128x128 tile of one leaf product M_r = S_r T_r of eq. (2).
// The S_r / T_r tiles are never stored in HBM: at every K step each thread loads its part of
// every source block of the leaf (16-byte vector loads on interior tiles), applies the
// power-of-two scaling exponents and the composite coefficient, sums the sources in table
// order and writes the result to LDS.  LDS is double-buffered and the global loads of step
// k+1 (the first two sources) are issued before the MFMA work of step k, so their latency is
// hidden behind the matrix cores; further sources of a high fan-in leaf are loaded after it.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "devtypes.h"
#include "launch.h"

namespace fastmm {
namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kNT = 256;
constexpr int kXcd = 8;

template <typename T>
struct Core;

// D(16x16) += A(16x4) B(4x16): lane l supplies A[l%16][l/16] and B[l/16][l%16];
// accumulator element v of lane l is D[row(l, v)][l%16].
template <>
struct Core<double> {
    typedef d4v acc_t;
    typedef double2 vec_t;
    static constexpr int VEC = 2, BK = 16, OCC = 1;
    __device__ static acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
    __device__ static double scale(double x, int e) { return ldexp(x, e); }
};
template <>
struct Core<float> {
    typedef f4v acc_t;
    typedef float4 vec_t;
    static constexpr int VEC = 4, BK = 32, OCC = 2;
    __device__ static acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
    __device__ static float scale(float x, int e) { return ldexpf(x, e); }
};

template <typename T>
struct PArgs {
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
    int vec_a, vec_b;  // 16-byte loads allowed (alignment of pointers, ld and block sizes)
    int small_ld;      // a 128-row (or BK-row) panel of either operand spans < 2^31 bytes
};

__device__ inline int64_t xcd_remap_tile(int64_t b, int64_t G) {
    const int64_t x = b % kXcd, j = b / kXcd;
    const int64_t per = G / kXcd, rem = G % kXcd;
    return ((x < rem) ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + j;
}

// Both tiles are k-contiguous (B stored transposed).  SWZ (FP32 without scaled loads): rows of
// 32 floats (128 bytes, eight 16-byte chunks), chunk c of row r kept at chunk c ^ (r mod 8);
// measured with SQ_LDS_BANK_CONFLICT on MI355X, the fragment reads (16 consecutive rows, one
// chunk per 16 lanes), the row-major A writes and the transposed B writes are all free of bank
// conflicts.  Otherwise rows padded by 16 bytes (one extra cycle per FP32 fragment read, but one
// lane offset fewer: the FP32 variants with scaled loads are short of registers).  idx(r, k):
// element (row r, k) for k a multiple of VEC; for r16 a multiple of 16,
// idx(r16 + r, k) = r16 LDS_K + idx(r, k).
template <typename T, bool SCALED>
struct Tile {
    typedef Core<T> C;
    static constexpr int BM = 128, BN = 128, BK = C::BK, VEC = C::VEC;
    static constexpr bool SWZ = sizeof(T) == 4 && !SCALED;
    static constexpr int LDS_K = SWZ ? BK : BK + 16 / (int)sizeof(T);
    __device__ static __forceinline__ int idx(int r, int k) {
        if constexpr (SWZ) return r * LDS_K + (((k / VEC) ^ (r & 7)) * VEC);
        else return r * LDS_K + k;
    }
    struct Smem {
        __attribute__((aligned(16))) T As[2][BM * LDS_K];
        __attribute__((aligned(16))) T Bs[2][BN * LDS_K];
    };
};

// One 128x128 output tile (tile row tm, tile column tn) of leaf `leaf` of the problem p.
// SCALED: the loads apply the scaling factors to the operands; SCALED_OUT: a direct output takes
// 2^(ea_i + eb_j) (with SCALED both, without SCALED only the output: operands already scaled).
// ONE: every leaf has one A and one B source with coefficient 1 (a single classical leaf, or the
// written leaf operands): the source blocks are read from the tables once, and each stage's
// loads go straight to the registers that are stored to LDS (no per-stage table reads, no
// coefficient products).
template <typename T, bool SCALED, bool DIRECT, bool SCALED_OUT = SCALED, bool ONE = false>
__device__ __forceinline__ void leaf_tile(const PArgs<T> &p, int leaf, int64_t tm, int64_t tn,
                                          typename Tile<T, SCALED>::Smem &sm) {
    typedef Core<T> C;
    constexpr int BM = 128, BN = 128, BK = C::BK, VEC = C::VEC;
    constexpr int TPRA = BK / VEC, RPPA = kNT / TPRA, NPA = BM / RPPA;  // A: threads/row, rows/pass
    // B is loaded in VEC x VEC blocks (VEC k-rows by VEC columns, consecutive lanes on
    // consecutive k-blocks) and written transposed, one 16-byte LDS write per column.
    constexpr int KBV = BK / VEC, NBT = KBV * (BN / VEC) / kNT, NPB = NBT * VEC;  // B: blocks, rows
    typedef Tile<T, SCALED> TL;
    constexpr int LDS_K = TL::LDS_K;
    constexpr int WM = 64, WN = 64, TM = WM / 16, TN = WN / 16;
    static_assert(NPA * RPPA == BM && NBT * kNT == KBV * (BN / VEC) && BK % 16 == 0, "tile shape");
    auto &As = sm.As;
    auto &Bs = sm.Bs;

    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    LeafEntry le = p.leaves[leaf];
    le.a_begin = __builtin_amdgcn_readfirstlane(le.a_begin);
    le.a_count = __builtin_amdgcn_readfirstlane(le.a_count);
    le.b_begin = __builtin_amdgcn_readfirstlane(le.b_begin);
    le.b_count = __builtin_amdgcn_readfirstlane(le.b_count);

    const int ra = t / TPRA, ka = (t % TPRA) * VEC;   // A: row within pass, k offset
    int kB[NBT], cB[NBT];  // B: the thread's blocks (k offset, column offset in the tile)
#pragma unroll
    for (int u = 0; u < NBT; ++u) kB[u] = ((t + kNT * u) % KBV) * VEC, cB[u] = ((t + kNT * u) / KBV) * VEC;
    // Byte offsets of the thread's vectors inside an interior tile: independent of the source
    // block and of the K stage (valid when 128 rows of the operands span < 2^31 bytes).  Used
    // for FP32 only: for FP64 the extra live offsets cost more than the address math they save.
    constexpr bool kInterior = sizeof(T) == 4;
    uint32_t voA[NPA], voB[NPB];
#pragma unroll
    for (int pa = 0; pa < NPA; ++pa) voA[pa] = (uint32_t)(((pa * RPPA + ra) * p.lda + ka) * sizeof(T));
#pragma unroll
    for (int pb = 0; pb < NPB; ++pb)
        voB[pb] = (uint32_t)(((kB[pb / VEC] + pb % VEC) * p.ldb + cB[pb / VEC]) * sizeof(T));

    // Load (with zero fill outside the operand and outside the leaf block) the thread's part
    // of one source block of A at K offset k0; values scaled by 2^(ep_col - ea_row).  Loads
    // outside the operand read the (valid) operand base instead and are replaced by zero, so
    // the loads themselves never branch; only the uniform interior/edge choice does.
    auto load_a = [&](const SrcEntry &se, int64_t k0, T (&v)[NPA][VEC]) {
        const int64_t row0 = (int64_t)se.br * p.mb + tm * BM;  // operand row of tile row 0
        const int64_t col0 = (int64_t)se.bc * p.kb + k0 + ka;  // operand column of this thread
        const bool full = p.vec_a && (k0 + BK <= p.kb) && ((int64_t)se.bc * p.kb + k0 + BK <= p.k);
        if (kInterior && full && (tm * BM + BM <= p.mb) && (row0 + BM <= p.m) && p.small_ld) {
            // interior tile: a work-group-uniform base and the thread's fixed 32-bit offsets
            const char *base = reinterpret_cast<const char *>(p.A + row0 * p.lda + (int64_t)se.bc * p.kb + k0);
#pragma unroll
            for (int pa = 0; pa < NPA; ++pa) {
                const typename C::vec_t x = *reinterpret_cast<const typename C::vec_t *>(
                    __builtin_assume_aligned(base + voA[pa], 16));
                const T *xs = reinterpret_cast<const T *>(&x);
#pragma unroll
                for (int e = 0; e < VEC; ++e) v[pa][e] = xs[e];
            }
        } else if (full) {
#pragma unroll
            for (int pa = 0; pa < NPA; ++pa) {
                const int r = pa * RPPA + ra;
                const bool rok = (tm * BM + r < p.mb) && (row0 + r < p.m);
                const T *src = rok ? p.A + (row0 + r) * p.lda + col0 : p.A;
                const typename C::vec_t x =
                    *reinterpret_cast<const typename C::vec_t *>(__builtin_assume_aligned(src, 16));
                const T *xs = reinterpret_cast<const T *>(&x);
#pragma unroll
                for (int e = 0; e < VEC; ++e) v[pa][e] = rok ? xs[e] : T(0);
            }
        } else {
#pragma unroll
            for (int pa = 0; pa < NPA; ++pa) {
                const int r = pa * RPPA + ra;
                const bool rok = (tm * BM + r < p.mb) && (row0 + r < p.m);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const bool ok = rok && (k0 + ka + e < p.kb) && (col0 + e < p.k);
                    const T x = *(ok ? p.A + (row0 + r) * p.lda + col0 + e : p.A);
                    v[pa][e] = ok ? x : T(0);
                }
            }
        }
        if (SCALED) {
#pragma unroll
            for (int pa = 0; pa < NPA; ++pa) {
                const int r = pa * RPPA + ra;
                const bool rok = (tm * BM + r < p.mb) && (row0 + r < p.m);
                const int er = p.sc.ea[rok ? row0 + r : 0];
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const bool cok = col0 + e < p.k;
                    const int ec = p.sc.ep[cok ? col0 + e : 0];
                    v[pa][e] = C::scale(v[pa][e], ec - er);
                }
            }
        }
    };
    // The thread's B blocks of one source block: row pb = u * VEC + vr of v holds k-row
    // kB[u] + vr, columns cB[u] .. cB[u] + VEC - 1; values scaled by 2^(-ep_row - eb_col).
    auto load_b = [&](const SrcEntry &se, int64_t k0, T (&v)[NPB][VEC]) {
        const int64_t row0 = (int64_t)se.br * p.kb + k0;      // operand row of k-row 0
        const int64_t colt = (int64_t)se.bc * p.nb + tn * BN;  // operand column of tile column 0
        const bool full = p.vec_b && (tn * BN + BN <= p.nb) && (colt + BN <= p.n);
        if (kInterior && full && (k0 + BK <= p.kb) && (row0 + BK <= p.k) && p.small_ld) {
            // interior tile: a work-group-uniform base and the thread's fixed 32-bit offsets
            const char *base = reinterpret_cast<const char *>(p.B + row0 * p.ldb + colt);
#pragma unroll
            for (int pb = 0; pb < NPB; ++pb) {
                const typename C::vec_t x = *reinterpret_cast<const typename C::vec_t *>(
                    __builtin_assume_aligned(base + voB[pb], 16));
                const T *xs = reinterpret_cast<const T *>(&x);
#pragma unroll
                for (int e = 0; e < VEC; ++e) v[pb][e] = xs[e];
            }
        } else if (full) {
#pragma unroll
            for (int pb = 0; pb < NPB; ++pb) {
                const int kr = kB[pb / VEC] + pb % VEC;
                const bool rok = (k0 + kr < p.kb) && (row0 + kr < p.k);
                const T *src = rok ? p.B + (row0 + kr) * p.ldb + colt + cB[pb / VEC] : p.B;
                const typename C::vec_t x =
                    *reinterpret_cast<const typename C::vec_t *>(__builtin_assume_aligned(src, 16));
                const T *xs = reinterpret_cast<const T *>(&x);
#pragma unroll
                for (int e = 0; e < VEC; ++e) v[pb][e] = rok ? xs[e] : T(0);
            }
        } else {
#pragma unroll
            for (int pb = 0; pb < NPB; ++pb) {
                const int kr = kB[pb / VEC] + pb % VEC;
                const bool rok = (k0 + kr < p.kb) && (row0 + kr < p.k);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int64_t cc = cB[pb / VEC] + e;
                    const bool ok = rok && (tn * BN + cc < p.nb) && (colt + cc < p.n);
                    const T x = *(ok ? p.B + (row0 + kr) * p.ldb + colt + cc : p.B);
                    v[pb][e] = ok ? x : T(0);
                }
            }
        }
        if (SCALED) {
#pragma unroll
            for (int pb = 0; pb < NPB; ++pb) {
                const int kr = kB[pb / VEC] + pb % VEC;
                const bool rok = (k0 + kr < p.kb) && (row0 + kr < p.k);
                const int er = p.sc.ep[rok ? row0 + kr : 0];
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int64_t col = colt + cB[pb / VEC] + e;
                    const int ec = p.sc.eb[col < p.n ? col : 0];
                    v[pb][e] = C::scale(v[pb][e], -er - ec);
                }
            }
        }
    };

    T sa[NPA][VEC], sb[NPB][VEC];   // summed S / T parts of the next stage
    T xa0[NPA][VEC], xb0[NPB][VEC];  // raw loads of source 0
    T xa1[NPA][VEC], xb1[NPB][VEC];  // raw loads of source 1

    // S/T part of the stage at k0: sources >= first, added to sa/sb (first == 0: assign)
    auto gather_rest = [&](int64_t k0, int first) {
        for (int q = first; q < le.a_count; ++q) {
            const SrcEntry se = p.asrc[le.a_begin + q];
            const T c = (T)se.coef;
            load_a(se, k0, xa0);
#pragma unroll
            for (int i = 0; i < NPA; ++i)
#pragma unroll
                for (int e = 0; e < VEC; ++e) sa[i][e] = (q == 0) ? c * xa0[i][e] : sa[i][e] + c * xa0[i][e];
        }
        for (int q = first; q < le.b_count; ++q) {
            const SrcEntry se = p.bsrc[le.b_begin + q];
            const T c = (T)se.coef;
            load_b(se, k0, xb0);
#pragma unroll
            for (int i = 0; i < NPB; ++i)
#pragma unroll
                for (int e = 0; e < VEC; ++e) sb[i][e] = (q == 0) ? c * xb0[i][e] : sb[i][e] + c * xb0[i][e];
        }
    };
    SrcEntry one_a{}, one_b{};  // ONE: the leaf's sources, read once (uniform)
    if constexpr (ONE) {
        one_a = p.asrc[le.a_begin], one_b = p.bsrc[le.b_begin];
        one_a.br = __builtin_amdgcn_readfirstlane(one_a.br), one_a.bc = __builtin_amdgcn_readfirstlane(one_a.bc);
        one_b.br = __builtin_amdgcn_readfirstlane(one_b.br), one_b.bc = __builtin_amdgcn_readfirstlane(one_b.bc);
    }
    // Issue the raw loads of sources 0 and 1 (those exist) of the stage at k0 (ONE: straight
    // into the registers stored next).
    auto prefetch = [&](int64_t k0) {
        if constexpr (ONE) {
            load_a(one_a, k0, sa);
            load_b(one_b, k0, sb);
            return;
        }
        load_a(p.asrc[le.a_begin], k0, xa0);
        if (le.a_count > 1) load_a(p.asrc[le.a_begin + 1], k0, xa1);
        load_b(p.bsrc[le.b_begin], k0, xb0);
        if (le.b_count > 1) load_b(p.bsrc[le.b_begin + 1], k0, xb1);
    };
    // Combine the prefetched sources (in source order) and gather the remaining ones.
    auto finish = [&](int64_t k0) {
        if constexpr (ONE) return;
        const T ca0 = (T)p.asrc[le.a_begin].coef, cb0 = (T)p.bsrc[le.b_begin].coef;
#pragma unroll
        for (int i = 0; i < NPA; ++i)
#pragma unroll
            for (int e = 0; e < VEC; ++e) sa[i][e] = ca0 * xa0[i][e];
#pragma unroll
        for (int i = 0; i < NPB; ++i)
#pragma unroll
            for (int e = 0; e < VEC; ++e) sb[i][e] = cb0 * xb0[i][e];
        if (le.a_count > 1) {
            const T c = (T)p.asrc[le.a_begin + 1].coef;
#pragma unroll
            for (int i = 0; i < NPA; ++i)
#pragma unroll
                for (int e = 0; e < VEC; ++e) sa[i][e] = sa[i][e] + c * xa1[i][e];
        }
        if (le.b_count > 1) {
            const T c = (T)p.bsrc[le.b_begin + 1].coef;
#pragma unroll
            for (int i = 0; i < NPB; ++i)
#pragma unroll
                for (int e = 0; e < VEC; ++e) sb[i][e] = sb[i][e] + c * xb1[i][e];
        }
        if (le.a_count > 2 || le.b_count > 2) {
            // remaining sources (their latency is not hidden)
            for (int q = 2; q < le.a_count; ++q) {
                const SrcEntry se = p.asrc[le.a_begin + q];
                const T c = (T)se.coef;
                load_a(se, k0, xa0);
#pragma unroll
                for (int i = 0; i < NPA; ++i)
#pragma unroll
                    for (int e = 0; e < VEC; ++e) sa[i][e] = sa[i][e] + c * xa0[i][e];
            }
            for (int q = 2; q < le.b_count; ++q) {
                const SrcEntry se = p.bsrc[le.b_begin + q];
                const T c = (T)se.coef;
                load_b(se, k0, xb0);
#pragma unroll
                for (int i = 0; i < NPB; ++i)
#pragma unroll
                    for (int e = 0; e < VEC; ++e) sb[i][e] = sb[i][e] + c * xb0[i][e];
            }
        }
    };
    static_assert(RPPA % 16 == 0, "pass rows");
    const int sto_a = TL::idx(ra, ka);
    int sto_b[NBT][VEC];
#pragma unroll
    for (int u = 0; u < NBT; ++u)
#pragma unroll
        for (int e = 0; e < VEC; ++e) sto_b[u][e] = TL::idx(cB[u] + e, kB[u]);
    auto store = [&](int s) {
#pragma unroll
        for (int pa = 0; pa < NPA; ++pa) {
            typename C::vec_t x;
            T *xs = reinterpret_cast<T *>(&x);
#pragma unroll
            for (int e = 0; e < VEC; ++e) xs[e] = sa[pa][e];
            *reinterpret_cast<typename C::vec_t *>(&As[s][pa * RPPA * LDS_K + sto_a]) = x;
        }
#pragma unroll
        for (int u = 0; u < NBT; ++u)
#pragma unroll
            for (int e = 0; e < VEC; ++e) {  // column cB + e, k-rows kB .. kB + VEC - 1
                typename C::vec_t x;
                T *xs = reinterpret_cast<T *>(&x);
#pragma unroll
                for (int vr = 0; vr < VEC; ++vr) xs[vr] = sb[u * VEC + vr][e];
                *reinterpret_cast<typename C::vec_t *>(&Bs[s][sto_b[u][e]]) = x;
            }
    };

    typename C::acc_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = typename C::acc_t{};

    const int64_t nk = (p.kb + BK - 1) / BK;
    if constexpr (ONE) prefetch(0);
    else gather_rest(0, 0);
    store(0);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        const bool more = kt + 1 < nk;
        if (more) prefetch((kt + 1) * BK);
        const T *as = As[cur];
        const T *bs = Bs[cur];
        // Each 16-k chunk takes four MFMA steps; step j uses k = 4g + j of the chunk from lane
        // group g = lane / 16, so a lane's operands for the four steps are 4 consecutive k of
        // one tile row: 16-byte LDS reads.
        const int g4 = 4 * (lane >> 4), l16 = lane & 15;
        // the fragments of 16-k chunk h: A rows and B columns of the wave's tile
        auto read_frag = [&](int h, T (&ea)[TM][4], T (&eb)[TN][4]) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int c = 0; c < 4; c += VEC) {
                    const typename C::vec_t x = *reinterpret_cast<const typename C::vec_t *>(
                        &as[(wm * WM + i * 16) * LDS_K + TL::idx(l16, 16 * h + g4 + c)]);
                    const T *xs = reinterpret_cast<const T *>(&x);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) ea[i][c + e] = xs[e];
                }
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int c = 0; c < 4; c += VEC) {
                    const typename C::vec_t x = *reinterpret_cast<const typename C::vec_t *>(
                        &bs[(wn * WN + j * 16) * LDS_K + TL::idx(l16, 16 * h + g4 + c)]);
                    const T *xs = reinterpret_cast<const T *>(&x);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) eb[j][c + e] = xs[e];
                }
        };
        // ONE with two chunks per stage: the second chunk's fragments are read before the
        // mid-stage stores (the stores go to the other buffer; the compiler cannot tell, and
        // would otherwise wait for these reads after the first chunk's MFMA work)
        constexpr bool EARLY = ONE && BK / 16 == 2;
        T ea1[TM][4], eb1[TN][4];
        if constexpr (EARLY) read_frag(1, ea1, eb1);
#pragma unroll
        for (int h = 0; h < BK / 16; ++h) {
            T ea[TM][4], eb[TN][4];
            if (EARLY && h == 1) {
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int c = 0; c < 4; ++c) ea[i][c] = ea1[i][c];
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int c = 0; c < 4; ++c) eb[j][c] = eb1[j][c];
            } else {
                read_frag(h, ea, eb);
            }
#pragma unroll
            for (int st = 0; st < 4; ++st) {
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) acc[i][j] = C::mma(ea[i][st], eb[j][st], acc[i][j]);
                // Half-way through the MFMA work: combine the prefetched sources of the next
                // stage and write them to the other LDS buffer (last read before the previous
                // barrier), so the VALU and LDS work overlaps the matrix cores.
                if (4 * h + st == BK / 8 - 1 && more) {
                    finish((kt + 1) * BK);
                    store(cur ^ 1);
                }
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = tm * BM + wm * WM + i * 16 + C::row(lane, v);
                const int64_t col = tn * BN + wn * WN + j * 16 + (lane & 15);
                T val = acc[i][j][v];
                if (DIRECT) {
                    if (row < p.m && col < p.n) {
                        if (SCALED_OUT) val = C::scale(val, p.sc.ea[row] + p.sc.eb[col]);
                        p.out[row * p.ldo + col] = val;
                    }
                } else {
                    if (row < p.mb && col < p.nb) p.out[(int64_t)leaf * p.leaf_stride + row * p.ldo + col] = val;
                }
            }
}

// Work-group-uniform values are moved to scalar registers explicitly, so that branches on the
// leaf's source counts stay scalar branches.  Tiles run in groups of 8 tile-rows, column by
// column inside a group, so the work-groups resident on one XCD share A row panels and B
// column panels in its L2.
__device__ __forceinline__ void tile_coords(int rem, int tiles_m, int tiles_n, int64_t &tm, int64_t &tn) {
    const int grp = rem / (8 * tiles_n);
    const int gsz = min(8, tiles_m - grp * 8);
    const int gidx = rem - grp * 8 * tiles_n;
    tm = __builtin_amdgcn_readfirstlane(grp * 8 + gidx % gsz);
    tn = __builtin_amdgcn_readfirstlane(gidx / gsz);
}

template <typename T, bool SCALED, bool DIRECT, bool SCALED_OUT = SCALED, bool ONE = false>
__global__ __launch_bounds__(kNT, Core<T>::OCC) void fmm_leaf_pipelined(PArgs<T> p) {
    __shared__ typename Tile<T, SCALED>::Smem sm;
    const int64_t tiles = (int64_t)p.tiles_m * p.tiles_n;
    const int bid = __builtin_amdgcn_readfirstlane((int)xcd_remap_tile(blockIdx.x, gridDim.x));
    const int leaf = __builtin_amdgcn_readfirstlane((int)(bid / tiles));
    const int rem = __builtin_amdgcn_readfirstlane((int)(bid - (int64_t)leaf * tiles));
    int64_t tm, tn;
    tile_coords(rem, p.tiles_m, p.tiles_n, tm, tn);
    leaf_tile<T, SCALED, DIRECT, SCALED_OUT, ONE>(p, leaf, tm, tn, sm);
}

// Batched launch over several problems of one output mode (each with its own plan tables):
// work-group w runs work item w, which belongs to the problem q with first[q] <= w < first[q+1]
// (problems ordered by the host, largest K first, so the longest items are dispatched first).
// The host launches one such kernel per (scaling, output) mode present in the batch, so each
// is the single-problem tile code with its register count and occupancy.
template <typename T, bool SCALED, bool DIRECT, bool ONE = false>
__global__ __launch_bounds__(kNT, Core<T>::OCC) void fmm_leaf_batched(const PArgs<T> *__restrict__ probs,
                                                                     const int64_t *__restrict__ first, int count,
                                                                     int64_t total) {
    __shared__ typename Tile<T, SCALED>::Smem sm;
    const int64_t w = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {  // last q with first[q] <= w
        const int mid = (lo + hi + 1) / 2;
        if (first[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    const int q = __builtin_amdgcn_readfirstlane(lo);
    const PArgs<T> p = probs[q];
    const int64_t tiles = (int64_t)p.tiles_m * p.tiles_n;
    const int64_t local = w - first[q];
    const int leaf = __builtin_amdgcn_readfirstlane((int)(local / tiles));
    const int rem = __builtin_amdgcn_readfirstlane((int)(local - (int64_t)leaf * tiles));
    int64_t tm, tn;
    tile_coords(rem, p.tiles_m, p.tiles_n, tm, tn);
    leaf_tile<T, SCALED, DIRECT, SCALED, ONE>(p, leaf, tm, tn, sm);
}


template <typename T>
PArgs<T> make_args(const LeafLaunch &L) {
    PArgs<T> a;
    a.A = (const T *)L.A;
    a.B = (const T *)L.B;
    a.out = (T *)L.out;
    a.lda = L.lda, a.ldb = L.ldb, a.ldo = L.ldo;
    a.m = L.m, a.k = L.k, a.n = L.n;
    a.mb = L.mb, a.kb = L.kb, a.nb = L.nb;
    a.leaf_stride = L.leaf_stride;
    a.tiles_m = (int)((L.mb + 127) / 128);
    a.tiles_n = (int)((L.nb + 127) / 128);
    a.leaves = L.leaves, a.asrc = L.asrc, a.bsrc = L.bsrc;
    a.sc = L.sc;
    constexpr int VEC = Core<T>::VEC;
    a.vec_a = ((uintptr_t)L.A % 16 == 0) && (L.lda % VEC == 0) && (L.kb % VEC == 0);
    a.vec_b = ((uintptr_t)L.B % 16 == 0) && (L.ldb % VEC == 0) && (L.nb % VEC == 0);
    a.small_ld = (128 * (L.lda + 8) * (int64_t)sizeof(T) < (int64_t(1) << 31)) &&
                 (128 * (L.ldb + 8) * (int64_t)sizeof(T) < (int64_t(1) << 31));
    return a;
}

template <typename T>
hipError_t go(const LeafLaunch &L, hipStream_t s) {
    const PArgs<T> a = make_args<T>(L);
    const int64_t blocks = (int64_t)a.tiles_m * a.tiles_n * L.nleaves;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const bool scaled = L.sc.ea != nullptr;
    dim3 grid((unsigned)blocks), block(kNT);
    // The single-source form only without scaled loads (with them the FP32 variant spills).
    if (L.direct && L.one && !(scaled && L.scale_in)) {
        if (scaled) hipLaunchKernelGGL((fmm_leaf_pipelined<T, false, true, true, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((fmm_leaf_pipelined<T, false, true, false, true>), grid, block, 0, s, a);
    } else if (L.direct) {
        if (scaled && !L.scale_in)
            hipLaunchKernelGGL((fmm_leaf_pipelined<T, false, true, true>), grid, block, 0, s, a);
        else if (scaled) hipLaunchKernelGGL((fmm_leaf_pipelined<T, true, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((fmm_leaf_pipelined<T, false, true>), grid, block, 0, s, a);
    } else {
        if (scaled) hipLaunchKernelGGL((fmm_leaf_pipelined<T, true, false>), grid, block, 0, s, a);
        else if (L.one) hipLaunchKernelGGL((fmm_leaf_pipelined<T, false, false, false, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((fmm_leaf_pipelined<T, false, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}


}  // namespace

size_t leaf_desc_bytes(Elem e) { return e == Elem::F64 ? sizeof(PArgs<double>) : sizeof(PArgs<float>); }

int64_t leaf_desc_build(const LeafLaunch &L, void *dst) {
    if (L.elem == Elem::F64) {
        const PArgs<double> a = make_args<double>(L);
        std::memcpy(dst, &a, sizeof(a));
        return (int64_t)a.tiles_m * a.tiles_n * L.nleaves;
    }
    const PArgs<float> a = make_args<float>(L);
    std::memcpy(dst, &a, sizeof(a));
    return (int64_t)a.tiles_m * a.tiles_n * L.nleaves;
}

template <typename T>
hipError_t batched_go(int scaled, int direct, int one, const void *descs, const int64_t *first, int count,
                      int64_t total, hipStream_t s) {
    const PArgs<T> *d = (const PArgs<T> *)descs;
    const dim3 grid((unsigned)total), block(kNT);
    if (one && !scaled) {
        if (direct) hipLaunchKernelGGL((fmm_leaf_batched<T, false, true, true>), grid, block, 0, s, d, first, count, total);
        else hipLaunchKernelGGL((fmm_leaf_batched<T, false, false, true>), grid, block, 0, s, d, first, count, total);
    } else if (scaled) {
        if (direct) hipLaunchKernelGGL((fmm_leaf_batched<T, true, true>), grid, block, 0, s, d, first, count, total);
        else hipLaunchKernelGGL((fmm_leaf_batched<T, true, false>), grid, block, 0, s, d, first, count, total);
    } else {
        if (direct) hipLaunchKernelGGL((fmm_leaf_batched<T, false, true>), grid, block, 0, s, d, first, count, total);
        else hipLaunchKernelGGL((fmm_leaf_batched<T, false, false>), grid, block, 0, s, d, first, count, total);
    }
    return hipGetLastError();
}

hipError_t launch_leaf_batched(Elem e, int scaled, int direct, int one, const void *descs, const int64_t *first,
                               int count, int64_t total, hipStream_t s) {
    if (total <= 0 || count <= 0) return hipSuccess;
    if (total > 0x7fffffffLL) return hipErrorInvalidValue;
    if (e == Elem::F64) return batched_go<double>(scaled, direct, one, descs, first, count, total, s);
    return batched_go<float>(scaled, direct, one, descs, first, count, total, s);
}

hipError_t launch_leaf_pipelined(const LeafLaunch &L, hipStream_t s) {
    if (L.elem == Elem::F64) return go<double>(L, s);
    return go<float>(L, s);
}

}  // namespace fastmm
