// Split-precision leaf products, pass 2 (pass 1, the limb planes, is plane_form.hip).
//
// fmm_limb_gemm: M_r = sum over the kept limb products S^(a) T^(b), the products of
// total order <= 2: x1y1 (one limb), x1y1 + x1y2 + x2y1 (two limbs), plus x1y3 + x2y2 + x3y1
// (three limbs), smallest terms first, on v_mfma_f32_16x16x32_{bf16,f16} with FP32
// accumulation.  The output is the leaf-product workspace (the W-combination follows) or, for
// a single classical leaf, C with the outside-scaling factors applied.  fmm_limb_fused forms
// the innermost level's operands in its own loads instead of reading planes.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "devtypes.h"
#include "fastmm.h"
#include "launch.h"
#include "limbs.h"

namespace fastmm {
namespace {

constexpr int kXcds = 8;

// ------------------------------------------------------------------ pass 2: limb GEMM
__device__ inline int64_t xcd_remap_g(int64_t b, int64_t G) {
    const int64_t x = b % kXcds, j = b / kXcds;
    const int64_t per = G / kXcds, rem = G % kXcds;
    return ((x < rem) ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + j;
}

// Limb products (a, b) kept for NL limbs, smallest first.
template <int NL>
struct Products;
template <>
struct Products<1> {
    static constexpr int n = 1;
    static constexpr int a[1] = {0}, b[1] = {0};
};
template <>
struct Products<2> {
    static constexpr int n = 3;
    static constexpr int a[3] = {0, 1, 0}, b[3] = {1, 0, 0};
};
template <>
struct Products<3> {
    static constexpr int n = 6;
    static constexpr int a[6] = {0, 1, 2, 0, 1, 0}, b[6] = {2, 1, 0, 1, 0, 0};
};

// Work-group of WM x WN waves, each a (BM/WM) x (BN/WN) tile of the BM x BN output tile: 2 x 2
// waves on 128 x 128 tiles, 4 x 2 waves of 64 x 128 on 256 x 256 tiles (measured on MI355X over
// 49 leaves of 4096^3: 2 % faster than 2 x 4 waves of 128 x 64; one work-group per CU, two waves
// per SIMD).  K stage 32; LDS double-buffered, rows of 32 halves (64 bytes, four 16-byte chunks)
// with chunk c of row r stored at chunk c ^ ((r / 2) mod 4), so that the 16-byte fragment reads
// (16 rows, one chunk) and the staging writes (consecutive chunks and rows) both fall on distinct
// banks (SQ_LDS_BANK_CONFLICT reads 0 for this kernel; swizzling with bit 3 of r as well gives 3
// conflict cycles per LDS instruction and 13 % more time).
template <int NL, int BM, int BN>
struct LimbSmem {
    __attribute__((aligned(16))) unsigned short As[2][NL][BM * 32];
    __attribute__((aligned(16))) unsigned short Bs[2][NL][BN * 32];
};

// Output tile (tm, tn) of leaf `leaf` of the problem a.
// DYN: the output mode (DIRECT, SCALED) is read from the descriptor at run time (batched launch).
template <bool HALF, int NL, int BM, int BN, int WM, int WN, bool SCALED, bool DIRECT, bool DYN = false>
__device__ __forceinline__ void limb_tile(const LimbGemm &a, int leaf, int64_t tm, int64_t tn,
                                          LimbSmem<NL, BM, BN> &sm) {
    constexpr int BK = 32, NT = 64 * WM * WN, RS = 32;
    constexpr int TI = BM / (16 * WM), TJ = BN / (16 * WN);  // 16 x 16 MFMA blocks per wave
    constexpr int CA = NL * BM * 4 / NT, CB = NL * BN * 4 / NT;  // 16-byte chunks per thread and stage
    static_assert(CA * NT == NL * BM * 4 && CB * NT == NL * BN * 4, "chunk split");
    typedef Products<NL> P;
    auto &As = sm.As;
    auto &Bs = sm.Bs;

    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave / WN, wn = wave % WN;

    // planes are blocked in BM x 32 tiles (BM == BN): the tile of stage kt is contiguous
    const unsigned short *Sp = a.S + (int64_t)leaf * a.s_leaf + tm * BM * a.kp;
    const unsigned short *Tp = a.T + (int64_t)leaf * a.t_leaf + tn * BN * a.kp;
    static_assert(BM == BN, "square tiles");
    auto swz = [](int r, int c) { return c ^ ((r >> 1) & 3); };
    // chunk u of this thread: limb, row, 16-byte column (consecutive lanes along k, then rows);
    // the same split for every stage
    auto chunk = [&](int u, int rows, int &l, int &r, int &kc) {
        const int c = t + NT * u;
        l = c / (rows * 4), r = (c % (rows * 4)) / 4, kc = c % 4;
    };
    // The staging registers are vector values (not arrays), so that they stay in VGPRs.
    typedef uint32_t stA_t __attribute__((ext_vector_type(4 * CA)));
    typedef uint32_t stB_t __attribute__((ext_vector_type(4 * CB)));
#define LIMB_LOAD(k0)                                                                                   \
    _Pragma("unroll") for (int u = 0; u < CA; ++u) {                                                    \
        int l, r, kc;                                                                                   \
        chunk(u, BM, l, r, kc);                                                                         \
        const uint4 w = *reinterpret_cast<const uint4 *>(Sp + l * a.s_plane + (k0) * BM + r * 32 + kc * 8); \
        ra[4 * u] = w.x, ra[4 * u + 1] = w.y, ra[4 * u + 2] = w.z, ra[4 * u + 3] = w.w;                 \
    }                                                                                                   \
    _Pragma("unroll") for (int u = 0; u < CB; ++u) {                                                    \
        int l, r, kc;                                                                                   \
        chunk(u, BN, l, r, kc);                                                                         \
        const uint4 w = *reinterpret_cast<const uint4 *>(Tp + l * a.t_plane + (k0) * BN + r * 32 + kc * 8); \
        rb[4 * u] = w.x, rb[4 * u + 1] = w.y, rb[4 * u + 2] = w.z, rb[4 * u + 3] = w.w;                 \
    }
#define LIMB_STORE(st)                                                                              \
    _Pragma("unroll") for (int u = 0; u < CA; ++u) {                                                \
        int l, r, kc;                                                                               \
        chunk(u, BM, l, r, kc);                                                                     \
        *reinterpret_cast<uint4 *>(&As[st][l][r * RS + 8 * swz(r, kc)]) =                           \
            uint4{ra[4 * u], ra[4 * u + 1], ra[4 * u + 2], ra[4 * u + 3]};                          \
    }                                                                                               \
    _Pragma("unroll") for (int u = 0; u < CB; ++u) {                                                \
        int l, r, kc;                                                                               \
        chunk(u, BN, l, r, kc);                                                                     \
        *reinterpret_cast<uint4 *>(&Bs[st][l][r * RS + 8 * swz(r, kc)]) =                           \
            uint4{rb[4 * u], rb[4 * u + 1], rb[4 * u + 2], rb[4 * u + 3]};                          \
    }
    stA_t ra;
    stB_t rb;

    g4v acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = g4v{0.f, 0.f, 0.f, 0.f};

    const int g = lane >> 4, l16 = lane & 15;
    const int64_t nk = a.kp / BK;
    LIMB_LOAD(0)
    LIMB_STORE(0)
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        const bool more = kt + 1 < nk;
        if (more) {
            LIMB_LOAD((kt + 1) * BK)
        }
        gs8 fa[TI][NL], fb[TJ][NL];
#pragma unroll
        for (int l = 0; l < NL; ++l) {
#pragma unroll
            for (int i = 0; i < TI; ++i) {
                const int rr = wm * (BM / WM) + i * 16 + l16;
                fa[i][l] = *reinterpret_cast<const gs8 *>(&As[cur][l][rr * RS + 8 * swz(rr, g)]);
            }
#pragma unroll
            for (int j = 0; j < TJ; ++j) {
                const int rr = wn * (BN / WN) + j * 16 + l16;
                fb[j][l] = *reinterpret_cast<const gs8 *>(&Bs[cur][l][rr * RS + 8 * swz(rr, g)]);
            }
        }
#pragma unroll
        for (int p = 0; p < P::n; ++p)
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TJ; ++j) acc[i][j] = LimbT<HALF>::mma(fa[i][P::a[p]], fb[j][P::b[p]], acc[i][j]);
        if (more) {  // the other buffer was last read before the previous barrier
            LIMB_STORE(cur ^ 1)
        }
        __syncthreads();
    }
#undef LIMB_LOAD
#undef LIMB_STORE

    const bool direct = DYN ? a.direct != 0 : DIRECT;
    const bool scaled = DYN ? a.sc.ea != nullptr : SCALED;
    // column exponents of the lane's TJ columns, loaded once (direct scaled output only)
    int ebj[TJ];
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
        const int64_t col = tn * BN + wn * (BN / WN) + j * 16 + l16;
        ebj[j] = (direct && scaled && col < a.n) ? a.sc.eb[col] : 0;
    }
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = tm * BM + wm * (BM / WM) + i * 16 + 4 * (lane >> 4) + v;  // inside the leaf block
            const int eai = (direct && scaled && row < a.m) ? a.post_exp + a.sc.ea[row] : 0;
#pragma unroll
            for (int j = 0; j < TJ; ++j) {
                const int64_t col = tn * BN + wn * (BN / WN) + j * 16 + l16;
                float val = acc[i][j][v];
                if (direct) {
                    if (row < a.m && col < a.n) {  // one power-of-two factor: exact unless it underflows
                        if (scaled) val = ldexpf(val, eai + ebj[j]);
                        a.out[row * a.ldo + col] = val;
                    }
                } else if (row < a.mb && col < a.nb) {
                    if (a.post_exp) val = ldexpf(val, a.post_exp);
                    a.out[(int64_t)leaf * a.leaf_stride + row * a.ldo + col] = val;
                }
            }
        }
}

// ------------------------------------------------------------------ limb GEMM, innermost level fused
// As limb_tile, with the limb tiles formed while staging instead of read from limb planes: every
// stage each thread loads its chunks (eight consecutive k of one row; 16-byte loads) of the up to
// Q source sub-blocks of its leaf's S_r and T_r^T (loads for stage k+1 issued before the MFMA
// work of stage k), sums them with the coefficients (times the row's outside-scaling factor, a
// power of two, so each term is exact and each sum rounds once, in source order), splits the
// sums into limbs and writes the 16-byte limb chunks to LDS.  The limb products, their order and
// the output are those of limb_tile.
template <bool HALF, int NL, int BM, int BN, int WM, int WN, int QA, int QB, bool M32>
__device__ __forceinline__ void limb_tile_fused(const LimbFused &a, int leaf, int64_t tm, int64_t tn,
                                                LimbSmem<NL, BM, BN> &sm) {
    constexpr int BK = 32, NT = 64 * WM * WN, RS = 32;
    constexpr int MS = M32 ? 32 : 16;  // MFMA block: 32 x 32 x 16 or 16 x 16 x 32
    constexpr int TI = BM / (MS * WM), TJ = BN / (MS * WN);
    typedef typename std::conditional<M32, g16v, g4v>::type acc_t;
    constexpr int NV = M32 ? 16 : 4;
    constexpr int CA = BM * 4 / NT, CB = BN * 4 / NT;  // 8-k chunks per thread and stage
    static_assert(CA * NT == BM * 4 && CB * NT == BN * 4, "chunk split");
    typedef Products<NL> P;
    auto &As = sm.As;
    auto &Bs = sm.Bs;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave / WN, wn = wave % WN;
    auto swz = [](int r, int c) { return c ^ ((r >> 1) & 3); };

    // The leaf's sources: the nonzeros of column r of the innermost U (A side) and V (B side),
    // in increasing index order; slot q holds the q-th (uniform values, found by a scan per slot).
    const int node = leaf / a.R, r = leaf - node * a.R;
    const int nsa = a.M0 * a.K0, nsb = a.K0 * a.N0;
    int na = 0, nb = 0;
    float ca[QA], cb[QB];
    int64_t ra0[QA], ka0[QA], rb0[QB], kb0[QB];  // first row and k offset of each source sub-block
#pragma unroll
    for (int q = 0; q < QA; ++q) {
        int idx = -1, cnt = 0;
        for (int i = 0; i < nsa; ++i)
            if (a.ucoef[i * a.R + r] != 0.f) {
                if (cnt == q) idx = i;
                ++cnt;
            }
        na = cnt < QA ? cnt : QA;
        ca[q] = idx >= 0 ? a.ucoef[idx * a.R + r] : 0.f;
        ra0[q] = idx >= 0 ? (int64_t)(idx % a.M0) * a.a.sb_rows : 0;
        ka0[q] = idx >= 0 ? (int64_t)(idx / a.M0) * a.kb : 0;
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
        int idx = -1, cnt = 0;
        for (int j = 0; j < nsb; ++j)
            if (a.vcoef[j * a.R + r] != 0.f) {
                if (cnt == q) idx = j;
                ++cnt;
            }
        nb = cnt < QB ? cnt : QB;
        cb[q] = idx >= 0 ? a.vcoef[idx * a.R + r] : 0.f;
        rb0[q] = idx >= 0 ? (int64_t)(idx / a.K0) * a.b.sb_rows : 0;
        kb0[q] = idx >= 0 ? (int64_t)(idx % a.K0) * a.kb : 0;
    }
    const float *XA = a.a.X + (int64_t)node * a.a.node_stride;
    const float *XB = a.b.X + (int64_t)node * a.b.node_stride;
    // Per source: element offset (32-bit) of the thread's first chunk inside the node operand;
    // chunk u lies 128 u rows further (rows r0 + 128 u of the tile, k chunk kc).  Bit u Q + q of
    // vmask: chunk u of source q lies inside the operand.  Factors: the coefficient times the
    // row's outside-scaling factor (a power of two), per chunk and source.
    static_assert(NT == 512 && CA == 2 && CB == 2, "thread layout");
    const int r0 = t >> 2, kc = t & 3;
    uint32_t ba[QA], bb[QB];
    uint32_t ma = 0, mbm = 0;
    float fa_[CA][QA], fb_[CB][QB];
#pragma unroll
    for (int q = 0; q < QA; ++q) {
        ba[q] = (uint32_t)((ra0[q] + tm * BM + r0) * a.a.ld + ka0[q] + 8 * kc);
#pragma unroll
        for (int u = 0; u < CA; ++u) {
            const int64_t lr = tm * BM + r0 + 128 * u, row = ra0[q] + lr;
            const bool ok = q < na && lr < a.mb && row < a.a.rows;
            ma |= ok ? 1u << (u * QA + q) : 0u;
            fa_[u][q] = (ok && a.a.e_row) ? ldexpf(ca[q], a.a.s_row * a.a.e_row[row] + a.a.pre_exp) : ca[q];
        }
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
        bb[q] = (uint32_t)((rb0[q] + tn * BN + r0) * a.b.ld + kb0[q] + 8 * kc);
#pragma unroll
        for (int u = 0; u < CB; ++u) {
            const int64_t lr = tn * BN + r0 + 128 * u, row = rb0[q] + lr;
            const bool ok = q < nb && lr < a.nb && row < a.b.rows;
            mbm |= ok ? 1u << (u * QB + q) : 0u;
            fb_[u][q] = (ok && a.b.e_row) ? ldexpf(cb[q], a.b.s_row * a.b.e_row[row] + a.b.pre_exp) : cb[q];
        }
    }
    const uint32_t stepa = (uint32_t)(128 * a.a.ld), stepb = (uint32_t)(128 * a.b.ld);
    // Raw source chunks of the next stage, as vector values (not arrays) so that they stay in
    // VGPRs: element 8 (u QA + q) + e of xa is element e of chunk u, source q.
    typedef float rawA_t __attribute__((ext_vector_type(8 * CA * QA)));
    typedef float rawB_t __attribute__((ext_vector_type(8 * CB * QB)));
    rawA_t xa;
    rawB_t xb;
#define FUSED_LOAD_SIDE(X, Q, BASE, MASK, STEP, OFF0, COLS, XP, k0)                                    \
    _Pragma("unroll") for (int u = 0; u < 2; ++u) {                                                    \
        const int64_t kk = (k0) + 8 * kc;                                                              \
        _Pragma("unroll") for (int q = 0; q < Q; ++q) {                                                \
            const bool ok = ((MASK >> (u * Q + q)) & 1u) && kk + 8 <= a.kb && OFF0[q] + kk + 8 <= COLS; \
            float4 w0 = make_float4(0.f, 0.f, 0.f, 0.f), w1 = w0;                                      \
            if (ok) {                                                                                  \
                const float4 *p4 = reinterpret_cast<const float4 *>(XP + BASE[q] + u * STEP + (k0));   \
                w0 = p4[0], w1 = p4[1];                                                                \
            }                                                                                          \
            const int b8 = 8 * (u * Q + q);                                                            \
            X[b8] = w0.x, X[b8 + 1] = w0.y, X[b8 + 2] = w0.z, X[b8 + 3] = w0.w;                        \
            X[b8 + 4] = w1.x, X[b8 + 5] = w1.y, X[b8 + 6] = w1.z, X[b8 + 7] = w1.w;                    \
        }                                                                                              \
    }
#define FUSED_LOAD(k0)                                                       \
    FUSED_LOAD_SIDE(xa, QA, ba, ma, stepa, ka0, a.a.cols, XA, k0)            \
    FUSED_LOAD_SIDE(xb, QB, bb, mbm, stepb, kb0, a.b.cols, XB, k0)
    const int rowa[2] = {r0, r0 + 128}, kca[2] = {kc, kc}, rowb[2] = {r0, r0 + 128}, kcb[2] = {kc, kc};
    // Sum each chunk's sources (v = f0 x0, then v = fma(f_q, x_q, v): every f x is exact, a
    // signed power of two or half of one, so each step rounds once, as a separate add would),
    // split into limbs and write the 16-byte limb chunks to LDS buffer st.
#define FUSED_STORE_SIDE(X, Q, NS, F, ROW, KC, S, st)                                                  \
    _Pragma("unroll") for (int u = 0; u < 2; ++u) {                                                    \
        float v[8];                                                                                    \
        _Pragma("unroll") for (int e = 0; e < 8; ++e) v[e] = F[u][0] * X[8 * (u * Q) + e];             \
        _Pragma("unroll") for (int q = 1; q < Q; ++q) {                                                \
            if (q < NS) {                                                                              \
                _Pragma("unroll") for (int e = 0; e < 8; ++e) v[e] =                                   \
                    __builtin_fmaf(F[u][q], X[8 * (u * Q + q) + e], v[e]);                             \
            }                                                                                          \
        }                                                                                              \
        unsigned short h[NL][8];                                                                       \
        _Pragma("unroll") for (int e = 0; e < 8; ++e) {                                                \
            float rr = v[e];                                                                           \
            _Pragma("unroll") for (int l = 0; l < NL; ++l) {                                           \
                float back;                                                                            \
                h[l][e] = LimbT<HALF>::split(rr, back);                                                \
                rr = rr - back;                                                                        \
            }                                                                                          \
        }                                                                                              \
        _Pragma("unroll") for (int l = 0; l < NL; ++l)                                                 \
            *reinterpret_cast<uint4 *>(&S[st][l][ROW[u] * RS + 8 * swz(ROW[u], KC[u])]) =              \
                uint4{(uint32_t)h[l][0] | ((uint32_t)h[l][1] << 16), (uint32_t)h[l][2] | ((uint32_t)h[l][3] << 16), \
                      (uint32_t)h[l][4] | ((uint32_t)h[l][5] << 16), (uint32_t)h[l][6] | ((uint32_t)h[l][7] << 16)}; \
    }
#define FUSED_STORE(st)                                   \
    FUSED_STORE_SIDE(xa, QA, na, fa_, rowa, kca, As, st) \
    FUSED_STORE_SIDE(xb, QB, nb, fb_, rowb, kcb, Bs, st)

    acc_t acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[i][j][v] = 0.f;
    const int g = lane >> 4, l16 = lane & 15;
    const int64_t nk = a.nk;
    FUSED_LOAD(0)
    FUSED_STORE(0)
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        const bool more = kt + 1 < nk;
        if (more) {
            FUSED_LOAD((kt + 1) * BK)
        }
        // one limb product at a time, its two fragment sets read from LDS just before use (the
        // raw chunks of the next stage take the registers that all products' fragments at once
        // would need)
        if constexpr (M32) {
            // two 16-k halves per stage; lane l reads row l % 32, chunk 2 h + l / 32
            const int l32 = lane & 31, hh = lane >> 5;
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int p = 0; p < P::n; ++p) {
                    gs8 fa[TI], fb[TJ];
#pragma unroll
                    for (int i = 0; i < TI; ++i) {
                        const int rr = wm * (BM / WM) + i * 32 + l32;
                        fa[i] = *reinterpret_cast<const gs8 *>(&As[cur][P::a[p]][rr * RS + 8 * swz(rr, 2 * h + hh)]);
                    }
#pragma unroll
                    for (int j = 0; j < TJ; ++j) {
                        const int rr = wn * (BN / WN) + j * 32 + l32;
                        fb[j] = *reinterpret_cast<const gs8 *>(&Bs[cur][P::b[p]][rr * RS + 8 * swz(rr, 2 * h + hh)]);
                    }
#pragma unroll
                    for (int i = 0; i < TI; ++i)
#pragma unroll
                        for (int j = 0; j < TJ; ++j) acc[i][j] = LimbT<HALF>::mma32(fa[i], fb[j], acc[i][j]);
                }
        } else {
#pragma unroll
            for (int p = 0; p < P::n; ++p) {
                gs8 fa[TI], fb[TJ];
#pragma unroll
                for (int i = 0; i < TI; ++i) {
                    const int rr = wm * (BM / WM) + i * 16 + l16;
                    fa[i] = *reinterpret_cast<const gs8 *>(&As[cur][P::a[p]][rr * RS + 8 * swz(rr, g)]);
                }
#pragma unroll
                for (int j = 0; j < TJ; ++j) {
                    const int rr = wn * (BN / WN) + j * 16 + l16;
                    fb[j] = *reinterpret_cast<const gs8 *>(&Bs[cur][P::b[p]][rr * RS + 8 * swz(rr, g)]);
                }
#pragma unroll
                for (int i = 0; i < TI; ++i)
#pragma unroll
                    for (int j = 0; j < TJ; ++j) acc[i][j] = LimbT<HALF>::mma(fa[i], fb[j], acc[i][j]);
            }
        }
        if (more) {  // the other buffer was last read before the previous barrier
            FUSED_STORE(cur ^ 1)
        }
        __syncthreads();
    }
#undef FUSED_LOAD
#undef FUSED_LOAD_SIDE
#undef FUSED_STORE_SIDE
#undef FUSED_STORE

    // Output: the leaf workspace, or (a single classical leaf) C with 2^(ea_i + eb_j) applied.
    const bool direct = a.direct != 0, scaled = a.sc.ea != nullptr;
    int ebj[TJ];
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
        const int64_t col = tn * BN + wn * (BN / WN) + j * MS + (M32 ? (lane & 31) : l16);
        ebj[j] = (direct && scaled && col < a.n) ? a.sc.eb[col] : 0;
    }
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int64_t row = tm * BM + wm * (BM / WM) + i * MS +
                                (M32 ? 8 * (v / 4) + 4 * (lane >> 5) + v % 4 : 4 * (lane >> 4) + v);
            const int eai = (direct && scaled && row < a.m) ? a.post_exp + a.sc.ea[row] : 0;
#pragma unroll
            for (int j = 0; j < TJ; ++j) {
                const int64_t col = tn * BN + wn * (BN / WN) + j * MS + (M32 ? (lane & 31) : l16);
                float val = acc[i][j][v];
                if (direct) {
                    if (row < a.m && col < a.n) {  // one power-of-two factor: exact unless it underflows
                        if (scaled) val = ldexpf(val, eai + ebj[j]);
                        a.out[row * a.ldo + col] = val;
                    }
                } else if (row < a.mb && col < a.nb) {
                    if (a.post_exp) val = ldexpf(val, a.post_exp);
                    a.out[(int64_t)leaf * a.leaf_stride + row * a.ldo + col] = val;
                }
            }
        }
}

template <bool HALF, int NL, int BM, int BN, int WM, int WN, int QA, int QB, bool M32>
__global__ __launch_bounds__(64 * WM * WN, 1) void fmm_limb_fused(LimbFused a) {
    __shared__ LimbSmem<NL, BM, BN> sm;
    const int64_t tiles = (int64_t)a.tiles_m * a.tiles_n;
    const int64_t item = xcd_remap_g(blockIdx.x, gridDim.x);
    const int leaf = __builtin_amdgcn_readfirstlane((int)(item / tiles));
    const int rem = __builtin_amdgcn_readfirstlane((int)(item - (int64_t)leaf * tiles));
    const int grp = rem / (8 * a.tiles_n);
    const int gsz = min(8, a.tiles_m - grp * 8);
    const int gidx = rem - grp * 8 * a.tiles_n;
    const int64_t tm = __builtin_amdgcn_readfirstlane(grp * 8 + gidx % gsz);
    const int64_t tn = __builtin_amdgcn_readfirstlane(gidx / gsz);
    limb_tile_fused<HALF, NL, BM, BN, WM, WN, QA, QB, M32>(a, leaf, tm, tn, sm);
}

// Item `item` (leaf-major, tiles in groups of 8 tile rows) of one problem -> (leaf, tm, tn).
__device__ __forceinline__ void limb_item(const LimbGemm &a, int64_t item, int &leaf, int64_t &tm, int64_t &tn) {
    const int64_t tiles = (int64_t)a.tiles_m * a.tiles_n;
    leaf = __builtin_amdgcn_readfirstlane((int)(item / tiles));
    const int rem = __builtin_amdgcn_readfirstlane((int)(item - (int64_t)leaf * tiles));
    const int grp = rem / (8 * a.tiles_n);
    const int gsz = min(8, a.tiles_m - grp * 8);
    const int gidx = rem - grp * 8 * a.tiles_n;
    tm = __builtin_amdgcn_readfirstlane(grp * 8 + gidx % gsz);
    tn = __builtin_amdgcn_readfirstlane(gidx / gsz);
}

template <bool HALF, int NL, int BM, int BN, int WM, int WN, bool SCALED, bool DIRECT>
__global__ __launch_bounds__(64 * WM * WN, 1) void fmm_limb_gemm(LimbGemm a) {
    __shared__ LimbSmem<NL, BM, BN> sm;
    int leaf;
    int64_t tm, tn;
    limb_item(a, xcd_remap_g(blockIdx.x, gridDim.x), leaf, tm, tn);
    limb_tile<HALF, NL, BM, BN, WM, WN, SCALED, DIRECT>(a, leaf, tm, tn, sm);
}

// Several problems in one launch: work-group w runs item w - first[q] of problem q, where
// first[q] <= w < first[q + 1] (problems ordered by the host, largest inner dimension first).
template <bool HALF, int NL, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN, 1) void fmm_limb_gemm_batched(const LimbGemm *__restrict__ descs,
                                                                       const int64_t *__restrict__ first, int count) {
    __shared__ LimbSmem<NL, BM, BN> sm;
    const int64_t w = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {  // last q with first[q] <= w
        const int mid = (lo + hi + 1) / 2;
        if (first[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    const int q = __builtin_amdgcn_readfirstlane(lo);
    const LimbGemm a = descs[q];
    int leaf;
    int64_t tm, tn;
    limb_item(a, w - first[q], leaf, tm, tn);
    limb_tile<HALF, NL, BM, BN, WM, WN, true, true, true>(a, leaf, tm, tn, sm);
}

template <bool HALF, int NL, int BM, int BN, int WM, int WN>
hipError_t gemm_go(const LimbGemm &g, int nleaves, hipStream_t s) {
    const int64_t blocks = (int64_t)g.tiles_m * g.tiles_n * nleaves;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const bool scaled = g.sc.ea != nullptr;
    const dim3 grid((unsigned)blocks), block(64 * WM * WN);
    if (g.direct) {
        if (scaled) hipLaunchKernelGGL((fmm_limb_gemm<HALF, NL, BM, BN, WM, WN, true, true>), grid, block, 0, s, g);
        else hipLaunchKernelGGL((fmm_limb_gemm<HALF, NL, BM, BN, WM, WN, false, true>), grid, block, 0, s, g);
    } else {
        hipLaunchKernelGGL((fmm_limb_gemm<HALF, NL, BM, BN, WM, WN, false, false>), grid, block, 0, s, g);
    }
    return hipGetLastError();
}

template <bool HALF, int NL, int BM, int BN, int WM, int WN>
hipError_t gemm_batched_go(const void *descs, const int64_t *first, int count, int64_t total, hipStream_t s) {
    if (total <= 0 || count <= 0) return hipSuccess;
    if (total > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((fmm_limb_gemm_batched<HALF, NL, BM, BN, WM, WN>), dim3((unsigned)total), dim3(64 * WM * WN), 0,
                       s, (const LimbGemm *)descs, first, count);
    return hipGetLastError();
}

template <bool HALF, int NL>
hipError_t gemm_batched_tile(int bm, const void *descs, const int64_t *first, int count, int64_t total,
                             hipStream_t s) {
    if constexpr (NL < 3) {
        if (bm == 256) return gemm_batched_go<HALF, NL, 256, 256, 4, 2>(descs, first, count, total, s);
    }
    return gemm_batched_go<HALF, NL, 128, 128, 2, 2>(descs, first, count, total, s);
}

template <bool HALF, int NL>
hipError_t gemm_tile(int bm, const LimbGemm &g, int nleaves, hipStream_t s) {
    if constexpr (NL < 3) {
        if (bm == 256) return gemm_go<HALF, NL, 256, 256, 4, 2>(g, nleaves, s);
    }
    return gemm_go<HALF, NL, 128, 128, 2, 2>(g, nleaves, s);
}

template <bool HALF, int NL, int QA, int QB>
hipError_t fused_go(const LimbFused &f, int nleaves, hipStream_t s) {
    const int64_t blocks = (int64_t)f.tiles_m * f.tiles_n * nleaves;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    if constexpr (NL < 3) {
        hipLaunchKernelGGL((fmm_limb_fused<HALF, NL, 256, 256, 2, 4, QA, QB, true>), dim3((unsigned)blocks), dim3(512), 0,
                           s, f);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

template <bool HALF, int NL>
hipError_t fused_q(const LimbFused &f, int qa, int qb, int nleaves, hipStream_t s) {
    if (qa <= 1 && qb <= 1) return fused_go<HALF, NL, 1, 1>(f, nleaves, s);
    if (qa <= 2 && qb <= 2) return fused_go<HALF, NL, 2, 2>(f, nleaves, s);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_limb_fused(int prec, const LimbFused &f, int nleaves, hipStream_t s) {
    const int qa = f.qa, qb = f.qb;  // most sources of a leaf on each side (the kernel's bound)
    switch (prec) {
        case FASTMM_BF16: return fused_q<false, 1>(f, qa, qb, nleaves, s);
        case FASTMM_F16: return fused_q<true, 1>(f, qa, qb, nleaves, s);
        case FASTMM_BF16X3: return fused_q<false, 2>(f, qa, qb, nleaves, s);
        case FASTMM_F16X3: return fused_q<true, 2>(f, qa, qb, nleaves, s);
    }
    return hipErrorInvalidValue;
}

int limb_count(int prec) {
    switch (prec) {
        case FASTMM_BF16:
        case FASTMM_F16: return 1;
        case FASTMM_BF16X3:
        case FASTMM_F16X3: return 2;
        case FASTMM_BF16X6: return 3;
    }
    return 0;
}

int limb_gemm_tile(int prec, int64_t mb, int64_t nb) {
    return (limb_count(prec) < 3 && mb >= 256 && nb >= 256) ? 256 : 128;
}

hipError_t launch_limb_gemm(int prec, int bm, const LimbGemm &g, int nleaves, hipStream_t s) {
    switch (prec) {
        case FASTMM_BF16: return gemm_tile<false, 1>(bm, g, nleaves, s);
        case FASTMM_F16: return gemm_tile<true, 1>(bm, g, nleaves, s);
        case FASTMM_BF16X3: return gemm_tile<false, 2>(bm, g, nleaves, s);
        case FASTMM_F16X3: return gemm_tile<true, 2>(bm, g, nleaves, s);
        case FASTMM_BF16X6: return gemm_tile<false, 3>(bm, g, nleaves, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_limb_gemm_batched(int prec, int bm, const void *descs, const int64_t *first, int count,
                                    int64_t total, hipStream_t s) {
    switch (prec) {
        case FASTMM_BF16: return gemm_batched_tile<false, 1>(bm, descs, first, count, total, s);
        case FASTMM_F16: return gemm_batched_tile<true, 1>(bm, descs, first, count, total, s);
        case FASTMM_BF16X3: return gemm_batched_tile<false, 2>(bm, descs, first, count, total, s);
        case FASTMM_F16X3: return gemm_batched_tile<true, 2>(bm, descs, first, count, total, s);
        case FASTMM_BF16X6: return gemm_batched_tile<false, 3>(bm, descs, first, count, total, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace fastmm
