// Limb planes of the split precisions (pass 1 of their leaf products): for every leaf r, every
// element of S_r = sum_i u_ir A_i (eq. (2), the composite sources of the leaf, scaling exponents
// applied) is formed in FP32 and split into limbs x = x_1 + x_2 (+ x_3), x_1 = rn(x),
// x_2 = rn(x - x_1), x_3 = rn(x - x_1 - x_2) (round to nearest even in bf16 or fp16; each
// residual is exact in FP32).  The limbs are written as 16-bit planes with k contiguous; T_r is
// written transposed (T_r^T, n-rows by k), so both GEMM operands have k contiguous.  Planes are
// zero-padded to the GEMM tiles and blocked in (tile rows) x 32 k pieces (the layout the limb
// GEMM reads).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "devtypes.h"
#include "fastmm.h"
#include "launch.h"
#include "limbs.h"

namespace fastmm {
namespace {

// ------------------------------------------------------------------ pass 1: limb planes
constexpr int kFT = 64;  // formation tile: 64 plane rows by 64 k

template <bool HALF, int NL, bool SCALED, bool KCONTIG>
__global__ __launch_bounds__(256) void form_planes(PlaneForm a) {
    __shared__ float tile[kFT][kFT + 1];
    const int t = threadIdx.x;
    const int leaf = blockIdx.z;
    const int64_t o0 = (int64_t)blockIdx.y * kFT, k0 = (int64_t)blockIdx.x * kFT;
    const LeafEntry le = a.leaves[leaf];
    const int begin = __builtin_amdgcn_readfirstlane(a.b_side ? le.b_begin : le.a_begin);
    const int count = __builtin_amdgcn_readfirstlane(a.b_side ? le.b_count : le.a_count);
    // element e of this thread: consecutive lanes walk the operand's contiguous direction
    int lo[16], lk[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        if (KCONTIG) lo[e] = e * 4 + t / 64, lk[e] = t % 64;
        else lk[e] = e * 4 + t / 64, lo[e] = t % 64;
    }
    float v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = 0.f;
    for (int q = 0; q < count; ++q) {
        const SrcEntry se = a.src[begin + q];
        const int64_t bo = a.b_side ? se.bc : se.br, bk = a.b_side ? se.br : se.bc;
        const float c = se.coef;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int64_t ob = o0 + lo[e], kb = k0 + lk[e];  // inside the leaf block
            const int64_t o = bo * a.rb + ob, kk = bk * a.kb + kb;  // inside op(X)
            const bool ok = ob < a.rb && kb < a.kb && o < a.R && kk < a.K;
            const float y = *(ok ? a.X + o * a.ld_o + kk * a.ld_k : a.X);
            float x = ok ? y : 0.f;
            if (SCALED) x = ldexpf(x, a.s_o * a.e_o[ok ? o : 0] + a.s_k * a.e_k[ok ? kk : 0] + a.pre_exp);
            v[e] = (q == 0) ? c * x : v[e] + c * x;
        }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) tile[lo[e]][lk[e]] = v[e];
    __syncthreads();
    // 64 rows x 8 chunks of 8 k: split and write 16 bytes per limb
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int cidx = t + 256 * u, ro = cidx / 8, rk = (cidx % 8) * 8;
        unsigned short h[NL][8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float r = tile[ro][rk + j];
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                float back;
                h[l][j] = LimbT<HALF>::split(r, back);
                r = r - back;
            }
        }
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            uint4 w;
            w.x = (uint32_t)h[l][0] | ((uint32_t)h[l][1] << 16);
            w.y = (uint32_t)h[l][2] | ((uint32_t)h[l][3] << 16);
            w.z = (uint32_t)h[l][4] | ((uint32_t)h[l][5] << 16);
            w.w = (uint32_t)h[l][6] | ((uint32_t)h[l][7] << 16);
            const int64_t o = o0 + ro, kk = k0 + rk;  // blocked layout: (bt rows) x (32 k) tiles
            *reinterpret_cast<uint4 *>(a.planes + (int64_t)leaf * a.leaf_stride + l * a.plane_stride +
                                       ((o / a.bt) * (a.kp / 32) + kk / 32) * (a.bt * 32) + (o % a.bt) * 32 +
                                       kk % 32) = w;
        }
    }
}

// The dense leaves x blocks coefficient table of form_regs in LDS (zero where a block is not
// one of the leaf's sources); the caller synchronises before reading it.
template <int NT>
__device__ inline void leaf_coef_table(const PlaneForm &a, int nleaves, float *rcoef) {
    const int t = threadIdx.x;
    const int nbo = a.nbo, nbk = a.nbk, nblk = nbo * nbk;
    for (int i = t; i < nleaves * nblk; i += NT) rcoef[i] = 0.f;
    __syncthreads();
    for (int leaf = t; leaf < nleaves; leaf += NT) {
        const LeafEntry le = a.leaves[leaf];
        const int begin = a.b_side ? le.b_begin : le.a_begin, count = a.b_side ? le.b_count : le.a_count;
        for (int q = 0; q < count; ++q) {
            const SrcEntry se = a.src[begin + q];
            const int bo = a.b_side ? se.bc : se.br, bk = a.b_side ? se.br : se.bc;
            rcoef[leaf * nblk + (a.b_side ? bo * nbk + bk : bk * nbo + bo)] += se.coef;
        }
    }
}

// For every leaf: the sum of the thread's KW-element chunk x[b] of every block b with the leaf's
// coefficients, split into limbs and written to plane row ob, k kb0 .. kb0 + KW - 1.
template <bool HALF, int NL, int NB, int KW>
__device__ inline void write_leaves(const PlaneForm &a, int nleaves, const float *rcoef, int nblk,
                                    const float (&x)[NB][KW], int64_t ob, int64_t kb0) {
    const int64_t o = ob, kk = kb0;  // plane row and k
    unsigned short *dst0 =
        a.planes + ((o / a.bt) * (a.kp / 32) + kk / 32) * (a.bt * 32) + (o % a.bt) * 32 + kk % 32;
    for (int leaf = 0; leaf < nleaves; ++leaf) {
        float v[KW];
        bool first = true;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const float c = b < nblk ? rcoef[leaf * nblk + b] : 0.f;
            if (c != 0.f) {
#pragma unroll
                for (int j = 0; j < KW; ++j) v[j] = first ? c * x[b][j] : v[j] + c * x[b][j];
                first = false;
            }
        }
        if (first) {
#pragma unroll
            for (int j = 0; j < KW; ++j) v[j] = 0.f;
        }
        uint32_t h[NL][KW / 2];
#pragma unroll
        for (int j = 0; j < KW; ++j) {
            float r = v[j];
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                float back;
                const uint32_t bits = LimbT<HALF>::split(r, back);
                r = r - back;
                h[l][j / 2] = (j & 1) ? (h[l][j / 2] | (bits << 16)) : bits;
            }
        }
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            unsigned short *dst = dst0 + (int64_t)leaf * a.leaf_stride + l * a.plane_stride;
            if constexpr (KW == 8) *reinterpret_cast<uint4 *>(dst) = uint4{h[l][0], h[l][1], h[l][2], h[l][3]};
            else *reinterpret_cast<uint2 *>(dst) = uint2{h[l][0], h[l][1]};
        }
    }
}

// ------------------------------------------------------------------ pass 1, all leaves at once
constexpr int kAllMaxCoef = 4096;  // leaves x blocks entries of the coefficient table (dynamic LDS)

// The limb planes of every leaf with every source element read from HBM once: a work-group
// takes one TR x 8 KW tile position inside the leaf blocks; each thread owns one KW-element k
// chunk there (KW consecutive k of one plane row, i.e. 2 KW bytes of every limb plane), holds
// that chunk of every block of op(X) (the nbo x nbk leaf-block grid, NB >= blocks) in registers,
// and for each leaf sums the leaf's blocks with its coefficients (a dense leaves x blocks table in
// LDS, zero where a block is not one of its sources), splits and writes its limb chunks
// directly, with no LDS round trip and no barrier per leaf.  Blocks are summed in the order of
// the rule's single block index at depth 1 (column-major for A, row-major over (n-block,
// k-block) for B), which is the order of the source lists there.  Thread layout: k-contiguous
// operands (KCONTIG): eight consecutive lanes take the eight chunks of one row; otherwise (B, n
// contiguous) 16 consecutive lanes take 16 consecutive rows of one chunk.  Small work-groups (TR = 16 or 32 rows) let several run per CU out of phase
// (one loading while another writes); a 512-thread version with one 64 x 64 tile per
// work-group, and the earlier LDS-transposing version with a barrier per leaf, both ran 5 %
// slower.  For o-contiguous operands, passing the 32 x 32 source tiles of all blocks through
// LDS once so that the writes take the k-contiguous layout ran 1.4-1.7x slower (the tiles
// allow two work-groups per CU, also when each walks several positions and loads the next
// while writing).
template <bool HALF, int NL, bool SCALED, bool KCONTIG, int NB, int TR, int KW>
__global__ __launch_bounds__(TR * 8) void form_regs(PlaneForm a, int nleaves) {
    constexpr int NT = TR * 8;
    extern __shared__ float rcoef[];  // nleaves x nblk
    const int t = threadIdx.x;
    const int nbo = a.nbo, nbk = a.nbk, nblk = nbo * nbk;
    leaf_coef_table<NT>(a, nleaves, rcoef);
    static_assert(TR % 16 == 0 && TR <= 64, "tile rows");
    static_assert(KW == 8 || KW == 4, "chunk width");
    int ol, kc;  // the thread's row and KW-wide k chunk in the TR x 8 KW tile
    if (KCONTIG) {
        ol = t >> 3, kc = t & 7;
    } else {
        // o contiguous in op(X): a wave takes 16 consecutive rows by four chunks (16 k), so each
        // load reads 64-byte runs of four k rows and each limb store writes 32-byte runs of 16
        // plane rows.  Measured on this side: 32 rows by two chunks (whole 128-byte lines read,
        // 16-byte runs written) 15 % slower, 8 rows by eight chunks 3 %, work-groups of 16 or 64
        // rows 3-5 %.
        const int wave = t >> 6, lane = t & 63;
        ol = (lane & 15) + 16 * (wave % (TR / 16)), kc = (lane >> 4) + 4 * (wave / (TR / 16));
    }
    // work-group (row tile x, k tile y): consecutive work-groups take consecutive TR-row slices
    // of the same 32-k plane pieces, so the work-groups in flight write whole pieces together
    const int64_t ob = (int64_t)blockIdx.x * TR + ol, kb0 = (int64_t)blockIdx.y * (8 * KW) + KW * kc;  // in the leaf block
    const bool vec = KCONTIG && (a.ld_o & 3) == 0 && ((uintptr_t)a.X & 15) == 0;
    float x[NB][KW];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int bo = a.b_side ? b / nbk : b % nbo, bk = a.b_side ? b % nbk : b / nbo;
        const int64_t o = (int64_t)bo * a.rb + ob, kk0 = (int64_t)bk * a.kb + kb0;  // in op(X)
        const bool row_ok = b < nblk && ob < a.rb && o < a.R;
        if (vec && row_ok && kb0 + KW <= a.kb && kk0 + KW <= a.K) {
            const float4 *p = reinterpret_cast<const float4 *>(a.X + o * a.ld_o + kk0);
#pragma unroll
            for (int h = 0; h < KW / 4; ++h) {
                const float4 u = p[h];
                x[b][4 * h] = u.x, x[b][4 * h + 1] = u.y, x[b][4 * h + 2] = u.z, x[b][4 * h + 3] = u.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < KW; ++j) {
                const bool ok = row_ok && kb0 + j < a.kb && kk0 + j < a.K;
                const float y = *(ok ? a.X + o * a.ld_o + (kk0 + j) * a.ld_k : a.X);
                x[b][j] = ok ? y : 0.f;
            }
        }
        if (SCALED && row_ok) {  // once per element, not once per leaf that uses it (exact: powers of two)
            const int eo = a.s_o * a.e_o[o] + a.pre_exp;
#pragma unroll
            for (int j = 0; j < KW; ++j) {
                const int64_t kk = kk0 + j;
                const int ek = (kb0 + j < a.kb && kk < a.K) ? a.s_k * a.e_k[kk] : 0;
                x[b][j] = ldexpf(x[b][j], eo + ek);
            }
        }
    }
    __syncthreads();  // coefficient table complete
    write_leaves<HALF, NL, NB, KW>(a, nleaves, rcoef, nblk, x, ob, kb0);
}

template <bool HALF, int NL, int NB>
hipError_t form_regs_go(const PlaneForm &f, int nleaves, hipStream_t s) {
    // small work-groups (two waves when k is contiguous, four otherwise): several per CU, out
    // of phase (one loading while another writes)
    // four-element k chunks: a wave's limb writes cover eight whole 64-byte plane rows of one
    // 32-k piece (eight-element chunks, 7 % slower, split them over two pieces)
    constexpr int TRK = 16, TRO = 32, KW = 4;
    if (f.kp / (8 * KW) > 65535) return hipErrorInvalidValue;
    const bool scaled = f.e_o != nullptr, kc = f.ld_k == 1;
    const int tr = kc ? TRK : TRO;
    const dim3 grid((unsigned)(f.rowsp / tr), (unsigned)(f.kp / (8 * KW))), block(tr * 8);
    const size_t lds = (size_t)nleaves * f.nbo * f.nbk * sizeof(float);
    if (scaled && kc) hipLaunchKernelGGL((form_regs<HALF, NL, true, true, NB, TRK, KW>), grid, block, lds, s, f, nleaves);
    else if (scaled) hipLaunchKernelGGL((form_regs<HALF, NL, true, false, NB, TRO, KW>), grid, block, lds, s, f, nleaves);
    else if (kc) hipLaunchKernelGGL((form_regs<HALF, NL, false, true, NB, TRK, KW>), grid, block, lds, s, f, nleaves);
    else hipLaunchKernelGGL((form_regs<HALF, NL, false, false, NB, TRO, KW>), grid, block, lds, s, f, nleaves);
    return hipGetLastError();
}

template <bool HALF, int NL>
hipError_t form_go(const PlaneForm &f, int nleaves, hipStream_t s) {
    if (f.rowsp <= 0 || f.kp <= 0 || nleaves <= 0) return hipSuccess;
    if (f.rowsp / kFT > 65535 || nleaves > 65535 || f.kp / kFT > 0x7fffffffLL) return hipErrorInvalidValue;
    // every source block read once when the block grid and the coefficient table are small
    // (a single block, the classical product, needs no sharing: the per-leaf kernel below
    // holds fewer registers and streams faster)
    const int64_t nblk = (int64_t)f.nbo * f.nbk;
    if (f.nbo > 0 && f.nbk > 0 && nblk > 1 && nblk <= 16 && nblk * nleaves <= kAllMaxCoef) {
        if (nblk <= 4) return form_regs_go<HALF, NL, 4>(f, nleaves, s);
        if (nblk <= 8) return form_regs_go<HALF, NL, 8>(f, nleaves, s);
        return form_regs_go<HALF, NL, 16>(f, nleaves, s);
    }
    const dim3 grid((unsigned)(f.kp / kFT), (unsigned)(f.rowsp / kFT), (unsigned)nleaves);
    const bool scaled = f.e_o != nullptr, kc = f.ld_k == 1;
    if (scaled && kc) hipLaunchKernelGGL((form_planes<HALF, NL, true, true>), grid, dim3(256), 0, s, f);
    else if (scaled) hipLaunchKernelGGL((form_planes<HALF, NL, true, false>), grid, dim3(256), 0, s, f);
    else if (kc) hipLaunchKernelGGL((form_planes<HALF, NL, false, true>), grid, dim3(256), 0, s, f);
    else hipLaunchKernelGGL((form_planes<HALF, NL, false, false>), grid, dim3(256), 0, s, f);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_form_planes(int prec, const PlaneForm &f, int nleaves, hipStream_t s) {
    switch (prec) {
        case FASTMM_BF16: return form_go<false, 1>(f, nleaves, s);
        case FASTMM_F16: return form_go<true, 1>(f, nleaves, s);
        case FASTMM_BF16X3: return form_go<false, 2>(f, nleaves, s);
        case FASTMM_F16X3: return form_go<true, 2>(f, nleaves, s);
        case FASTMM_BF16X6: return form_go<false, 3>(f, nleaves, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace fastmm
