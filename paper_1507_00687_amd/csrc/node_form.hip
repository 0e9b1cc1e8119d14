// Node operands written out one recursion level at a time (eq. (2)): form_node (LDS-staged,
// any orientation, limb planes at the last level of the split precisions) and
// form_node_direct (register-only, where the operand keeps its orientation).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "devtypes.h"
#include "fastmm.h"
#include "launch.h"
#include "limbs.h"

namespace fastmm {
namespace {

// ------------------------------------------------------------------ pass 1, level by level
// One recursion level of the operand formation for a node operand X (eq. (1)): the node's nS
// sub-blocks X_s are read once and all R children C_c = sum_s coef[s][c] X_s are written, as
// blocks of the element type T (inner levels, and every level of the FP64 / FP32 paths) or as
// limb planes (last level of the split precisions, T = float).  Each work-group handles a
// TO x 64 tile position (o, kk) of the child blocks: it stages the nS sub-block tiles in LDS,
// then forms every child tile from them (for an operand with o contiguous written o-major, a
// register-only form with 16-row x 16-k waves, 64-byte runs both ways, ran 12 % slower than
// this staged one, whose stores write whole 256-byte rows).  Children of node q are numbered
// q R + c, the order of the composite leaves (first level most significant).  Blocks are
// written o-major (element (o, kk) at o * y_ld + kk) or, with kmajor, k-major (element (o, kk)
// at kk * y_ld + o: a B-side operand written back in its own row-major k x n orientation).
template <typename T, int TO>
__global__ __launch_bounds__(256) void form_node(NodeForm a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char node_lds[];
    T *ntile = reinterpret_cast<T *>(node_lds);  // [nS][TO][65], then the nS x R_ coefficients
    const int t = threadIdx.x;
    const int q = blockIdx.z;
    const int64_t o0 = (int64_t)blockIdx.y * TO, k0 = (int64_t)blockIdx.x * 64;
    const int nS = a.nO * a.nK;
    const bool kc = a.ld_k == 1;
    const T *X = reinterpret_cast<const T *>(a.X) + (a.first ? 0 : (int64_t)q * a.node_stride);
    float *coef = reinterpret_cast<float *>(ntile + nS * TO * 65);
    for (int i = t; i < nS * a.R_; i += 256) coef[i] = a.coef[(int64_t)q * a.coef_stride + i];
    for (int sb = 0; sb < nS; ++sb) {
        const int ob = a.side_b ? sb / a.nK : sb % a.nO, kbk = a.side_b ? sb % a.nK : sb / a.nO;
        for (int e = t; e < TO * 64; e += 256) {
            // consecutive lanes along the operand's contiguous direction
            const int lo = kc ? e / 64 : e % TO, lk = kc ? e % 64 : e / TO;
            const int64_t oc = o0 + lo, kcn = k0 + lk;  // inside the child block
            const int64_t o = ob * a.cb_o + oc, kk = kbk * a.cb_k + kcn;  // inside the node operand
            bool ok = oc < a.cb_o && kcn < a.cb_k;
            if (a.first) ok = ok && o < a.R && kk < a.K;
            const T y = *(ok ? X + o * a.ld_o + kk * a.ld_k : X);
            T x = ok ? y : T(0);
            if (a.first && a.e_o) x = ldexp(x, a.s_o * a.e_o[ok ? o : 0] + a.s_k * a.e_k[ok ? kk : 0] + a.pre_exp);
            ntile[(sb * TO + lo) * 65 + lk] = x;
        }
    }
    __syncthreads();
    T *Y = reinterpret_cast<T *>(a.Y);
    if (!a.last && a.kmajor) {
        // (child, k row, 8-wide o chunk): eight consecutive o of one k row per thread, read down
        // a column of the staged tiles (row stride 65: distinct banks)
        constexpr int OC = TO / 8;
        for (int w = t; w < a.R_ * 64 * OC; w += 256) {
            const int c = w / (64 * OC), task = w - c * (64 * OC);
            const int rk = task / OC, ro = (task % OC) * 8;
            T v[8];
            bool first = true;
            for (int sb = 0; sb < nS; ++sb) {
                const float u = coef[sb * a.R_ + c];
                if (u == 0.f) continue;
                const T *src = &ntile[(sb * TO + ro) * 65 + rk];
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = first ? (T)u * src[j * 65] : v[j] + (T)u * src[j * 65];
                first = false;
            }
            if (first) {
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = T(0);
            }
            const int64_t child = (int64_t)q * a.R_ + c, o = o0 + ro, kk = k0 + rk;
            if (kk < a.cb_k && o < a.y_ld) {
                T *dst = Y + child * a.y_stride + kk * a.y_ld + o;
                if constexpr (sizeof(T) == 4) {
                    *reinterpret_cast<float4 *>(dst) = make_float4(v[0], v[1], v[2], v[3]);
                    *reinterpret_cast<float4 *>(dst + 4) = make_float4(v[4], v[5], v[6], v[7]);
                } else {
#pragma unroll
                    for (int j = 0; j < 8; j += 2) *reinterpret_cast<double2 *>(dst + j) = make_double2(v[j], v[j + 1]);
                }
            }
        }
        return;
    }
    // (child, task) pairs flattened, so that every thread has work when TO x 8 < 256
    for (int w = t; w < a.R_ * TO * 8; w += 256) {
        const int c = w / (TO * 8), task = w - c * (TO * 8);
        // eight consecutive lanes cover one row's 64 k, so a wave writes whole rows: 256
        // contiguous bytes of an FP32 child, or two 512-byte runs of a plane piece (rows of
        // a piece are adjacent).  The LDS row stride of 65 words keeps the reads at most
        // two-way bank conflicted.
        const int ro = task / 8, rk = (task % 8) * 8;
        T v[8];
        bool first = true;
        for (int sb = 0; sb < nS; ++sb) {
            const float u = coef[sb * a.R_ + c];
            if (u == 0.f) continue;
            const T *src = &ntile[(sb * TO + ro) * 65 + rk];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = first ? (T)u * src[j] : v[j] + (T)u * src[j];
            first = false;
        }
        if (first) {
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = T(0);
        }
        const int64_t child = (int64_t)q * a.R_ + c, o = o0 + ro, kk = k0 + rk;
        if constexpr (sizeof(T) == 4) {
            if (a.last) {
                unsigned short h[3][8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    float r = v[j];
#pragma unroll
                    for (int l = 0; l < 3; ++l) {
                        float back;
                        h[l][j] = a.half ? LimbT<true>::split(r, back) : LimbT<false>::split(r, back);
                        r = r - back;
                    }
                }
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    if (l >= a.nl) break;
                    uint4 w;
                    w.x = (uint32_t)h[l][0] | ((uint32_t)h[l][1] << 16);
                    w.y = (uint32_t)h[l][2] | ((uint32_t)h[l][3] << 16);
                    w.z = (uint32_t)h[l][4] | ((uint32_t)h[l][5] << 16);
                    w.w = (uint32_t)h[l][6] | ((uint32_t)h[l][7] << 16);
                    *reinterpret_cast<uint4 *>(a.planes + child * a.leaf_stride + l * a.plane_stride +
                                               ((o / a.bt) * (a.kp / 32) + kk / 32) * (a.bt * 32) + (o % a.bt) * 32 +
                                               kk % 32) = w;
                }
                continue;
            }
        }
        if (o < a.cb_o && kk < a.y_ld) {
            T *dst = Y + child * a.y_stride + o * a.y_ld + kk;
            if constexpr (sizeof(T) == 4) {
                *reinterpret_cast<float4 *>(dst) = make_float4(v[0], v[1], v[2], v[3]);
                *reinterpret_cast<float4 *>(dst + 4) = make_float4(v[4], v[5], v[6], v[7]);
            } else {
#pragma unroll
                for (int j = 0; j < 8; j += 2) *reinterpret_cast<double2 *>(dst + j) = make_double2(v[j], v[j + 1]);
            }
        }
    }
}

// form_node without the LDS stage, where the operand's contiguous direction is the output's
// (k for o-major blocks, o for k-major ones: every level of row-major operands): a thread holds
// V consecutive elements of one row of each of the nS sub-blocks in registers (one 16-byte load
// each where aligned and inside the block) and writes V elements of every child, summing the
// sub-blocks in the same order with the same operations as form_node (bitwise equal results).
// Rows r and the contiguous position p of the child block: (o, kk) for o-major output, (kk, o)
// for k-major; p runs over the padded row length y_ld, whose padding is written as zeros.
template <typename T, int MAXS>
__global__ __launch_bounds__(256) void form_node_direct(NodeForm a, int64_t rows, int64_t chunks) {
    constexpr int V = 16 / (int)sizeof(T);
    typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type vec_t;
    const int64_t item = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (item >= rows * chunks) return;
    const int q = blockIdx.z;
    const int64_t r = item / chunks, p0 = (item - r * chunks) * V;
    const bool km = a.kmajor != 0;
    const int64_t oc0 = km ? p0 : r, kc0 = km ? r : p0;  // child block coordinates of element 0
    const int64_t step_o = km ? 1 : 0, step_k = km ? 0 : 1;
    const int nS = a.nO * a.nK;
    const T *X = reinterpret_cast<const T *>(a.X) + (a.first ? 0 : (int64_t)q * a.node_stride);
    const int64_t ld_p = km ? a.ld_o : a.ld_k;  // 1 here
    T x[MAXS][V];
#pragma unroll
    for (int sb = 0; sb < MAXS; ++sb) {
        if (sb >= nS) continue;  // (not break: a fully unrolled loop keeps x in registers)
        const int ob = a.side_b ? sb / a.nK : sb % a.nO, kbk = a.side_b ? sb % a.nK : sb / a.nO;
        const int64_t o0 = ob * a.cb_o + oc0, k0 = kbk * a.cb_k + kc0;  // inside the node operand
        const T *src = X + o0 * a.ld_o + k0 * a.ld_k;
        // all V elements inside the child block and the operand, and 16-byte aligned
        const bool in_blk = km ? (oc0 + V <= a.cb_o && kc0 < a.cb_k) : (kc0 + V <= a.cb_k && oc0 < a.cb_o);
        const bool in_op = !a.first || (km ? (o0 + V <= a.R && k0 < a.K) : (k0 + V <= a.K && o0 < a.R));
        if (in_blk && in_op && ld_p == 1 && ((uintptr_t)src & 15) == 0) {
            const vec_t w = *reinterpret_cast<const vec_t *>(src);
            const T *ws = reinterpret_cast<const T *>(&w);
#pragma unroll
            for (int j = 0; j < V; ++j) x[sb][j] = ws[j];
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const int64_t oc = oc0 + j * step_o, kcn = kc0 + j * step_k;
                bool ok = oc < a.cb_o && kcn < a.cb_k;
                const int64_t o = ob * a.cb_o + oc, kk = kbk * a.cb_k + kcn;
                if (a.first) ok = ok && o < a.R && kk < a.K;
                const T y = *(ok ? X + o * a.ld_o + kk * a.ld_k : X);
                x[sb][j] = ok ? y : T(0);
            }
        }
        if (a.first && a.e_o) {
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const int64_t oc = oc0 + j * step_o, kcn = kc0 + j * step_k;
                const int64_t o = ob * a.cb_o + oc, kk = kbk * a.cb_k + kcn;
                const bool ok = oc < a.cb_o && kcn < a.cb_k && o < a.R && kk < a.K;
                x[sb][j] = ldexp(x[sb][j], a.s_o * a.e_o[ok ? o : 0] + a.s_k * a.e_k[ok ? kk : 0] + a.pre_exp);
            }
        }
    }
    T *Y = reinterpret_cast<T *>(a.Y);
    for (int c = 0; c < a.R_; ++c) {
        T v[V];
        bool first = true;
#pragma unroll
        for (int sb = 0; sb < MAXS; ++sb) {
            const float u = sb < nS ? a.coef[(int64_t)q * a.coef_stride + sb * a.R_ + c] : 0.f;
            if (u == 0.f) continue;
#pragma unroll
            for (int j = 0; j < V; ++j) v[j] = first ? (T)u * x[sb][j] : v[j] + (T)u * x[sb][j];
            first = false;
        }
        if (first) {
#pragma unroll
            for (int j = 0; j < V; ++j) v[j] = T(0);
        }
        vec_t w;
        T *ws = reinterpret_cast<T *>(&w);
#pragma unroll
        for (int j = 0; j < V; ++j) ws[j] = v[j];
        const int64_t child = (int64_t)q * a.R_ + c;
        *reinterpret_cast<vec_t *>(Y + child * a.y_stride + r * a.y_ld + p0) = w;
    }
}

// The last level of form_node (limb planes) without the LDS stage, for inner node operands whose
// k is contiguous (o-major blocks): a thread owns one 8-element chunk of a leaf plane (rows o of
// a bt x 32 piece, k in steps of 8), numbered in the planes' memory order, so that consecutive
// threads write consecutive 16 bytes and four threads read one 128-byte row segment of each
// sub-block.  It holds the 8 elements of each of the nS sub-blocks in registers and writes that
// chunk of every child's limb planes, with the same sums and splits as form_node (bitwise equal
// planes).  Elements outside the child block (the planes' padding) are zeros.
template <int MAXS>
__global__ __launch_bounds__(256) void form_planes_direct(NodeForm a, int64_t chunks) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= chunks) return;
    const int q = blockIdx.z;
    const int64_t per_piece = a.bt * 4, kpieces = a.kp / 32;
    const int64_t piece = g / per_piece, w = g - piece * per_piece;
    const int64_t oc = (piece / kpieces) * a.bt + w / 4, kc0 = (piece % kpieces) * 32 + (w % 4) * 8;
    const int nS = a.nO * a.nK;
    const float *X = reinterpret_cast<const float *>(a.X) + (int64_t)q * a.node_stride;
    float x[MAXS][8];
#pragma unroll
    for (int sb = 0; sb < MAXS; ++sb) {
        if (sb >= nS) continue;  // (not break: a fully unrolled loop keeps x in registers)
        const int ob = a.side_b ? sb / a.nK : sb % a.nO, kbk = a.side_b ? sb % a.nK : sb / a.nO;
        const float *src = X + (ob * a.cb_o + oc) * a.ld_o + kbk * a.cb_k + kc0;
        if (oc < a.cb_o && kc0 + 8 <= a.cb_k && ((uintptr_t)src & 15) == 0) {
            const float4 u0 = *reinterpret_cast<const float4 *>(src);
            const float4 u1 = *reinterpret_cast<const float4 *>(src + 4);
            x[sb][0] = u0.x, x[sb][1] = u0.y, x[sb][2] = u0.z, x[sb][3] = u0.w;
            x[sb][4] = u1.x, x[sb][5] = u1.y, x[sb][6] = u1.z, x[sb][7] = u1.w;
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const bool ok = oc < a.cb_o && kc0 + j < a.cb_k;
                const float y = *(ok ? src + j : X);
                x[sb][j] = ok ? y : 0.f;
            }
        }
    }
    for (int c = 0; c < a.R_; ++c) {
        float v[8];
        bool first = true;
#pragma unroll
        for (int sb = 0; sb < MAXS; ++sb) {
            const float u = sb < nS ? a.coef[(int64_t)q * a.coef_stride + sb * a.R_ + c] : 0.f;
            if (u == 0.f) continue;
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = first ? u * x[sb][j] : v[j] + u * x[sb][j];
            first = false;
        }
        if (first) {
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = 0.f;
        }
        unsigned short h[3][8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float r = v[j];
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                float back;
                h[l][j] = a.half ? LimbT<true>::split(r, back) : LimbT<false>::split(r, back);
                r = r - back;
            }
        }
        unsigned short *dst = a.planes + ((int64_t)q * a.R_ + c) * a.leaf_stride + g * 8;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            if (l >= a.nl) break;
            uint4 wv;
            wv.x = (uint32_t)h[l][0] | ((uint32_t)h[l][1] << 16);
            wv.y = (uint32_t)h[l][2] | ((uint32_t)h[l][3] << 16);
            wv.z = (uint32_t)h[l][4] | ((uint32_t)h[l][5] << 16);
            wv.w = (uint32_t)h[l][6] | ((uint32_t)h[l][7] << 16);
            *reinterpret_cast<uint4 *>(dst + l * a.plane_stride) = wv;
        }
    }
}

}  // namespace

hipError_t launch_form_node(int prec, const NodeForm &f, int nodes, hipStream_t s) {
    NodeForm a = f;
    a.nl = limb_count(prec);
    a.half = (prec == FASTMM_F16 || prec == FASTMM_F16X3) ? 1 : 0;
    const bool dbl = prec == FASTMM_F64;
    if (a.last && (dbl || prec == FASTMM_F32)) return hipErrorInvalidValue;  // planes: split precisions only
    const int nS = a.nO * a.nK;
    if (nS < 1 || nS > 16 || nodes <= 0) return nodes <= 0 ? hipSuccess : hipErrorInvalidValue;
    const int TO = nS <= 4 ? 32 : (nS <= 8 ? 16 : 8);
    // extent of the child blocks the grid covers: planes (rowsp x kp), o-major blocks
    // (cb_o x y_ld) or k-major blocks (y_ld x cb_k, o along the rows' contiguous direction)
    const int64_t ext_o = a.last ? a.rowsp : (a.kmajor ? a.y_ld : a.cb_o);
    const int64_t ext_k = a.last ? a.kp : (a.kmajor ? a.cb_k : a.y_ld);
    const int64_t gx = (ext_k + 63) / 64, gy = (ext_o + TO - 1) / TO;
    if (gx <= 0 || gy <= 0) return hipSuccess;
    if (gx > 0x7fffffffLL || gy > 65535 || nodes > 65535) return hipErrorInvalidValue;
    if (a.kmajor && (a.y_ld % 8 != 0)) return hipErrorInvalidValue;
    // limb planes from k-contiguous inner node operands: no LDS transpose needed
    if (a.last && !a.first && a.ld_k == 1 && a.bt > 0 && a.rowsp % a.bt == 0 && a.kp % 32 == 0 &&
        ((uintptr_t)a.planes & 15) == 0 && a.plane_stride % 8 == 0 && a.leaf_stride % 8 == 0) {
        const int64_t chunks = a.rowsp * a.kp / 8, blocks = (chunks + 255) / 256;
        if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
        const dim3 g((unsigned)blocks, 1, (unsigned)nodes);
        if (nS <= 4) hipLaunchKernelGGL((form_planes_direct<4>), g, dim3(256), 0, s, a, chunks);
        else if (nS <= 8) hipLaunchKernelGGL((form_planes_direct<8>), g, dim3(256), 0, s, a, chunks);
        else hipLaunchKernelGGL((form_planes_direct<16>), g, dim3(256), 0, s, a, chunks);
        return hipGetLastError();
    }
    // the operand's contiguous direction is the output's: no LDS transpose needed
    const bool direct = !a.last && ((a.ld_k == 1 && !a.kmajor) || (a.ld_o == 1 && a.kmajor)) && a.y_ld % 8 == 0 &&
                        ((uintptr_t)a.Y & 15) == 0 && a.y_stride % 8 == 0;
    if (direct) {
        const int64_t rows = a.kmajor ? a.cb_k : a.cb_o, chunks = a.y_ld / (dbl ? 2 : 4);
        const int64_t blocks = (rows * chunks + 255) / 256;
        if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
        const dim3 g((unsigned)blocks, 1, (unsigned)nodes);
        if (dbl) {
            if (nS <= 4) hipLaunchKernelGGL((form_node_direct<double, 4>), g, dim3(256), 0, s, a, rows, chunks);
            else if (nS <= 8) hipLaunchKernelGGL((form_node_direct<double, 8>), g, dim3(256), 0, s, a, rows, chunks);
            else hipLaunchKernelGGL((form_node_direct<double, 16>), g, dim3(256), 0, s, a, rows, chunks);
        } else {
            if (nS <= 4) hipLaunchKernelGGL((form_node_direct<float, 4>), g, dim3(256), 0, s, a, rows, chunks);
            else if (nS <= 8) hipLaunchKernelGGL((form_node_direct<float, 8>), g, dim3(256), 0, s, a, rows, chunks);
            else hipLaunchKernelGGL((form_node_direct<float, 16>), g, dim3(256), 0, s, a, rows, chunks);
        }
        return hipGetLastError();
    }
    const dim3 grid((unsigned)gx, (unsigned)gy, (unsigned)nodes);
    const size_t es = dbl ? sizeof(double) : sizeof(float);
    const size_t lds = (size_t)nS * TO * 65 * es + (size_t)nS * a.R_ * sizeof(float);
    if (dbl) {
        if (TO == 32) hipLaunchKernelGGL((form_node<double, 32>), grid, dim3(256), lds, s, a);
        else if (TO == 16) hipLaunchKernelGGL((form_node<double, 16>), grid, dim3(256), lds, s, a);
        else hipLaunchKernelGGL((form_node<double, 8>), grid, dim3(256), lds, s, a);
    } else {
        if (TO == 32) hipLaunchKernelGGL((form_node<float, 32>), grid, dim3(256), lds, s, a);
        else if (TO == 16) hipLaunchKernelGGL((form_node<float, 16>), grid, dim3(256), lds, s, a);
        else hipLaunchKernelGGL((form_node<float, 8>), grid, dim3(256), lds, s, a);
    }
    return hipGetLastError();
}

}  // namespace fastmm
