// Host-side launchers of the device kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "devtypes.h"

namespace fastmm {

// Element type tag of a launch.
enum class Elem { F64, F32 };

// Leaf-product launch: every work-group computes one BMxBN tile of one leaf product
// M_r = S_r T_r, forming the S_r / T_r tiles from their source blocks while loading them
// (coefficients and scaling exponents applied in registers), and writes the tile either to
// the leaf workspace (direct == 0) or, for a single classical leaf, straight to C with the
// outside-scaling factors applied (direct == 1).
struct LeafLaunch {
    Elem elem;
    int prec;  // fastmm_precision
    const void *A;
    const void *B;
    void *out;
    int64_t lda, ldb, ldo;
    int transA, transB;
    int64_t m, k, n;
    int64_t mb, kb, nb;
    int64_t leaf_stride;
    int nleaves;
    const LeafEntry *leaves;
    const SrcEntry *asrc;
    const SrcEntry *bsrc;
    ScaleExps sc;
    int direct;
    int scale_in = 1;  // with sc and a direct output: 0 takes the operands as already scaled
                       // (only the output takes 2^(ea_i + eb_j)); row-major operands only
    int one = 0;       // every leaf has one A and one B source, coefficient 1 (row-major operands)
};

// W-combination: C_block(P,S) = sum over its DestEntry list of coef * M_leaf, then
// multiplied by 2^(ea_i + eb_j); writes every C element exactly once.
struct CombineLaunch {
    Elem elem;
    const void *M;  // leaf workspace
    int64_t leaf_stride;
    void *C;
    int64_t ldc;
    int64_t m, n, mb, nb;
    int NB;  // blocks per row of the output block grid (N0^L)
    const BlockDests *bdest;
    const DestEntry *dest;
    ScaleExps sc;
    // One or two levels of <2,K0,2> rules with at most 8 products each, every product live
    // (leaf r1 R2 + r2): kron = 1 sums C_p1 = sum_r1 w1[p1][r1] M_r1; kron = 2 sums level by
    // level, C_(p1,p2) = sum_r1 w1[p1][r1] sum_r2 w2[p2][r2] M_(r1,r2) (p = i N0 + j, output
    // block row 2 i1 + i2, column 2 j1 + j2); each product read once, the lists above unused.
    // kron = 3: one level of any rule with at most 16 output blocks (R2 of them, NB per row)
    // and at most 64 products (R1), every product live: the lists, expanded in LDS, are
    // summed from registers with each product read once.
    // kron = 4: two levels of one rule with at most 16 output blocks (M0 N0) and at most 64
    // products (R1 = R) that kron = 2 does not cover, level by level: the children of each
    // first-level node into its product (nodes: R blocks of M0 mb x N0 nb), then those into C,
    // both from the one-level lists bdest1 / dest1.
    int kron = 0;
    int R1 = 0, R2 = 0;
    float w1[4][8] = {}, w2[4][8] = {};
    const BlockDests *bdest1 = nullptr;
    const DestEntry *dest1 = nullptr;
    void *nodes = nullptr;
    int M0 = 0, N0 = 0;
};

// Node operands of the first recursion level, written out: node q (q < nodes) of op(X)
// (R x K, element (row, col) at X[row * ld_r + col * ld_c], zero outside) is the sum over its
// source list (A side: asrc of the depth-1 tables, B side: bsrc) of coef * block (br, bc), the
// blocks rb x cb; every element is multiplied by 2^(s_r e_r[row] + s_c e_c[col]) when e_r is
// not null.  Node q goes to Y + q * y_stride (rb x cb, row stride y_ld).
struct NodeDense {
    Elem elem;
    const void *X;
    int64_t ld_r, ld_c, R, K, rb, cb;
    const LeafEntry *nodes;
    const SrcEntry *src;
    int b_side;
    const int32_t *e_r, *e_c;
    int s_r, s_c;
    void *Y;
    int64_t y_stride, y_ld;
};

// Scaling-step reductions (Algorithms 1-3).  `kind` 'O' or 'I'.  Operands are op(A) (m x k)
// and op(B) (k x n).  `maxA`, `maxB` hold (m | k) and (k | n) maxima scratch of the element
// type; `exps` are updated in place; `flags` are two int32 (stop, fail) for the optional
// stopping test (tau > 0).
struct ScaleStep {
    Elem elem;
    char kind;
    const void *A;
    const void *B;
    int64_t lda, ldb;
    int transA, transB;
    int64_t m, k, n;
    int32_t *ea, *ep, *eb;
    void *maxA, *maxB;
    int32_t *flags;
    double tau;
    int test;       // apply the stopping test at this step
    int o_nearest;  // O step: power of two nearest to the max (else the smallest >= it)
};

// Fused one-level launch for <2,2,2;7> rules with coefficients in {0, +1, -1}: every
// work-group computes one 64x64 tile position of the four output sub-blocks of one node (a
// product of the outer L-1 levels, or the whole problem at depth 1), forming the node's
// operands from its outer sources, the seven S_r / T_r fragments, the products and the W-sums
// in one pass.  Sub-blocks are mb x kb (A) and kb x nb (B), i.e. the leaf blocks of the full
// recursion; node operands are 2mb x 2kb and 2kb x 2nb.  node_stride == 0: single node, the
// result goes to C (out / ldo) with the outside-scaling factors; otherwise node q's
// 2mb x 2nb product goes to out + q * node_stride (row stride 2nb).
struct NodeLaunch {
    Elem elem;
    const void *A;
    const void *B;
    void *out;
    int64_t lda, ldb, ldo;
    int64_t m, k, n;
    int64_t mb, kb, nb;
    int64_t node_stride;
    int nnodes;
    const LeafEntry *outer;
    const SrcEntry *asrc;
    const SrcEntry *bsrc;
    ScaleExps sc;       // the operands come scaled; sc scales the depth-1 output only
    uint32_t masks[6];  // (U+, U-, V+, V-, W+, W-): bit s*7+r marks coefficient +1 / -1
};
// Whether a compiled fused kernel exists for this sign pattern.
bool node222_supported(const uint32_t masks[6]);
// The same for the transposed-rotation patterns (node_fused_t.hip).
bool node222_t_supported(const uint32_t masks[6]);
hipError_t launch_node222_t(const NodeLaunch &L, hipStream_t s);
hipError_t launch_node222(const NodeLaunch &L, hipStream_t s);

// Split precisions, pass 1: limb planes of the leaf operands.  Plane row o, column kk of leaf
// r holds limb l of the leaf operand element (o, kk): for A, S_r(i, kk); for B, T_r(kk, j)
// transposed (o = j).  op(X)(o, kk) = X[o * ld_o + kk * ld_k] for o < R, kk < K; the leaf's
// source blocks (b_side: SrcEntry (br, bc) = (k block, o block)) are rb x kb; every value is
// multiplied by 2^(s_o e_o[o] + s_k e_k[kk]) when e_o is not null.  Planes are rowsp x kp
// (multiples of 64 and of bt; the padding is written as zeros), limb l of leaf r at
// planes + r * leaf_stride + l * plane_stride, blocked in bt x 32 pieces (see bt).
struct PlaneForm {
    const float *X;
    int64_t ld_o, ld_k;
    int64_t R, K;
    int64_t rb, kb;
    int64_t rowsp, kp;
    int64_t bt;  // plane blocking: element (o, kk) at ((o/bt)(kp/32) + kk/32)(32 bt) + (o%bt) 32 + kk%32
    const LeafEntry *leaves;
    const SrcEntry *src;
    int b_side;
    const int32_t *e_o, *e_k;
    int s_o, s_k;
    int pre_exp;  // with scaling (e_o not null): every value also times 2^pre_exp
    unsigned short *planes;
    int64_t plane_stride, leaf_stride;
    int nbo, nbk;  // leaf-block grid of op(X): nbo blocks along o, nbk along k (0: unknown)
};
// Pass 2: M_r = sum of the kept limb products of S_r and T_r, for every leaf and every
// bm x bm tile of the padded planes (bm = limb_gemm_tile); out is the leaf workspace (leaf r at out + r *
// leaf_stride, mb x nb, row stride ldo) or, with direct, C (m x n, ldc = ldo) with the
// outside-scaling factors 2^(ea_i + eb_j) applied.
struct LimbGemm {
    const unsigned short *S, *T;
    int64_t kp, s_plane, s_leaf, t_plane, t_leaf;
    float *out;
    int64_t ldo, leaf_stride, mb, nb, m, n;
    ScaleExps sc;
    int post_exp;  // every product times 2^post_exp (undoes the formation's pre_exp)
    int tiles_m, tiles_n;
    int direct;
};
// Split precisions with the innermost recursion level formed in the GEMM's tile loads (eq. (1)
// applied while staging).  Leaf (node q = leaf / R, innermost product r = leaf % R) multiplies
// S_r = sum_i U_ir X_i by T_r = sum_j V_jr Y_j, where X_i are the sub-blocks of node q's A operand
// and Y_j those of its B operand.  Both operands are FP32 with k contiguous: the A operand row-
// major (rows of m), the B operand stored transposed (rows of n).  Sub-block i of the A operand
// sits at row block i % M0, k block i / M0; sub-block j of the B operand at row block j / K0, k
// block j % K0 (eq. (1): blocks column-major).  S_r and T_r^T are formed in FP32 from the loaded
// tiles, sources in increasing index order, split into limbs and staged in LDS for the limb
// products, so no limb planes are written.
struct FusedSide {
    const float *X;             // node q's operand at X + q * node_stride, row stride ld
    int64_t ld, node_stride;
    int64_t rows, cols;         // valid extent of a node operand (zero beyond: virtual padding)
    int64_t sb_rows;            // rows of a sub-block (mb or nb); its k extent is LimbFused::kb
    const int32_t *e_row;       // outside scaling: row r of the operand times 2^(s_row e_row[r] + pre_exp)
    int s_row, pre_exp;
};
struct LimbFused {
    FusedSide a, b;
    const float *ucoef, *vcoef;  // innermost rule: U (M0 K0 x R) and V (K0 N0 x R), row-major
    int M0, K0, N0, R;
    int qa, qb;                  // most nonzeros in a column of U, of V (<= 2)
    int64_t kb, nk;              // leaf inner dimension, and its 32-k stages
    float *out;
    int64_t ldo, leaf_stride, mb, nb, m, n;
    ScaleExps sc;
    int post_exp;
    int tiles_m, tiles_n;
    int direct;
};
hipError_t launch_limb_fused(int prec, const LimbFused &f, int nleaves, hipStream_t s);
// Operand formation level by level (split precisions; written-out leaf operands of the FP64 /
// FP32 paths): one recursion level.  Elements are double for FP64, float otherwise.  The
// node operand of node q is op(X) itself on the first level (element (o, kk) at
// X[o * ld_o + kk * ld_k], zero outside R x K, scaled by 2^(s_o e_o[o] + s_k e_k[kk] + pre_exp)
// when e_o is not null) or, below it, the block X + q * node_stride (element (o, kk) at
// o * ld_o + kk).  It has nO x nK sub-blocks of cb_o x cb_k; sub-block s sits at o-block
// (side_b ? s / nK : s % nO) and k-block (side_b ? s % nK : s / nO) (eq. (1): A and B blocks
// column-major).  Child c = sum_s coef[s * R_ + c] X_s of node q gets index q * R_ + c and is
// written either as limb planes (last: same layout as PlaneForm, rowsp x kp, blocked by bt) or as
// a block Y + index * y_stride: o-major with row stride y_ld (a multiple of 8, >= cb_k; columns
// cb_k .. y_ld-1 written as zeros) or, with kmajor, k-major (cb_k rows of y_ld >= cb_o, a
// multiple of 8; columns cb_o .. y_ld-1 written as zeros).
struct NodeForm {
    const void *X;  // float (split precisions, FP32) or double (FP64) elements
    int64_t ld_o, ld_k, R, K;
    int64_t node_stride;
    int first;
    int nO, nK, side_b, R_;
    const float *coef;
    int64_t coef_stride;  // node q's coefficients at coef + q coef_stride (0: one table for all)
    int64_t cb_o, cb_k;
    const int32_t *e_o, *e_k;
    int s_o, s_k, pre_exp;
    int last;
    void *Y;
    int64_t y_stride, y_ld;
    int kmajor;  // FP blocks written k-major (element (o, kk) at kk * y_ld + o; y_ld a multiple of 8)
    unsigned short *planes;
    int64_t rowsp, kp, bt, plane_stride, leaf_stride;
    int nl, half;  // set by launch_form_node from the precision
};
hipError_t launch_form_node(int prec, const NodeForm &f, int nodes, hipStream_t s);
int limb_count(int prec);                   // limbs per element of a split precision
int limb_gemm_tile(int prec, int64_t mb, int64_t nb);  // square tile of the limb GEMM (128 or 256)
hipError_t launch_form_planes(int prec, const PlaneForm &f, int nleaves, hipStream_t s);
hipError_t launch_limb_gemm(int prec, int bm, const LimbGemm &g, int nleaves, hipStream_t s);
// Several problems in one launch: descs holds count LimbGemm descriptors (device memory, all
// with planes blocked for the tile bm), first[count + 1] the prefix sums of their items
// (leaves x tiles); `total` = first[count] work-groups.
hipError_t launch_limb_gemm_batched(int prec, int bm, const void *descs, const int64_t *first, int count,
                                    int64_t total, hipStream_t s);

hipError_t launch_leaf(const LeafLaunch &L, hipStream_t s);
// Pipelined 128x128-tile version for row-major (non-transposed) operands.
hipError_t launch_leaf_pipelined(const LeafLaunch &L, hipStream_t s);
// Batched version (row-major operands, FP64/FP32): leaf_desc_build writes the device
// descriptor of one problem's launch to `dst` (leaf_desc_bytes(e) bytes, host memory) and
// returns its number of work items; launch_leaf_batched runs `total` items of `count` problems
// that share one mode (scaled operands or not, output to C or to the leaf workspace, one: every
// leaf with one source of coefficient 1, unscaled), with the descriptors and the item prefix
// offsets first[count + 1] in device memory, one work-group per item.
size_t leaf_desc_bytes(Elem e);
int64_t leaf_desc_build(const LeafLaunch &L, void *dst);
hipError_t launch_leaf_batched(Elem e, int scaled, int direct, int one, const void *descs, const int64_t *first,
                               int count, int64_t total, hipStream_t s);
// out (C x R) = in^T for a row-major R x C matrix (FP32 or FP64).
hipError_t launch_transpose(Elem e, const void *in, int64_t ldi, int64_t R, int64_t C, void *out, int64_t ldo,
                            hipStream_t s);
hipError_t launch_combine(const CombineLaunch &L, hipStream_t s);
hipError_t launch_node_dense(const NodeDense &f, int nodes, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t value, hipStream_t s);
hipError_t launch_zero_elems(Elem e, void *C, int64_t ldc, int64_t m, int64_t n, hipStream_t s);
hipError_t launch_scale_step(const ScaleStep &S, hipStream_t s);

}  // namespace fastmm
