// Plain data shared by the host planner and the device kernels.
#pragma once

#include <cstdint>

namespace fastmm {

// One source block of a leaf operand: S_r (or T_r) = sum over entries of coef * block
// (br, bc) of the padded operand, blocks of the leaf size (eq. (2) unrolled over L levels:
// the composite coefficient is the product of the per-level coefficients, eq. (ST_exact)).
struct SrcEntry {
    int32_t br, bc;
    float coef;  // dyadic rationals: exact in float
    int32_t pad_;
};

// Per leaf: its A-source and B-source ranges in the SrcEntry arrays.
struct LeafEntry {
    int32_t a_begin, a_count, b_begin, b_count;
};

// One contribution to an output block: coef * M_leaf.
struct DestEntry {
    int32_t leaf;
    float coef;
};

// Per output block (row-major over the M0^L x N0^L block grid): its DestEntry range.
struct BlockDests {
    int32_t begin, count;
};

// Scaling state in device memory: power-of-two exponents of the cumulative factors.
//   A' = diag(2^-ea) op(A) diag(2^ep),   B' = diag(2^-ep) op(B) diag(2^-eb).
struct ScaleExps {
    const int32_t *ea;  // m (nullptr: no scaling)
    const int32_t *ep;  // k
    const int32_t *eb;  // n
};

}  // namespace fastmm
