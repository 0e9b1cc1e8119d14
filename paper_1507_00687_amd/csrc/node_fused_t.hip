// Fused one-level kernel (node_fused.h) for the transposes of the cyclic rotations of
// Strassen's rule and Winograd's variant: the rules of the backward products dA = G B^T and
// dB = A^T G (section 3.1: a rule for <M0,K0,N0> gives, transposed, one for <N0,K0,M0>).
#include "node_fused.h"

namespace fastmm {
namespace {

// (U+, U-, V+, V-, W+, W-) masks of the three transposed rotations of each rule, as the registry
// forms them (algo_transposed_rotation).
#define FASTMM_NODE222_T_PATTERNS(X)                                                   \
    X(0x168a815u, 0x8000020u, 0x4a50549u, 0x0400010u, 0xa321223u, 0x0800008u)          \
    X(0x4a50549u, 0x0400010u, 0xa321223u, 0x0800008u, 0x168a815u, 0x8000020u)          \
    X(0xa321223u, 0x0800008u, 0x168a815u, 0x8000020u, 0x4a50549u, 0x0400010u)          \
    X(0x70c0345u, 0x0910020u, 0xe2d7083u, 0x0000400u, 0xd808829u, 0x0023410u)          \
    X(0xe2d7083u, 0x0000400u, 0xd808829u, 0x0023410u, 0x70c0345u, 0x0910020u)          \
    X(0xd808829u, 0x0023410u, 0x70c0345u, 0x0910020u, 0xe2d7083u, 0x0000400u)

FASTMM_NODE_DISPATCH(FASTMM_NODE222_T_PATTERNS)

}  // namespace

bool node222_t_supported(const uint32_t masks[6]) { return node_match(masks); }

hipError_t launch_node222_t(const NodeLaunch &L, hipStream_t s) {
    bool found = false;
    return L.elem == Elem::F64 ? node_go<double>(L, s, &found) : node_go<float>(L, s, &found);
}

}  // namespace fastmm
