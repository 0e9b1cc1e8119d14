// Fused one-level kernel (node_fused.h) for Strassen's rule, Winograd's variant and the two
// cyclic rotations of each; the entry points of both pattern sets.
#include "node_fused.h"

namespace fastmm {
namespace {

// The sign patterns compiled here: the rules as the registry holds them ((U+, U-, V+, V-, W+,
// W-) masks).  A rule is matched against them coefficient by coefficient, so a pattern is only
// ever used for a rule that equals it.
#define FASTMM_NODE222_PATTERNS(X)                                                     \
    X(0x1741115u, 0x8000020u, 0xa292423u, 0x0800008u, 0x4a28a49u, 0x0400010u)          \
    X(0x4a28a49u, 0x0400010u, 0x1741115u, 0x8000020u, 0xa292423u, 0x0800008u)          \
    X(0xa292423u, 0x0800008u, 0x4a28a49u, 0x0400010u, 0x1741115u, 0x8000020u)          \
    X(0x7019845u, 0x0802220u, 0xd840129u, 0x01a0410u, 0xe385a83u, 0x0020000u)          \
    X(0xe385a83u, 0x0020000u, 0x7019845u, 0x0802220u, 0xd840129u, 0x01a0410u)          \
    X(0xd840129u, 0x01a0410u, 0xe385a83u, 0x0020000u, 0x7019845u, 0x0802220u)

FASTMM_NODE_DISPATCH(FASTMM_NODE222_PATTERNS)

}  // namespace

bool node222_supported(const uint32_t masks[6]) { return node_match(masks) || node222_t_supported(masks); }

hipError_t launch_node222(const NodeLaunch &L, hipStream_t s) {
    bool found = false;
    const hipError_t e = L.elem == Elem::F64 ? node_go<double>(L, s, &found) : node_go<float>(L, s, &found);
    return found ? e : launch_node222_t(L, s);
}

}  // namespace fastmm
