// C ABI of the library: argument checking, the recursion planner (levels, padding, the
// composite leaf task tables of eq. (2)), the scaling schedule of Algorithms 1-3 and the
// launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "devtypes.h"
#include "fastmm.h"
#include "fastmm_internal.h"
#include "launch.h"

namespace fastmm {

namespace {
thread_local std::string g_last_error;

// Phase timing (fastmm_profile_enable): events recorded around each phase of each call:
// scaling, operand formation (split precisions), products, W-combination.
constexpr int kPhases = 4;
struct PhaseEvents {
    hipEvent_t ev[kPhases + 1];
};
struct Profiler {
    bool on = false;
    std::vector<PhaseEvents> pending;
    std::vector<hipEvent_t> pool;
    double ms[kPhases] = {0, 0, 0, 0};
    int calls = 0;
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
};
thread_local Profiler g_prof;
}

void set_error(const std::string &msg) { g_last_error = msg; }

namespace {
thread_local bool g_no_alloc = false;
}
void set_no_alloc(bool on) { g_no_alloc = on; }
bool no_alloc() { return g_no_alloc; }

namespace {

fastmm_status fail(fastmm_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

fastmm_status hip_fail(hipError_t e, const char *what) {
    return fail(FASTMM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Device copy of the composite task tables for L levels of one algorithm.  They depend only
// on the algorithm and L (block sizes are launch arguments), so a plan caches one per L.
struct Tables {
    int L = 0;
    int nleaves = 0;
    int MB = 1, KB = 1, NB = 1;  // M0^L, K0^L, N0^L blocks per dimension
    LeafEntry *leaves = nullptr;
    SrcEntry *asrc = nullptr;
    SrcEntry *bsrc = nullptr;
    BlockDests *bdest = nullptr;
    float *ucoef = nullptr, *vcoef = nullptr;  // the rule's U (M0K0 x R) and V (K0N0 x R), row-major
    // per-level rules (fastmm_plan_set_levels): level l's U and V, same layout (else empty);
    // tree plans: level l's nodes' U and V one after another, node q at q M0K0 R (resp. K0N0 R)
    std::vector<float *> lucoef, lvcoef;
    DestEntry *dest = nullptr;
    // Leaf r's operands written out as block r of a stacked operand: one source each, (r, 0)
    // with coefficient 1 (the FP64 / FP32 paths with written-out leaf operands).
    LeafEntry *wleaves = nullptr;
    SrcEntry *wsrc = nullptr;
    float *unit = nullptr;  // the 1 x 1 x 1 rule's U = V = [1]
    int device = -1;
    ~Tables() {
        if (device >= 0) {
            int cur = 0;
            (void)hipGetDevice(&cur);
            (void)hipSetDevice(device);
            (void)hipFree(leaves);
            (void)hipFree(asrc);
            (void)hipFree(bsrc);
            (void)hipFree(bdest);
            (void)hipFree(dest);
            (void)hipFree(ucoef);
            (void)hipFree(vcoef);
            for (float *x : lucoef) (void)hipFree(x);
            for (float *x : lvcoef) (void)hipFree(x);
            (void)hipFree(wleaves);
            (void)hipFree(wsrc);
            (void)hipFree(unit);
            (void)hipSetDevice(cur);
        }
    }
};

struct HostTables {
    std::vector<LeafEntry> leaves;
    std::vector<SrcEntry> asrc, bsrc;
    std::vector<BlockDests> bdest;
    std::vector<DestEntry> dest;
    int MB = 1, KB = 1, NB = 1;
};

// Nonzeros of column r of a coefficient matrix: (row, numerator).
std::vector<std::vector<std::pair<int, int64_t>>> col_nonzeros(const std::vector<int64_t> &X, int rows, int R) {
    std::vector<std::vector<std::pair<int, int64_t>>> nz(R);
    for (int r = 0; r < R; ++r)
        for (int i = 0; i < rows; ++i)
            if (X[(size_t)i * R + r] != 0) nz[r].push_back({i, X[(size_t)i * R + r]});
    return nz;
}

const size_t kMaxTableEntries = size_t(1) << 24;

// Unroll L levels of the rule into the composite leaf list (eq. (ST_exact)): leaf
// r = (r_1..r_L) has A sources prod_l U[i_l, r_l] A_(i_1..i_L), B sources likewise, and
// contributes prod_l W[k_l, r_l] M_r to output block (k_1..k_L).  Level 1 is the most
// significant digit of every composite block coordinate.
// Composite tables of eq. (2) unrolled over L levels.  rule_at(l, node) gives the rule of
// level l (0-based) at breadth-first node index `node` of that level: every node of a level
// shares the level's <M0,K0,N0;R> (stationary: one rule; uniform non-stationary, section 3.3:
// one rule per level; non-uniform, section 3.4: one rule per node, node [l, r_1 .. r_{l-1}]
// at (r_1 .. r_{l-1} read in the levels' mixed radix)).
template <typename RuleAt>
bool build_tables(int L, RuleAt rule_at, HostTables &ht, std::string &err) {
    std::vector<int> M0(L), K0(L), N0(L), R(L);
    ht.MB = ht.KB = ht.NB = 1;
    for (int l = 0; l < L; ++l) {
        const Algo *x = rule_at(l, 0);
        M0[l] = x->M0, K0[l] = x->K0, N0[l] = x->N0, R[l] = x->R;
        ht.MB *= M0[l], ht.KB *= K0[l], ht.NB *= N0[l];
    }
    struct NZ {
        std::vector<std::vector<std::pair<int, int64_t>>> U, V, W;
        int den_U, den_V, den_W;
    };
    std::map<const Algo *, NZ> nzs;
    auto nz_of = [&](const Algo *x) -> const NZ & {
        auto it = nzs.find(x);
        if (it == nzs.end())
            it = nzs.emplace(x, NZ{col_nonzeros(x->U, x->M0 * x->K0, x->R), col_nonzeros(x->V, x->K0 * x->N0, x->R),
                                   col_nonzeros(x->W, x->M0 * x->N0, x->R), x->den_U, x->den_V, x->den_W})
                     .first;
        return it->second;
    };
    std::vector<std::vector<DestEntry>> per_block((size_t)ht.MB * ht.NB);
    int64_t nleaves_all = 1;
    for (int l = 0; l < L; ++l) {
        nleaves_all *= R[l];
        if (nleaves_all > (int64_t)1 << 22) {
            err = "too many leaves";
            return false;
        }
    }
    std::vector<int> r(L, 0);
    std::vector<const NZ *> lv(L, nullptr);  // the rule of each level on this leaf's path
    for (int64_t leaf_all = 0; leaf_all < nleaves_all; ++leaf_all) {
        {  // odometer: r[0] most significant
            int64_t x = leaf_all;
            for (int l = L - 1; l >= 0; --l) r[l] = (int)(x % R[l]), x /= R[l];
        }
        int64_t prefix = 0;
        for (int l = 0; l < L; ++l) {
            const Algo *x = rule_at(l, prefix);
            if (x->M0 != M0[l] || x->K0 != K0[l] || x->N0 != N0[l] || x->R != R[l]) {
                err = "rules of one level differ in shape";
                return false;
            }
            lv[l] = &nz_of(x);
            prefix = prefix * R[l] + r[l];
        }
        bool zero = false;
        for (int l = 0; l < L; ++l)
            if (lv[l]->U[r[l]].empty() || lv[l]->V[r[l]].empty() || lv[l]->W[r[l]].empty()) zero = true;
        if (zero) continue;  // this product never reaches C
        const int leaf = (int)ht.leaves.size();
        LeafEntry le{(int32_t)ht.asrc.size(), 0, (int32_t)ht.bsrc.size(), 0};
        // cartesian products over levels of the per-level nonzero lists
        // which: 0 = U (A sources), 1 = V (B sources), 2 = W (C destinations)
        auto expand = [&](int which, bool is_c, std::vector<SrcEntry> *out_src) {
            auto list = [&](int l) -> const std::vector<std::pair<int, int64_t>> & {
                return which == 0 ? lv[l]->U[r[l]] : which == 1 ? lv[l]->V[r[l]] : lv[l]->W[r[l]];
            };
            std::vector<int> idx(L, 0);
            while (true) {
                int64_t br = 0, bc = 0;
                double coef = 1.0;
                for (int l = 0; l < L; ++l) {
                    const auto &e = list(l)[idx[l]];
                    const int den = which == 0 ? lv[l]->den_U : which == 1 ? lv[l]->den_V : lv[l]->den_W;
                    // block grid of this level's operand: rowsz x colsz blocks
                    const int rowsz = which == 1 ? K0[l] : M0[l];
                    const int colsz = which == 0 ? K0[l] : N0[l];
                    int p, q;
                    if (is_c) {  // row-major single index over M0 x N0
                        p = e.first / colsz, q = e.first % colsz;
                    } else {  // column-major single index over rowsz x colsz
                        p = e.first % rowsz, q = e.first / rowsz;
                    }
                    br = br * rowsz + p;
                    bc = bc * colsz + q;
                    coef *= std::ldexp((double)e.second, -den);
                }
                if (is_c) {
                    per_block[(size_t)br * ht.NB + bc].push_back({(int32_t)leaf, (float)coef});
                } else {
                    out_src->push_back({(int32_t)br, (int32_t)bc, (float)coef, 0});
                }
                int l = L - 1;
                while (l >= 0 && ++idx[l] == (int)list(l).size()) idx[l] = 0, --l;
                if (l < 0) break;
            }
        };
        expand(0, false, &ht.asrc);
        expand(1, false, &ht.bsrc);
        expand(2, true, nullptr);
        le.a_count = (int32_t)(ht.asrc.size() - le.a_begin);
        le.b_count = (int32_t)(ht.bsrc.size() - le.b_begin);
        ht.leaves.push_back(le);
        if (ht.asrc.size() + ht.bsrc.size() > kMaxTableEntries) {
            err = "task table too large for this algorithm and depth";
            return false;
        }
    }
    ht.bdest.resize(per_block.size());
    for (size_t b = 0; b < per_block.size(); ++b) {
        ht.bdest[b] = {(int32_t)ht.dest.size(), (int32_t)per_block[b].size()};
        ht.dest.insert(ht.dest.end(), per_block[b].begin(), per_block[b].end());
    }
    return true;
}

template <typename X>
hipError_t upload(X **dst, const std::vector<X> &src) {
    *dst = nullptr;
    size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(X);
    hipError_t e = hipMalloc((void **)dst, bytes);
    if (e != hipSuccess) return e;
    if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(X), hipMemcpyHostToDevice);
    return e;
}

struct Shape {
    int L;
    int64_t Mp, Kp, Np, mb, kb, nb;
};

}  // namespace
}  // namespace fastmm

struct fastmm_plan_s {
    int algo = 0;
    int depth = 0;
    int cutoff = 1;
    fastmm_scaling sc{0, 0, 0.0, 0, 0};
    int prec = FASTMM_F64;
    int fuse = FASTMM_FUSE_AUTO;  // fastmm_fusion
    int tile = 0;  // split precisions: limb-GEMM output tile (0: by the leaf-block shape; 128; 256)
    // Non-uniform recursion: the rule id of every internal node, breadth first (empty: `algo`
    // at every node).
    std::vector<int> tree;
    // Uniform non-stationary recursion: the rule id of every level (empty: `algo` at every
    // level).  At most one of `tree` and `levels` is set.
    std::vector<int> levels;
    std::mutex mu;
    std::map<std::pair<int, int>, std::unique_ptr<fastmm::Tables>> tables;  // (L, device)
    // Sub-plans of the backward pass (made on first use): [0] forms dA = G B^T with the
    // transpose of the rotation [V,W,U], [1] forms dB = A^T G with the transpose of [W,U,V].
    std::unique_ptr<fastmm_plan_s> grad[2];
    // Scaling at every level: the plans of the first level's node products, by the depth of
    // the call that uses them (made on first use).
    std::map<int, std::unique_ptr<fastmm_plan_s>> node_plans;
};

namespace fastmm {
namespace {

const Algo &plan_algo(const fastmm_plan_s *p) { return *algo_get(p->algo); }

// The rule of level l (0-based) of a stationary or uniform non-stationary plan.
const Algo &level_algo(const fastmm_plan_s *p, int l) {
    return p->levels.empty() ? plan_algo(p) : *algo_get(p->levels[(size_t)l]);
}

bool build_plan_tables(const fastmm_plan_s *p, int L, HostTables &ht, std::string &err) {
    if (!p->tree.empty()) {
        const int R = plan_algo(p).R;
        std::vector<int64_t> off(L + 1, 0);  // breadth-first index of each level's first node
        for (int l = 1, cnt = 1; l <= L; ++l, cnt *= R) off[l] = off[l - 1] + cnt;
        if ((int64_t)p->tree.size() < off[L]) {
            err = "recursion tree has fewer nodes than the levels used";
            return false;
        }
        return build_tables(L, [&](int l, int64_t node) { return algo_get(p->tree[(size_t)(off[l] + node)]); }, ht,
                            err);
    }
    return build_tables(L, [&](int l, int64_t) { return &level_algo(p, l); }, ht, err);
}

constexpr int64_t kBlockAlign = 8;

Shape shape_of(const fastmm_plan_s *p, int64_t m, int64_t k, int64_t n) {
    Shape s{0, m, k, n, m, k, n};
    // Recurse while levels remain and every child dimension ceil(dim / prod of base sizes so
    // far) >= cutoff (each level with its own rule's base sizes).
    int64_t pm = 1, pk = 1, pn = 1;
    int L = 0;
    for (int l = 0; l < p->depth; ++l) {
        const Algo &a = level_algo(p, l);
        if (a.M0 * a.K0 * a.N0 <= 1) break;
        pm *= a.M0, pk *= a.K0, pn *= a.N0;
        if ((m + pm - 1) / pm < p->cutoff || (k + pk - 1) / pk < p->cutoff || (n + pn - 1) / pn < p->cutoff) {
            pm /= a.M0, pk /= a.K0, pn /= a.N0;
            break;
        }
        ++L;
    }
    s.L = L;
    // Leaf blocks are rounded up to a multiple of kBlockAlign elements when there is a level, so
    // every block starts 16-byte aligned (vector loads in every precision); the extra zero
    // padding is at most kBlockAlign - 1 rows / columns per block.
    auto block = [&](int64_t dim, int64_t prod) {
        const int64_t b = (dim + prod - 1) / prod;
        return L > 0 ? (b + kBlockAlign - 1) / kBlockAlign * kBlockAlign : b;
    };
    s.mb = block(m, pm), s.kb = block(k, pk), s.nb = block(n, pn);
    s.Mp = s.mb * pm, s.Kp = s.kb * pk, s.Np = s.nb * pn;
    return s;
}

int leaf_count(const Algo &a, int L) {
    // Leaves whose columns of U, V and W are all nonzero (the others are dropped).
    int live = 0;
    for (int r = 0; r < a.R; ++r) {
        bool u = false, v = false, w = false;
        for (int i = 0; i < a.M0 * a.K0; ++i) u |= a.U[(size_t)i * a.R + r] != 0;
        for (int j = 0; j < a.K0 * a.N0; ++j) v |= a.V[(size_t)j * a.R + r] != 0;
        for (int k2 = 0; k2 < a.M0 * a.N0; ++k2) w |= a.W[(size_t)k2 * a.R + r] != 0;
        live += (u && v && w);
    }
    int64_t c = 1;
    for (int l = 0; l < L; ++l) c *= live;
    return (int)c;
}

// Leaves of a plan at L levels: the live products of every level multiplied out (tree plans
// have every product live).
int plan_leaf_count(const fastmm_plan_s *p, int L) {
    if (!p->tree.empty()) return leaf_count(plan_algo(p), L);
    int64_t c = 1;
    for (int l = 0; l < L; ++l) c *= leaf_count(level_algo(p, l), 1);
    return (int)c;
}

size_t elem_size(int prec) { return prec == FASTMM_F64 ? 8 : 4; }

// Sign masks (U+, U-, V+, V-, W+, W-) of a <2,2,2;7> rule whose coefficients are all in
// {0, +1, -1}: bit s*7+r is set where row s, column r holds +1 (resp. -1).  False otherwise.
bool rule_masks_222(const Algo &a, uint32_t m[6]) {
    if (a.M0 != 2 || a.K0 != 2 || a.N0 != 2 || a.R != 7) return false;
    const std::vector<int64_t> *X[3] = {&a.U, &a.V, &a.W};
    const int den[3] = {a.den_U, a.den_V, a.den_W};
    for (int t = 0; t < 3; ++t) {
        m[2 * t] = m[2 * t + 1] = 0;
        for (int s = 0; s < 4; ++s)
            for (int r = 0; r < 7; ++r) {
                const int64_t v = (*X[t])[(size_t)s * 7 + r];
                if (v == 0) continue;
                if (den[t] != 0) return false;
                if (v == 1) m[2 * t] |= 1u << (s * 7 + r);
                else if (v == -1) m[2 * t + 1] |= 1u << (s * 7 + r);
                else return false;
            }
    }
    return true;
}

bool is_split(int prec) { return prec >= FASTMM_BF16 && prec <= FASTMM_BF16X6; }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Split-precision plane sizes: limbs per element, limb-GEMM tile rows, plane rows (A side,
// B side) and plane row length, all padded to the GEMM and formation tiles.
struct SplitDims {
    int nl, bm;
    int64_t mbp, nbp, kp;
};

int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

// The limb-GEMM tile of a plan on a shape: the plan's own setting, else by the leaf blocks.
int plan_tile(const fastmm_plan_s *p, const Shape &s) {
    return p->tile ? p->tile : limb_gemm_tile(p->prec, s.mb, s.nb);
}

// bm_force (a batch's common tile) overrides the plan's tile.
SplitDims split_dims(const fastmm_plan_s *p, const Shape &s, int bm_force = 0) {
    SplitDims d;
    d.nl = limb_count(p->prec);
    d.bm = bm_force ? bm_force : plan_tile(p, s);
    d.mbp = round_up(s.mb, d.bm), d.nbp = round_up(s.nb, d.bm), d.kp = round_up(s.kb, 64);
    return d;
}

// Split precisions form the leaf operands from the composite source lists (form_planes: every
// leaf reads its own sources, (nnz(U)/R)^L of them on average) or level by level (form_node:
// every level reads each node operand once and writes all R children).  The composite pass
// streams better; the level-by-level one wins once the average fan-in is large (measured on
// MI355X at n = 8192: <4,2,4> depth 2, fan-in ~12, 5.7 against 8.1 ms; Strassen depth 2,
// fan-in 2.9, 1.75 against 0.95 ms).  Level by level needs every product live (then the
// composite leaves are exactly the R^L children, in the same order).
bool level_formation(const fastmm_plan_s *p, const Shape &s) {
    const Algo &a = plan_algo(p);
    if (s.L < 2 || !p->tree.empty() || !p->levels.empty()) return false;  // one rule at every node only
    int64_t all = 1;
    for (int l = 0; l < s.L; ++l) all *= a.R;
    if (leaf_count(a, s.L) != all) return false;
    int64_t nu = 0, nv = 0;
    for (int64_t x : a.U) nu += x != 0;
    for (int64_t x : a.V) nv += x != 0;
    const double fan = 0.5 * (std::pow((double)nu / a.R, s.L) + std::pow((double)nv / a.R, s.L));
    return fan > 8.0;
}

// Geometry of the inner levels 1 .. L-1 of one operand side (FP32 children in the workspace):
// child block size, row stride, bytes per child, byte offset of the level; the last entry's
// offset is the total.
struct InnerLevel {
    int64_t cb_o, cb_k, y_ld, y_stride, count;
    size_t off;
    int64_t k_ld, k_stride;  // the same blocks k-major (element (o, kk) at kk k_ld + o)
};
std::vector<InnerLevel> inner_levels(const fastmm_plan_s *p, const Shape &s, bool side_b) {
    const size_t es = p->prec == FASTMM_F64 ? 8 : 4;
    const int64_t O = side_b ? s.Np : s.Mp, K = s.Kp;
    std::vector<InnerLevel> v;
    int64_t po = 1, pk = 1, count = 1;
    size_t off = 0;
    for (int l = 1; l < s.L; ++l) {
        const Algo &a = level_algo(p, l - 1);  // the rule that forms level l's nodes
        po *= side_b ? a.N0 : a.M0, pk *= a.K0, count *= a.R;
        InnerLevel e;
        e.cb_o = O / po, e.cb_k = K / pk, e.y_ld = (e.cb_k + 7) / 8 * 8, e.y_stride = e.cb_o * e.y_ld;
        e.k_ld = (e.cb_o + 7) / 8 * 8, e.k_stride = e.cb_k * e.k_ld;
        e.count = count, e.off = off;
        off = align256(off + es * (size_t)count * std::max(e.y_stride, e.k_stride));
        v.push_back(e);
    }
    v.push_back(InnerLevel{0, 0, 0, 0, 0, off, 0, 0});
    return v;
}

// Workspace layout: [ea m][ep k][eb n][flags 2] int32 | [maxA max(m,k)][maxB max(k,n)] elems |
// split precisions: [S limb planes][T^T limb planes] 16-bit | [leaf products nleaves * mb * nb]
// elems.
struct WsLayout {
    size_t ea, ep, eb, flags, maxA, maxB, sp, tp, ia, ib, xa, xb, leaves, nodes, total;
};

// Whether a product takes the fused one-level kernel: FP64/FP32, at least one level, row-major
// operands and a rule with a compiled sign pattern.  FASTMM_FUSE_AUTO takes it for FP32 from
// depth 3 only, where it saves the innermost level's formation and the list-form W-combination
// of three levels (Strassen n = 16384: 157 against 146 effective TFLOP/s); at depths 1 and 2 the
// written path below, whose leaf kernel runs at 0.78 of the FP32 peak against the fused
// kernel's 0.72, is as fast or faster (n = 8192 depth 1: 133 against 129; depth 2: 138 against
// 137, n = 16384: 151 against 144).  The FP64 fused kernel (one work-group per CU, source-list
// loads) runs at 0.45 of the FP64 peak; the written path beats it at every depth (n = 8192 depth
// 2: 63 against 43).
bool fused_path(const fastmm_plan_s *p, const Shape &s, int transA, int transB, uint32_t masks[6]) {
    if (p->fuse == FASTMM_FUSE_OFF || p->fuse == FASTMM_FUSE_WRITTEN || s.L < 1 || transA || transB) return false;
    if (!p->tree.empty() || !p->levels.empty()) return false;  // the fused kernel: one rule, every level
    if (p->prec != FASTMM_F64 && p->prec != FASTMM_F32) return false;
    if (p->fuse == FASTMM_FUSE_AUTO && (p->prec == FASTMM_F64 || s.L < 3)) return false;
    return rule_masks_222(plan_algo(p), masks) && node222_supported(masks);
}

// FP64 / FP32 written leaves: every leaf operand S_r (mb x kb) and T_r (kb x nb) is written out
// level by level, stacked (leaf r's S_r at rows r mb .. of an R^L mb x xa_ld matrix, T_r
// likewise at rows r kb of an R^L kb x xb_ld matrix, row strides multiples of 8), and the leaf
// kernel multiplies the stacked blocks in its single-source form.  With the composite lists
// instead, every work-group re-reads (nnz(U)/R)^L source tiles per K stage and sums them with
// their coefficients: 1.7-3.3 tiles at depth 1, ~11 for <4,2,4;26> at depth 2.  Measured on
// MI355X at n = 8192, FP32 depth 1: <4,2,4> 129.9 against 69.7 effective TFLOP/s, <3,2,3>
// 117.6 against 75.9, Laderman 109.5 against 61.6 (classical 121).  Needs every product live (the
// leaves are then the R^L children, in the composite order) and one rule at every node.
bool written_leaves(const fastmm_plan_s *p, const Shape &s) {
    if (is_split(p->prec) || s.L < 1) return false;
    if (p->fuse == FASTMM_FUSE_OFF) return false;  // the composite-list leaf path only
    for (int l = 0; l < s.L; ++l) {  // one rule per level (per-level rules included)
        const Algo &a = level_algo(p, l);
        if (leaf_count(a, 1) != a.R || a.M0 * a.K0 > 16 || a.K0 * a.N0 > 16) return false;
    }
    return true;
}

// The written path is taken where it applies and the fused kernel does not (the fused kernel,
// where it applies to row-major operands, comes first; transposed operands are copied).
bool written_taken(const fastmm_plan_s *p, const Shape &s) {
    uint32_t masks[6];
    return written_leaves(p, s) && !fused_path(p, s, 0, 0, masks);
}

// The fused path from depth 2: the node operands of the L-1 outer levels are written level by
// level first (the scaling factors and transposes applied at the first level), so that the fused
// kernel reads one source per node operand.  Summing the two or more sources of every node
// operand in the kernel's load stage doubled its loads per MFMA (Strassen depth 2 FP32 at
// n=8192: 0.47 of the FP32 peak, against 0.61 at depth 1).
bool fused_written(const fastmm_plan_s *p, const Shape &s) {
    uint32_t masks[6];
    return s.L >= 2 && fused_path(p, s, 0, 0, masks);
}

struct WrittenDims {
    int64_t xa_ld, xb_ld;
};
WrittenDims written_dims(const Shape &s) { return WrittenDims{round_up(s.kb, 8), round_up(s.nb, 8)}; }

int max_col_nnz(const std::vector<int64_t> &X, int rows, int R) {
    int mx = 0;
    for (int r = 0; r < R; ++r) {
        int c = 0;
        for (int i = 0; i < rows; ++i) c += X[(size_t)i * R + r] != 0;
        mx = std::max(mx, c);
    }
    return mx;
}

// Split precisions with the innermost recursion level formed in the limb GEMM's tile loads
// (fmm_limb_fused): the node operands of the outer levels are written out in FP32 level by level
// (at depth <= 1 the operands themselves, B read transposed, copied only when their layout needs
// it), the GEMM forms each leaf's S_r and T_r^T from them while staging; no limb planes.  For
// one rule at every node with every product live, at most 2 sources per column of U and V
// (the raw chunks of a stage sit in registers beside the accumulators; 4 spill), at most two
// limbs and 256 x 256 output tiles.
//
// Measured on MI355X, this path is slower than limb planes: Strassen depth 2 at n = 16384 F16X3
// took 26.7 ms in fmm_limb_fused against 17.2 ms in fmm_limb_gemm (plus 2.8 ms of plane formation;
// the FP32 node operands of depth 2 cost as much, 2.8 ms); classical 28.0 against 21.9.  The
// fused GEMM keeps every stage's raw FP32 chunks in registers beside the accumulators (256
// VGPRs, a few spills), so it runs the 32 x 32 x 16 MFMA form and leaves the per-stage sums and
// splits unoverlapped.  It is therefore taken only when asked for (FASTMM_FUSE_ALWAYS).
bool fused_split(const fastmm_plan_s *p, const Shape &s) {
    if (!is_split(p->prec) || limb_count(p->prec) > 2 || p->fuse != FASTMM_FUSE_ALWAYS) return false;
    if (!p->tree.empty() || !p->levels.empty()) return false;
    if (plan_tile(p, s) != 256) return false;
    if (s.L >= 1) {
        const Algo &a = plan_algo(p);
        int64_t all = 1;
        for (int l = 0; l < s.L; ++l) all *= a.R;
        if (leaf_count(a, s.L) != all) return false;
        if (max_col_nnz(a.U, a.M0 * a.K0, a.R) > 2 || max_col_nnz(a.V, a.K0 * a.N0, a.R) > 2) return false;
    }
    // 32-bit element offsets inside one node operand (rows x row length, both sides)
    const Algo &a = plan_algo(p);
    const int64_t pm = s.L >= 1 ? s.mb * a.M0 : s.Mp, pn = s.L >= 1 ? s.nb * a.N0 : s.Np;
    const int64_t pk = round_up(s.L >= 1 ? s.kb * a.K0 : s.Kp, 8);
    return pm * pk < ((int64_t)1 << 31) && pn * pk < ((int64_t)1 << 31);
}

// The scaling part of a workspace (exponents, flags, maxima); returns its end.
size_t scaling_layout(const fastmm_plan_s *p, int64_t m, int64_t k, int64_t n, WsLayout &w) {
    const size_t es = elem_size(p->prec);
    size_t off = 0;
    if (p->sc.mode != FASTMM_SCALE_NONE) {
        w.ea = off, off = align256(off + 4 * (size_t)m);
        w.ep = off, off = align256(off + 4 * (size_t)k);
        w.eb = off, off = align256(off + 4 * (size_t)n);
        w.flags = off, off = align256(off + 16);
        w.maxA = off, off = align256(off + es * (size_t)std::max(m, k));
        w.maxB = off, off = align256(off + es * (size_t)std::max(k, n));
    }
    return off;
}

bool two_pass_combine(const fastmm_plan_s *p, const Shape &s);

// batch: the layout of a problem inside a batched call, where FP32/FP64 products take written
// leaf operands wherever they apply (the batched launch has no fused kernel: the path of
// FASTMM_FUSE_WRITTEN).
WsLayout ws_layout(const fastmm_plan_s *p, const Shape &s, int64_t m, int64_t k, int64_t n, int bm_force = 0,
                   bool batch = false) {
    WsLayout w{};
    const bool written = batch ? written_leaves(p, s) : written_taken(p, s);
    const size_t es = elem_size(p->prec);
    size_t off = scaling_layout(p, m, k, n, w);
    if (is_split(p->prec) && bm_force == 0 && fused_split(p, s)) {
        // node operands: depth <= 1 the copies of op(A) and op(B)^T (used when their layout
        // needs one), deeper the FP32 children of the outer levels
        if (s.L <= 1) {
            const int64_t kt = round_up(s.Kp, 8);
            w.xa = off, off = align256(off + 4 * (size_t)s.Mp * kt);
            w.xb = off, off = align256(off + 4 * (size_t)s.Np * kt);
        } else {
            w.ia = off, off = align256(off + inner_levels(p, s, false).back().off);
            w.ib = off, off = align256(off + inner_levels(p, s, true).back().off);
        }
    } else if (is_split(p->prec)) {
        const SplitDims d = split_dims(p, s, bm_force);
        const size_t nleaves = (size_t)plan_leaf_count(p, s.L);
        w.sp = off, off = align256(off + 2 * nleaves * d.nl * (size_t)d.mbp * d.kp);
        w.tp = off, off = align256(off + 2 * nleaves * d.nl * (size_t)d.nbp * d.kp);
        if (level_formation(p, s)) {
            w.ia = off, off = align256(off + inner_levels(p, s, false).back().off);
            w.ib = off, off = align256(off + inner_levels(p, s, true).back().off);
        }
    } else if (!is_split(p->prec) && !batch && fused_written(p, s)) {
        // FP64 / FP32 fused from depth 2: the outer levels' node operands (the last of them
        // stacked as the fused kernel's operands)
        w.ia = off, off = align256(off + inner_levels(p, s, false).back().off);
        w.ib = off, off = align256(off + inner_levels(p, s, true).back().off);
    } else if (!is_split(p->prec) && !written) {
        // FP64 / FP32: row-major copies of op(A) and op(B), scaled, for scaled plans and for
        // transposed operands (prescale_operands)
        w.xa = off, off = align256(off + es * (size_t)s.Mp * round_up(s.Kp, 8));
        w.xb = off, off = align256(off + es * (size_t)s.Kp * round_up(s.Np, 8));
    } else if (written) {
        const WrittenDims wd = written_dims(s);
        const size_t nleaves = (size_t)plan_leaf_count(p, s.L);
        w.ia = off, off = align256(off + inner_levels(p, s, false).back().off);
        w.ib = off, off = align256(off + inner_levels(p, s, true).back().off);
        w.xa = off, off = align256(off + es * nleaves * (size_t)s.mb * wd.xa_ld);
        w.xb = off, off = align256(off + es * nleaves * (size_t)s.kb * wd.xb_ld);
    }
    w.leaves = off;
    if (s.L > 0) off = align256(off + es * (size_t)plan_leaf_count(p, s.L) * s.mb * s.nb);
    if (two_pass_combine(p, s)) {  // the first-level node products of the two-pass combination
        const Algo &a = plan_algo(p);
        w.nodes = off, off = align256(off + es * (size_t)a.R * (a.M0 * s.mb) * (a.N0 * s.nb));
    }
    w.total = off;
    return w;
}

std::string schedule_of(const fastmm_scaling &sc) {
    switch (sc.mode) {
        case FASTMM_SCALE_NONE: return "";
        case FASTMM_SCALE_OUTSIDE: return "O";
        case FASTMM_SCALE_INSIDE: return "I";
        case FASTMM_SCALE_OUT_IN: return "OI";
        case FASTMM_SCALE_IN_OUT: return "IO";
        case FASTMM_SCALE_REPEATED: {
            std::string s;
            for (int t = 0; t < sc.steps; ++t) s += (t % 2 == 0) ? 'O' : 'I';
            return s;
        }
    }
    return "";
}

// The W-combination reads each product once, in registers, for one or two levels of
// <2,K0,2> rules with at most 8 products each, every product live (leaf of (r1, r2):
// r1 R2 + r2), summing level by level; otherwise it follows the composite destination lists.
void set_kron(const fastmm_plan_s *p, int levels, int nleaves, CombineLaunch &Cb) {
    Cb.kron = 0;
    if (levels < 1 || levels > 2 || !p->tree.empty()) return;
    const Algo &a1 = level_algo(p, 0);
    if (levels == 1 && (a1.M0 != 2 || a1.N0 != 2 || a1.R > 8)) {
        // 16 output blocks (<4,2,4>): dense W from the lists, products streamed once.  With
        // 9 output blocks (<3,2,3>, <3,3,3>) the list form measured faster (0.18 against
        // 0.21 ms at n = 8192) and stays.
        if (a1.M0 * a1.N0 == 16 && a1.R <= 64 && nleaves == a1.R)
            Cb.kron = 3, Cb.R1 = a1.R, Cb.R2 = a1.M0 * a1.N0;
        return;
    }
    if (a1.M0 != 2 || a1.N0 != 2 || a1.R > 8) return;
    for (int k = 0; k < 4; ++k)
        for (int r = 0; r < a1.R; ++r) Cb.w1[k][r] = (float)a1.w(k, r);
    Cb.R1 = a1.R;
    if (levels == 1) {
        if (nleaves == a1.R) Cb.kron = 1;
        return;
    }
    const Algo &a2 = level_algo(p, 1);
    if (a2.M0 != 2 || a2.N0 != 2 || a2.R > 8 || nleaves != a1.R * a2.R) return;
    for (int k = 0; k < 4; ++k)
        for (int r = 0; r < a2.R; ++r) Cb.w2[k][r] = (float)a2.w(k, r);
    Cb.R2 = a2.R, Cb.kron = 2;
}

// Two levels of one rule with 16 output blocks per level (<4,2,4> and its rotations): combined
// level by level, each level from the one-level lists (CombineLaunch::kron = 4) through the R
// first-level node products.  The composite-list form re-reads each output block's ~100
// contributing products from cache (FETCH about 10x the products' bytes); measured at
// n = 8192 FP32: 1.02 -> 0.54 ms, F16X3 n = 16384: 5.2 -> 2.5 ms.  With 9 output blocks the
// lists stay (<3,2,3> depth 2: 0.44 against 0.76 ms two-pass; Laderman 1.26 against 1.14).
bool two_pass_combine(const fastmm_plan_s *p, const Shape &s) {
    if (s.L != 2 || !p->tree.empty() || !p->levels.empty()) return false;
    const Algo &a = plan_algo(p);
    return a.M0 * a.N0 == 16 && a.R <= 64 && leaf_count(a, 2) == (int64_t)a.R * a.R;
}

fastmm_status get_tables(fastmm_plan_s *p, int L, Tables **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> g(p->mu);
    auto key = std::make_pair(L, dev);
    auto it = p->tables.find(key);
    if (it != p->tables.end()) {
        *out = it->second.get();
        return FASTMM_OK;
    }
    if (no_alloc())
        return fail(FASTMM_EUNSUPPORTED, "the plan's task tables for " + std::to_string(L) +
                                             " levels are not on this device yet; one fastmm_gemm call with this "
                                             "plan and shape on the device uploads them");
    HostTables ht;
    std::string err;
    if (!build_plan_tables(p, L, ht, err)) return fail(FASTMM_EUNSUPPORTED, err);
    std::unique_ptr<Tables> t(new Tables());
    t->L = L;
    t->nleaves = (int)ht.leaves.size();
    t->MB = ht.MB, t->KB = ht.KB, t->NB = ht.NB;
    t->device = dev;
    if ((e = upload(&t->leaves, ht.leaves)) != hipSuccess || (e = upload(&t->asrc, ht.asrc)) != hipSuccess ||
        (e = upload(&t->bsrc, ht.bsrc)) != hipSuccess || (e = upload(&t->bdest, ht.bdest)) != hipSuccess ||
        (e = upload(&t->dest, ht.dest)) != hipSuccess)
        return hip_fail(e, "uploading task tables");
    {
        auto coefs = [](const Algo &a, std::vector<float> &u, std::vector<float> &v) {
            u.assign((size_t)a.M0 * a.K0 * a.R, 0.f), v.assign((size_t)a.K0 * a.N0 * a.R, 0.f);
            for (int i = 0; i < a.M0 * a.K0; ++i)
                for (int r = 0; r < a.R; ++r) u[(size_t)i * a.R + r] = (float)a.u(i, r);
            for (int j = 0; j < a.K0 * a.N0; ++j)
                for (int r = 0; r < a.R; ++r) v[(size_t)j * a.R + r] = (float)a.v(j, r);
        };
        std::vector<float> u, v;
        coefs(plan_algo(p), u, v);
        if ((e = upload(&t->ucoef, u)) != hipSuccess || (e = upload(&t->vcoef, v)) != hipSuccess)
            return hip_fail(e, "uploading coefficients");
        if (!p->levels.empty() || !p->tree.empty()) {
            t->lucoef.assign((size_t)L, nullptr), t->lvcoef.assign((size_t)L, nullptr);
            int64_t off = 0, nodes = 1;  // breadth-first index of the level's first tree node
            for (int l = 0; l < L; ++l, off += nodes, nodes *= plan_algo(p).R) {
                std::vector<float> ul, vl;
                for (int64_t q = 0; q < (p->tree.empty() ? 1 : nodes); ++q) {
                    coefs(p->tree.empty() ? level_algo(p, l) : *algo_get(p->tree[(size_t)(off + q)]), u, v);
                    ul.insert(ul.end(), u.begin(), u.end()), vl.insert(vl.end(), v.begin(), v.end());
                }
                if ((e = upload(&t->lucoef[(size_t)l], ul)) != hipSuccess ||
                    (e = upload(&t->lvcoef[(size_t)l], vl)) != hipSuccess)
                    return hip_fail(e, "uploading coefficients");
            }
        }
    }
    {
        std::vector<LeafEntry> wl((size_t)t->nleaves);
        std::vector<SrcEntry> ws((size_t)t->nleaves);
        for (int r = 0; r < t->nleaves; ++r) wl[(size_t)r] = LeafEntry{r, 1, r, 1}, ws[(size_t)r] = SrcEntry{r, 0, 1.f, 0};
        if ((e = upload(&t->wleaves, wl)) != hipSuccess || (e = upload(&t->wsrc, ws)) != hipSuccess ||
            (e = upload(&t->unit, std::vector<float>{1.f})) != hipSuccess)
            return hip_fail(e, "uploading tables");
    }
    *out = t.get();
    p->tables[key] = std::move(t);
    return FASTMM_OK;
}

// The W-combination of a product's leaves: the register forms of set_kron, else two levels of
// one rule level by level (two_pass_combine, through w.nodes), else the composite lists.
fastmm_status set_combine(fastmm_plan_s *p, const Shape &s, const Tables *tab, char *ws, const WsLayout &w,
                          CombineLaunch &Cb) {
    set_kron(p, s.L, tab->nleaves, Cb);
    if (Cb.kron != 0 || !two_pass_combine(p, s)) return FASTMM_OK;
    Tables *t1 = nullptr;
    const fastmm_status st = get_tables(p, 1, &t1);
    if (st != FASTMM_OK) return st;
    const Algo &a = plan_algo(p);
    Cb.kron = 4, Cb.R1 = a.R, Cb.M0 = a.M0, Cb.N0 = a.N0;
    Cb.bdest1 = t1->bdest, Cb.dest1 = t1->dest, Cb.nodes = ws + w.nodes;
    return FASTMM_OK;
}

bool ranges_overlap(const void *a, size_t abytes, const void *b, size_t bbytes) {
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + bbytes && pb < pa + abytes;
}

size_t span_bytes(int64_t rows, int64_t cols, int64_t ld, size_t es) {
    if (rows <= 0 || cols <= 0) return 0;
    return ((size_t)(rows - 1) * (size_t)ld + (size_t)cols) * es;
}

// Scaling steps on op(A), op(B); leaves the exponents in the workspace.
fastmm_status run_scaling(fastmm_plan_s *p, const void *A, int64_t lda, int transA, const void *B, int64_t ldb,
                          int transB, int64_t m, int64_t k, int64_t n, char *ws, const WsLayout &w, hipStream_t st,
                          ScaleExps *exps) {
    *exps = ScaleExps{nullptr, nullptr, nullptr};
    if (p->sc.mode == FASTMM_SCALE_NONE) return FASTMM_OK;
    int32_t *ea = (int32_t *)(ws + w.ea), *ep = (int32_t *)(ws + w.ep), *eb = (int32_t *)(ws + w.eb);
    int32_t *flags = (int32_t *)(ws + w.flags);
    hipError_t e;
    if ((e = launch_fill_i32(ea, m, 0, st)) != hipSuccess || (e = launch_fill_i32(ep, k, 0, st)) != hipSuccess ||
        (e = launch_fill_i32(eb, n, 0, st)) != hipSuccess || (e = launch_fill_i32(flags, 4, 0, st)) != hipSuccess)
        return hip_fail(e, "scaling init");
    const std::string sched = schedule_of(p->sc);
    bool seen_o = false;
    for (char kind : sched) {
        ScaleStep S;
        S.elem = p->prec == FASTMM_F64 ? Elem::F64 : Elem::F32;
        S.kind = kind;
        S.A = A, S.B = B, S.lda = lda, S.ldb = ldb, S.transA = transA, S.transB = transB;
        S.m = m, S.k = k, S.n = n;
        S.ea = ea, S.ep = ep, S.eb = eb;
        S.maxA = ws + w.maxA, S.maxB = ws + w.maxB;
        S.flags = flags;
        S.tau = p->sc.tau;
        S.o_nearest = p->sc.o_round == FASTMM_O_ROUND_NEAREST ? 1 : 0;
        // The stopping test (stopping-criterion theorem, section 6.3) applies to every step after
        // the first O step.
        S.test = (p->sc.tau > 0.0 && seen_o) ? 1 : 0;
        if (kind == 'O') seen_o = true;
        if ((e = launch_scale_step(S, st)) != hipSuccess) return hip_fail(e, "scaling step");
    }
    *exps = ScaleExps{ea, ep, eb};
    return FASTMM_OK;
}

fastmm_status check_plan(fastmm_plan_t p) {
    if (!p) return fail(FASTMM_EINVAL, "null plan");
    return FASTMM_OK;
}

}  // namespace
}  // namespace fastmm

using namespace fastmm;

extern "C" {

int fastmm_version(void) { return 1; }

const char *fastmm_strerror(fastmm_status s) {
    switch (s) {
        case FASTMM_OK: return "ok";
        case FASTMM_EINVAL: return "invalid argument";
        case FASTMM_EBRENT: return "coefficients fail the Brent equations";
        case FASTMM_ESHAPE: return "inconsistent shape or leading dimension";
        case FASTMM_ENOMEM: return "out of memory";
        case FASTMM_EHIP: return "HIP runtime error";
        case FASTMM_EUNSUPPORTED: return "unsupported combination";
        case FASTMM_EALIAS: return "output overlaps an input";
        case FASTMM_EWORKSPACE: return "workspace too small";
    }
    return "unknown status";
}

const char *fastmm_last_error(void) { return g_last_error.c_str(); }

fastmm_status fastmm_profile_enable(int enable) {
    g_prof.on = enable != 0;
    return FASTMM_OK;
}

fastmm_status fastmm_profile_read(double *ms_scaling, double *ms_form, double *ms_leaf, double *ms_combine,
                                  int *calls) {
    for (PhaseEvents &pe : g_prof.pending) {
        hipError_t e = hipEventSynchronize(pe.ev[kPhases]);
        if (e != hipSuccess) return hip_fail(e, "profile sync");
        for (int ph = 0; ph < kPhases; ++ph) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, pe.ev[ph], pe.ev[ph + 1]) == hipSuccess) g_prof.ms[ph] += t;
        }
        for (int i = 0; i <= kPhases; ++i) g_prof.pool.push_back(pe.ev[i]);
        ++g_prof.calls;
    }
    g_prof.pending.clear();
    if (ms_scaling) *ms_scaling = g_prof.ms[0];
    if (ms_form) *ms_form = g_prof.ms[1];
    if (ms_leaf) *ms_leaf = g_prof.ms[2];
    if (ms_combine) *ms_combine = g_prof.ms[3];
    if (calls) *calls = g_prof.calls;
    for (double &x : g_prof.ms) x = 0;
    g_prof.calls = 0;
    return FASTMM_OK;
}

fastmm_status fastmm_algo_register(int M0, int K0, int N0, int R, const int64_t *num_U, const int64_t *num_V,
                                   const int64_t *num_W, int log2_den, int *algo_out) {
    if (M0 < 1 || K0 < 1 || N0 < 1 || R < 1 || M0 > 16 || K0 > 16 || N0 > 16 || R > 4096 || !num_U || !num_V ||
        !num_W || !algo_out || log2_den < 0 || log2_den > 30)
        return fail(FASTMM_EINVAL, "fastmm_algo_register: bad arguments");
    Algo a;
    a.name = "user";
    a.M0 = M0, a.K0 = K0, a.N0 = N0, a.R = R;
    a.U.assign(num_U, num_U + (size_t)M0 * K0 * R);
    a.V.assign(num_V, num_V + (size_t)K0 * N0 * R);
    a.W.assign(num_W, num_W + (size_t)M0 * N0 * R);
    a.den_U = a.den_V = a.den_W = log2_den;
    for (int64_t x : a.U) if (x > (1 << 20) || x < -(1 << 20)) return fail(FASTMM_EINVAL, "coefficient too large");
    for (int64_t x : a.V) if (x > (1 << 20) || x < -(1 << 20)) return fail(FASTMM_EINVAL, "coefficient too large");
    for (int64_t x : a.W) if (x > (1 << 20) || x < -(1 << 20)) return fail(FASTMM_EINVAL, "coefficient too large");
    if (brent_violations(a) != 0) return fail(FASTMM_EBRENT, "registered algorithm fails the Brent equations");
    const int id = algo_register(std::move(a));
    if (id < 0) return fail(FASTMM_ENOMEM, "algorithm registry full");
    *algo_out = id;
    return FASTMM_OK;
}

fastmm_status fastmm_algo_info(int algo, int *M0, int *K0, int *N0, int *R, int *nnz, double *Q, double *E) {
    const Algo *a = algo_get(algo);
    if (!a) return fail(FASTMM_EINVAL, "unknown algorithm id");
    const Quantities q = quantities(*a);
    if (M0) *M0 = a->M0;
    if (K0) *K0 = a->K0;
    if (N0) *N0 = a->N0;
    if (R) *R = a->R;
    if (nnz) *nnz = q.nnz;
    if (Q) *Q = q.Q;
    if (E) *E = q.E;
    return FASTMM_OK;
}

fastmm_status fastmm_algo_stability(int algo, int levels, double *stab_exp, double *flops_frac,
                                    double *rel_instability) {
    const Algo *a = algo_get(algo);
    if (!a) return fail(FASTMM_EINVAL, "unknown algorithm id");
    if (levels < 0) return fail(FASTMM_EINVAL, "negative number of levels");
    const Quantities q = quantities(*a);
    const double base = (double)a->M0 * a->K0 * a->N0;
    if (stab_exp) {
        if (a->M0 == a->K0 && a->K0 == a->N0) {
            *stab_exp = std::log(q.E) / std::log((double)a->N0);
        } else {  // cyclic use of the rule and its two rotations: a square <P,P,P> rule per 3 levels
            double e = q.E;
            for (int t = 1; t <= 2; ++t) {
                const int rid = algo_rotated(algo, t);
                const Algo *r = rid >= 0 ? algo_get(rid) : nullptr;
                if (!r) return fail(FASTMM_EUNSUPPORTED, "rotation of the rule not available");
                e *= quantities(*r).E;
            }
            *stab_exp = std::log(e) / std::log(base);
        }
    }
    if (flops_frac) *flops_frac = std::pow((double)a->R / base, levels);
    if (rel_instability) *rel_instability = std::pow(q.E / ((double)a->K0 * a->K0), levels);
    return FASTMM_OK;
}

fastmm_status fastmm_algo_coeffs(int algo, double *U, double *V, double *W) {
    const Algo *a = algo_get(algo);
    if (!a) return fail(FASTMM_EINVAL, "unknown algorithm id");
    for (int i = 0; U && i < a->M0 * a->K0; ++i)
        for (int r = 0; r < a->R; ++r) U[(size_t)i * a->R + r] = a->u(i, r);
    for (int j = 0; V && j < a->K0 * a->N0; ++j)
        for (int r = 0; r < a->R; ++r) V[(size_t)j * a->R + r] = a->v(j, r);
    for (int k = 0; W && k < a->M0 * a->N0; ++k)
        for (int r = 0; r < a->R; ++r) W[(size_t)k * a->R + r] = a->w(k, r);
    return FASTMM_OK;
}

fastmm_status fastmm_plan_create(fastmm_plan_t *out, int algo, int depth, int cutoff, const fastmm_scaling *scaling,
                                 int precision) {
    if (!out) return fail(FASTMM_EINVAL, "null output pointer");
    *out = nullptr;
    if (!algo_get(algo)) return fail(FASTMM_EINVAL, "unknown algorithm id");
    if (depth < 0 || depth > 8) return fail(FASTMM_EINVAL, "depth must be in [0, 8]");
    if (cutoff < 1) return fail(FASTMM_EINVAL, "cutoff must be >= 1");
    if (precision < FASTMM_F64 || precision > FASTMM_BF16X6) return fail(FASTMM_EINVAL, "unknown precision");
    fastmm_scaling sc{FASTMM_SCALE_NONE, 0, 0.0, 0, FASTMM_O_ROUND_UP};
    if (scaling) {
        sc = *scaling;
        if (sc.mode < FASTMM_SCALE_NONE || sc.mode > FASTMM_SCALE_REPEATED)
            return fail(FASTMM_EINVAL, "unknown scaling mode");
        if (sc.mode == FASTMM_SCALE_REPEATED && (sc.steps < 1 || sc.steps > 256))
            return fail(FASTMM_EINVAL, "repeated scaling needs 1 <= steps <= 256");
        if (!(sc.tau >= 0.0) || std::isinf(sc.tau)) return fail(FASTMM_EINVAL, "tau must be finite and >= 0");
        if (sc.per_level != 0 && sc.per_level != 1) return fail(FASTMM_EINVAL, "per_level must be 0 or 1");
        if (sc.o_round != FASTMM_O_ROUND_UP && sc.o_round != FASTMM_O_ROUND_NEAREST)
            return fail(FASTMM_EINVAL, "unknown O-step rounding");
    }
    fastmm_plan_s *p = new (std::nothrow) fastmm_plan_s();
    if (!p) return fail(FASTMM_ENOMEM, "plan allocation");
    p->algo = algo;
    p->depth = depth;
    p->cutoff = cutoff;
    p->sc = sc;
    p->prec = precision;
    *out = p;
    return FASTMM_OK;
}

fastmm_status fastmm_plan_destroy(fastmm_plan_t plan) {
    delete plan;
    return FASTMM_OK;
}

fastmm_status fastmm_plan_shape(fastmm_plan_t plan, int64_t m, int64_t k, int64_t n, int *levels, int64_t *Mp,
                                int64_t *Kp, int64_t *Np) {
    if (check_plan(plan)) return FASTMM_EINVAL;
    if (m < 0 || k < 0 || n < 0) return fail(FASTMM_EINVAL, "negative size");
    const Shape s = shape_of(plan, m, k, n);
    if (levels) *levels = s.L;
    if (Mp) *Mp = s.Mp;
    if (Kp) *Kp = s.Kp;
    if (Np) *Np = s.Np;
    return FASTMM_OK;
}

fastmm_status fastmm_plan_set_fusion(fastmm_plan_t plan, int mode) {
    if (check_plan(plan)) return FASTMM_EINVAL;
    if (mode < FASTMM_FUSE_OFF || mode > FASTMM_FUSE_WRITTEN) return fail(FASTMM_EINVAL, "unknown fusion mode");
    std::lock_guard<std::mutex> g(plan->mu);
    plan->fuse = mode;
    for (auto &r : plan->grad)
        if (r) r->fuse = plan->fuse;
    plan->node_plans.clear();  // remade with the new mode on next use
    return FASTMM_OK;
}

fastmm_status fastmm_plan_set_tile(fastmm_plan_t plan, int tile) {
    if (check_plan(plan)) return FASTMM_EINVAL;
    if (tile != 0 && tile != 128 && tile != 256) return fail(FASTMM_EINVAL, "tile must be 0, 128 or 256");
    if (tile != 0 && !is_split(plan->prec)) return fail(FASTMM_EUNSUPPORTED, "the tile applies to split precisions");
    if (tile == 256 && limb_count(plan->prec) > 2) return fail(FASTMM_EUNSUPPORTED, "256 tiles take at most two limbs");
    std::lock_guard<std::mutex> g(plan->mu);
    plan->tile = tile;
    for (auto &r : plan->grad)
        if (r) r->tile = tile;
    plan->node_plans.clear();
    return FASTMM_OK;
}

fastmm_status fastmm_plan_set_tree(fastmm_plan_t plan, const int *node_algos, int64_t count) {
    if (check_plan(plan)) return FASTMM_EINVAL;
    const Algo &a = plan_algo(plan);
    std::vector<int> tree;
    if (count > 0) {
        if (plan->sc.per_level && plan->sc.mode != FASTMM_SCALE_NONE)
            return fail(FASTMM_EUNSUPPORTED, "scaling at every level needs one rule per level, not a tree");
        if (!node_algos) return fail(FASTMM_EINVAL, "null node rule list");
        int64_t need = 0, lev = 1;
        for (int l = 0; l < plan->depth; ++l, lev *= a.R) {
            need += lev;
            if (need > 4096) return fail(FASTMM_EINVAL, "recursion tree too large");
        }
        if (count != need)
            return fail(FASTMM_ESHAPE, "the tree needs one rule per internal node: " + std::to_string(need));
        for (int64_t i = 0; i < count; ++i) {
            const Algo *x = algo_get(node_algos[i]);
            if (!x) return fail(FASTMM_EINVAL, "unknown rule id in the tree");
            if (x->M0 != a.M0 || x->K0 != a.K0 || x->N0 != a.N0 || x->R != a.R)
                return fail(FASTMM_ESHAPE, "every node rule must have the plan rule's <M0,K0,N0;R>");
            if (leaf_count(*x, 1) != x->R) return fail(FASTMM_EUNSUPPORTED, "node rules must have every product live");
        }
        tree.assign(node_algos, node_algos + count);
    }
    std::lock_guard<std::mutex> g(plan->mu);
    plan->tree = std::move(tree);
    plan->levels.clear();
    plan->tables.clear();  // rebuilt for the new tree on next use
    for (auto &r : plan->grad) r.reset();
    plan->node_plans.clear();
    return FASTMM_OK;
}

fastmm_status fastmm_plan_set_levels(fastmm_plan_t plan, const int *level_algos, int count) {
    if (check_plan(plan)) return FASTMM_EINVAL;
    std::vector<int> lv;
    if (count > 0) {
        if (!level_algos) return fail(FASTMM_EINVAL, "null level rule list");
        if (count != plan->depth) return fail(FASTMM_ESHAPE, "one rule per level of the plan's depth");
        for (int i = 0; i < count; ++i) {
            const Algo *x = algo_get(level_algos[i]);
            if (!x) return fail(FASTMM_EINVAL, "unknown rule id for a level");
            if (x->M0 * x->K0 * x->N0 <= 1) return fail(FASTMM_EINVAL, "a level rule must split the product");
        }
        lv.assign(level_algos, level_algos + count);
    } else if (count < 0) {
        return fail(FASTMM_EINVAL, "negative count");
    }
    std::lock_guard<std::mutex> g(plan->mu);
    plan->levels = std::move(lv);
    plan->tree.clear();
    plan->tables.clear();
    for (auto &r : plan->grad) r.reset();
    plan->node_plans.clear();
    return FASTMM_OK;
}

namespace fastmm {
namespace {
bool every_level(const fastmm_plan_s *p, const Shape &s);
fastmm_status every_level_total(fastmm_plan_s *p, const Shape &s, int64_t m, int64_t k, int64_t n, size_t *bytes);
}  // namespace
}  // namespace fastmm

fastmm_status fastmm_plan_path(fastmm_plan_t plan, int64_t m, int64_t k, int64_t n, int transA, int transB,
                               int *path) {
    if (check_plan(plan)) return FASTMM_EINVAL;
    if (!path || m < 0 || k < 0 || n < 0) return fail(FASTMM_EINVAL, "bad arguments");
    const Shape s = shape_of(plan, m, k, n);
    uint32_t masks[6];
    // FP64 / FP32 transposed operands are copied to row-major first (gemm_ex), so the fused
    // kernel's choice does not depend on the transposition flags
    (void)transA, (void)transB;
    *path = every_level(plan, s)                         ? FASTMM_PATH_EVERY_LEVEL
            : fused_path(plan, s, 0, 0, masks)           ? FASTMM_PATH_FUSED
            : written_taken(plan, s)                     ? FASTMM_PATH_WRITTEN
            : fused_split(plan, s)                       ? FASTMM_PATH_FUSED_LOADS
                                                         : FASTMM_PATH_LEAF;
    return FASTMM_OK;
}

fastmm_status fastmm_workspace_size(fastmm_plan_t plan, int64_t m, int64_t k, int64_t n, size_t *bytes) {
    if (check_plan(plan)) return FASTMM_EINVAL;
    if (!bytes || m < 0 || k < 0 || n < 0) return fail(FASTMM_EINVAL, "bad arguments");
    const Shape s = shape_of(plan, m, k, n);
    if (every_level(plan, s)) return every_level_total(plan, s, m, k, n, bytes);
    *bytes = ws_layout(plan, s, m, k, n).total;
    return FASTMM_OK;
}

namespace fastmm {
namespace {
// Split precisions, pass 1: the limb planes of every leaf's S_r and T_r^T (scaling applied),
// composite or level by level; fills the plane part of the limb-GEMM launch g.
// Profiler marks of one call: event 0 when it starts, one event as each phase (scaling,
// operand formation, products, W-combination) ends; phases not reached are recorded empty
// when the call returns, on every exit path.
struct PhaseMarks {
    bool prof;
    PhaseEvents pe{};
    hipStream_t st;
    int next = 1;
    explicit PhaseMarks(hipStream_t s, bool record = true) : prof(g_prof.on && record && !no_alloc()), st(s) {
        if (!prof) return;
        for (int i = 0; i <= kPhases; ++i) pe.ev[i] = g_prof.get();
        (void)hipEventRecord(pe.ev[0], st);
    }
    void mark() {
        if (prof && next <= kPhases) (void)hipEventRecord(pe.ev[next++], st);
    }
    ~PhaseMarks() {
        if (!prof) return;
        while (next <= kPhases) (void)hipEventRecord(pe.ev[next++], st);
        g_prof.pending.push_back(pe);
    }
};

hipError_t split_form(fastmm_plan_s *plan, const Shape &s, const SplitDims &d, const void *A, int64_t lda,
                      int transA, const void *B, int64_t ldb, int transB, int64_t m, int64_t k, int64_t n,
                      const ScaleExps &exps, char *ws, const WsLayout &w, const Tables *tab, hipStream_t st,
                      LimbGemm &g) {
    hipError_t e;
    // After an O step the operands have row / column maxima in (1/2, 1]; fp16 limbs are then
    // moved up by 2^8 (exact), away from fp16's subnormal range, and the products down by
    // 2^-16.  Inside steps alone only balance A against B (their entries keep any size), so
    // a schedule without an O step takes no offset: with it, entries above 65504 / 2^8 would
    // overflow the fp16 limbs.
    const bool f16 = plan->prec == FASTMM_F16 || plan->prec == FASTMM_F16X3;
    const int pre = (f16 && exps.ea && schedule_of(plan->sc).find('O') != std::string::npos) ? 8 : 0;
    PlaneForm fa{};
    fa.X = (const float *)A;
    fa.ld_o = transA ? 1 : lda, fa.ld_k = transA ? lda : 1;  // op(A)(i, kk)
    fa.R = m, fa.K = k, fa.rb = s.mb, fa.kb = s.kb, fa.rowsp = d.mbp, fa.kp = d.kp, fa.bt = d.bm;
    fa.leaves = tab->leaves, fa.src = tab->asrc, fa.b_side = 0;
    fa.e_o = exps.ea, fa.e_k = exps.ep, fa.s_o = -1, fa.s_k = 1, fa.pre_exp = pre;  // 2^(ep_kk - ea_i)
    fa.planes = (unsigned short *)(ws + w.sp), fa.plane_stride = d.mbp * d.kp;
    fa.leaf_stride = d.nl * d.mbp * d.kp;
    fa.nbo = s.mb > 0 ? (int)(s.Mp / s.mb) : 0, fa.nbk = s.kb > 0 ? (int)(s.Kp / s.kb) : 0;
    PlaneForm fb{};
    fb.X = (const float *)B;
    fb.ld_o = transB ? ldb : 1, fb.ld_k = transB ? 1 : ldb;  // op(B)(kk, j) as T^T(j, kk)
    fb.R = n, fb.K = k, fb.rb = s.nb, fb.kb = s.kb, fb.rowsp = d.nbp, fb.kp = d.kp, fb.bt = d.bm;
    fb.leaves = tab->leaves, fb.src = tab->bsrc, fb.b_side = 1;
    fb.e_o = exps.eb, fb.e_k = exps.ep, fb.s_o = -1, fb.s_k = -1, fb.pre_exp = pre;  // 2^(-ep_kk - eb_j)
    fb.planes = (unsigned short *)(ws + w.tp), fb.plane_stride = d.nbp * d.kp;
    fb.leaf_stride = d.nl * d.nbp * d.kp;
    fb.nbo = s.nb > 0 ? (int)(s.Np / s.nb) : 0, fb.nbk = s.kb > 0 ? (int)(s.Kp / s.kb) : 0;
    if (level_formation(plan, s)) {
        // level by level: every level reads its node operands once and writes all R children
        const Algo &al = plan_algo(plan);
        auto form_side = [&](bool side_b) -> hipError_t {
            const PlaneForm &pf = side_b ? fb : fa;
            const std::vector<InnerLevel> lv = inner_levels(plan, s, side_b);
            char *ibase = ws + (side_b ? w.ib : w.ia);
            int64_t nodes = 1;
            for (int l = 1; l <= s.L; ++l) {
                NodeForm nf{};
                if (l == 1) {
                    nf.X = pf.X, nf.ld_o = pf.ld_o, nf.ld_k = pf.ld_k, nf.R = pf.R, nf.K = pf.K, nf.first = 1;
                    nf.e_o = pf.e_o, nf.e_k = pf.e_k, nf.s_o = pf.s_o, nf.s_k = pf.s_k, nf.pre_exp = pf.pre_exp;
                } else {
                    const InnerLevel &in = lv[l - 2];
                    nf.X = (const float *)(ibase + in.off), nf.ld_o = in.y_ld, nf.ld_k = 1;
                    nf.node_stride = in.y_stride, nf.first = 0;
                }
                nf.nO = side_b ? al.N0 : al.M0, nf.nK = al.K0, nf.side_b = side_b ? 1 : 0, nf.R_ = al.R;
                nf.coef = side_b ? tab->vcoef : tab->ucoef;
                if (l == s.L) {
                    nf.cb_o = pf.rb, nf.cb_k = pf.kb, nf.last = 1;
                    nf.planes = pf.planes, nf.rowsp = pf.rowsp, nf.kp = pf.kp, nf.bt = pf.bt;
                    nf.plane_stride = pf.plane_stride, nf.leaf_stride = pf.leaf_stride;
                } else {
                    const InnerLevel &out = lv[l - 1];
                    nf.cb_o = out.cb_o, nf.cb_k = out.cb_k, nf.last = 0;
                    nf.Y = (float *)(ibase + out.off), nf.y_ld = out.y_ld, nf.y_stride = out.y_stride;
                }
                if (nodes > 65535) return hipErrorInvalidValue;
                hipError_t er = launch_form_node(plan->prec, nf, (int)nodes, st);
                if (er != hipSuccess) return er;
                nodes *= al.R;
            }
            return hipSuccess;
        };
        if ((e = form_side(false)) != hipSuccess || (e = form_side(true)) != hipSuccess)
            return e;
    } else if ((e = launch_form_planes(plan->prec, fa, tab->nleaves, st)) != hipSuccess ||
               (e = launch_form_planes(plan->prec, fb, tab->nleaves, st)) != hipSuccess) {
        return e;
    }
    g = LimbGemm{};
    g.S = fa.planes, g.T = fb.planes, g.kp = d.kp;
    g.s_plane = fa.plane_stride, g.s_leaf = fa.leaf_stride, g.t_plane = fb.plane_stride, g.t_leaf = fb.leaf_stride;
    g.mb = s.mb, g.nb = s.nb, g.m = m, g.n = n, g.sc = exps, g.post_exp = -2 * pre;
    g.tiles_m = (int)(d.mbp / d.bm), g.tiles_n = (int)(d.nbp / d.bm);
    return hipSuccess;
}

// Split precisions with the innermost level formed in the limb GEMM's loads (fused_split): the
// node operands of both sides (FP32, k contiguous; B's stored transposed), then fmm_limb_fused
// over all leaves x tiles.  Fills f except the output fields.
hipError_t fused_split_operands(fastmm_plan_s *plan, const Shape &s, const void *A, int64_t lda, int transA,
                                const void *B, int64_t ldb, int transB, int64_t m, int64_t k, int64_t n,
                                const ScaleExps &exps, int pre, char *ws, const WsLayout &w, const Tables *tab,
                                hipStream_t st, LimbFused &f) {
    const Algo &al = plan_algo(plan);
    const bool i_step = schedule_of(plan->sc).find('I') != std::string::npos;
    f = LimbFused{};
    if (s.L <= 1) {
        // The operands themselves are the node operand: op(A) (m x k) and op(B)^T (n x k), read in
        // place when k-contiguous, 16-byte aligned, k a multiple of 8 and without inside factors
        // (the row factors of an O step are applied while loading); else copied once by a 1 x 1
        // level of form_node, which applies every factor.
        const int64_t kt = round_up(s.Kp, 8);
        auto side = [&](bool side_b) -> hipError_t {
            const void *X = side_b ? B : A;
            const int64_t ld = side_b ? ldb : lda;
            const bool krow = side_b ? transB != 0 : transA == 0;  // stored rows of op(X) with k contiguous
            const int64_t rows = side_b ? n : m;
            FusedSide &fs = side_b ? f.b : f.a;
            // (32-bit element offsets: the stored operand must span less than 2^31 elements)
            if (krow && !i_step && k % 8 == 0 && ld % 4 == 0 && ((uintptr_t)X & 15) == 0 &&
                rows * ld < ((int64_t)1 << 31)) {
                fs.X = (const float *)X, fs.ld = ld, fs.rows = rows, fs.cols = k;
                fs.e_row = side_b ? exps.eb : exps.ea, fs.s_row = -1, fs.pre_exp = pre;
                return hipSuccess;
            }
            NodeForm nf{};
            nf.X = X;
            if (side_b) nf.ld_o = transB ? ldb : 1, nf.ld_k = transB ? 1 : ldb;
            else nf.ld_o = transA ? 1 : lda, nf.ld_k = transA ? lda : 1;
            nf.R = rows, nf.K = k, nf.first = 1;
            nf.e_o = side_b ? exps.eb : exps.ea, nf.e_k = exps.ep, nf.s_o = -1, nf.s_k = side_b ? -1 : 1;
            nf.pre_exp = exps.ea ? pre : 0;
            nf.nO = 1, nf.nK = 1, nf.side_b = side_b ? 1 : 0, nf.R_ = 1, nf.coef = tab->unit;
            nf.cb_o = rows, nf.cb_k = kt, nf.last = 0;
            nf.Y = ws + (side_b ? w.xb : w.xa), nf.y_ld = kt, nf.y_stride = rows * kt;
            fs.X = (const float *)nf.Y, fs.ld = kt, fs.rows = rows, fs.cols = kt, fs.e_row = nullptr;
            return launch_form_node(FASTMM_F32, nf, 1, st);
        };
        hipError_t e = side(false);
        if (e == hipSuccess) e = side(true);
        if (e != hipSuccess) return e;
        f.a.node_stride = f.b.node_stride = 0;
    } else {
        // levels 1 .. L-1 written out (the first one scaled); the innermost level in the GEMM
        auto side = [&](bool side_b) -> hipError_t {
            const std::vector<InnerLevel> lv = inner_levels(plan, s, side_b);
            char *ibase = ws + (side_b ? w.ib : w.ia);
            int64_t nodes = 1;
            for (int l = 1; l < s.L; ++l) {
                NodeForm nf{};
                if (l == 1) {
                    nf.X = side_b ? B : A;
                    if (side_b) nf.ld_o = transB ? ldb : 1, nf.ld_k = transB ? 1 : ldb, nf.R = n;
                    else nf.ld_o = transA ? 1 : lda, nf.ld_k = transA ? lda : 1, nf.R = m;
                    nf.K = k, nf.first = 1;
                    nf.e_o = side_b ? exps.eb : exps.ea, nf.e_k = exps.ep, nf.s_o = -1, nf.s_k = side_b ? -1 : 1;
                    nf.pre_exp = exps.ea ? pre : 0;
                } else {
                    const InnerLevel &in = lv[(size_t)l - 2];
                    nf.X = ibase + in.off, nf.ld_o = in.y_ld, nf.ld_k = 1;
                    nf.node_stride = in.y_stride, nf.first = 0;
                }
                nf.nO = side_b ? al.N0 : al.M0, nf.nK = al.K0, nf.side_b = side_b ? 1 : 0, nf.R_ = al.R;
                nf.coef = side_b ? tab->vcoef : tab->ucoef;
                const InnerLevel &out = lv[(size_t)l - 1];
                nf.cb_o = out.cb_o, nf.cb_k = out.cb_k, nf.last = 0;
                nf.Y = ibase + out.off, nf.y_ld = out.y_ld, nf.y_stride = out.y_stride;
                if (nodes > 65535) return hipErrorInvalidValue;
                hipError_t er = launch_form_node(plan->prec, nf, (int)nodes, st);
                if (er != hipSuccess) return er;
                nodes *= al.R;
            }
            const InnerLevel &last = lv[(size_t)s.L - 2];
            FusedSide &fs = side_b ? f.b : f.a;
            fs.X = (const float *)(ibase + last.off), fs.ld = last.y_ld, fs.node_stride = last.y_stride;
            fs.rows = last.cb_o, fs.cols = last.cb_k, fs.e_row = nullptr;
            return hipSuccess;
        };
        hipError_t e = side(false);
        if (e == hipSuccess) e = side(true);
        if (e != hipSuccess) return e;
    }
    f.a.sb_rows = s.mb, f.b.sb_rows = s.nb;
    if (s.L >= 1) {
        f.ucoef = tab->ucoef, f.vcoef = tab->vcoef, f.M0 = al.M0, f.K0 = al.K0, f.N0 = al.N0, f.R = al.R;
        f.qa = max_col_nnz(al.U, al.M0 * al.K0, al.R), f.qb = max_col_nnz(al.V, al.K0 * al.N0, al.R);
    } else {
        f.ucoef = f.vcoef = tab->unit, f.M0 = f.K0 = f.N0 = f.R = 1, f.qa = f.qb = 1;
    }
    // leaf inner dimension in whole 8-element chunks (a multiple of 8 from depth 1; at depth 0
    // the copies are zero-padded to it and a direct operand has k % 8 == 0)
    f.kb = round_up(s.kb, 8), f.nk = (f.kb + 31) / 32;
    f.mb = s.mb, f.nb = s.nb, f.m = m, f.n = n, f.sc = exps, f.post_exp = -2 * pre;
    f.tiles_m = (int)((s.mb + 255) / 256), f.tiles_n = (int)((s.nb + 255) / 256);
    return hipSuccess;
}

// FP64 / FP32: row-major copies A2 = op(A) (m x lda2) and B2 = op(B) (k x ldb2) in the workspace,
// with the scaling factors applied when `scale` (A' = diag(2^-ea) op(A) diag(2^ep),
// B' = diag(2^-ep) op(B) diag(2^-eb)), by a 1 x 1 level of form_node.  The product kernels then
// read plain row-major operands: a scaled product applies each factor once here instead of once
// per source in every K stage of every tile that reads the element, and transposed operands
// take the fast row-major kernels.
hipError_t prescale_operands(fastmm_plan_s *plan, const Shape &s, const void *A, int64_t lda, int transA,
                             const void *B, int64_t ldb, int transB, int64_t m, int64_t k, int64_t n,
                             const ScaleExps &exps, bool scale, char *ws, const WsLayout &w, const Tables *tab,
                             hipStream_t st, const void **A2, int64_t *lda2, const void **B2, int64_t *ldb2) {
    (void)s;
    // Without scaling only a transposed operand is copied; the other is used in place.
    const bool copy_a = scale || transA, copy_b = scale || transB;
    const int prec = plan->prec == FASTMM_F64 ? FASTMM_F64 : FASTMM_F32;
    const int64_t ka = round_up(k, 8), nbl = round_up(n, 8);
    NodeForm fa{};
    fa.X = A, fa.ld_o = transA ? 1 : lda, fa.ld_k = transA ? lda : 1, fa.R = m, fa.K = k, fa.first = 1;
    if (scale) fa.e_o = exps.ea, fa.e_k = exps.ep, fa.s_o = -1, fa.s_k = 1;
    fa.nO = 1, fa.nK = 1, fa.side_b = 0, fa.R_ = 1, fa.coef = tab->unit;
    fa.cb_o = m, fa.cb_k = k, fa.last = 0, fa.Y = ws + w.xa, fa.y_ld = ka, fa.y_stride = m * ka;
    NodeForm fb{};
    fb.X = B, fb.ld_o = transB ? ldb : 1, fb.ld_k = transB ? 1 : ldb, fb.R = n, fb.K = k, fb.first = 1;
    if (scale) fb.e_o = exps.eb, fb.e_k = exps.ep, fb.s_o = -1, fb.s_k = -1;
    fb.nO = 1, fb.nK = 1, fb.side_b = 1, fb.R_ = 1, fb.coef = tab->unit;
    fb.cb_o = n, fb.cb_k = k, fb.last = 0, fb.Y = ws + w.xb, fb.y_ld = nbl, fb.y_stride = k * nbl, fb.kmajor = 1;
    hipError_t e = copy_a ? launch_form_node(prec, fa, 1, st) : hipSuccess;
    if (e == hipSuccess && copy_b) e = launch_form_node(prec, fb, 1, st);
    if (copy_a) *A2 = ws + w.xa, *lda2 = ka;
    else *A2 = A, *lda2 = lda;
    if (copy_b) *B2 = ws + w.xb, *ldb2 = nbl;
    else *B2 = B, *ldb2 = ldb;
    return e;
}

// FP64 / FP32 with written-out leaf operands: the leaf operands of both sides level by level
// (the first level scaled), S_r stacked at ws + xa (o-major), T_r at ws + xb (k-major, B's own
// orientation), so that the leaf kernel reads each as one row-major source block.
// With upto = s.L - 1 (the fused path from depth 2) the levels stop at the node operands of the
// innermost level's nodes, written where inner_levels puts level L-1, the A side o-major (node q
// at rows q cb_o) and the B side k-major (node q at rows q cb_k, row stride cb_o): stacked
// row-major operands with one source per node.
hipError_t form_written(fastmm_plan_s *plan, const Shape &s, const void *A, int64_t lda, int transA, const void *B,
                        int64_t ldb, int transB, int64_t m, int64_t k, int64_t n, const ScaleExps &exps, char *ws,
                        const WsLayout &w, const Tables *tab, hipStream_t st, int upto) {
    const WrittenDims wd = written_dims(s);
    auto form_side = [&](bool side_b) -> hipError_t {
        const std::vector<InnerLevel> lv = inner_levels(plan, s, side_b);
        char *ibase = ws + (side_b ? w.ib : w.ia);
        int64_t nodes = 1;
        for (int l = 1; l <= upto; ++l) {
            NodeForm nf{};
            if (l == 1) {
                if (side_b) {
                    nf.X = B, nf.ld_o = transB ? ldb : 1, nf.ld_k = transB ? 1 : ldb, nf.R = n;
                    nf.e_o = exps.eb, nf.s_o = -1, nf.s_k = -1;  // 2^(-ep_kk - eb_j)
                } else {
                    nf.X = A, nf.ld_o = transA ? 1 : lda, nf.ld_k = transA ? lda : 1, nf.R = m;
                    nf.e_o = exps.ea, nf.s_o = -1, nf.s_k = 1;  // 2^(ep_kk - ea_i)
                }
                nf.K = k, nf.first = 1, nf.e_k = exps.ep, nf.pre_exp = 0;
            } else {
                // A side o-major, B side k-major (each in its operand's own orientation, so that
                // every level is formed without a transpose)
                const InnerLevel &in = lv[l - 2];
                nf.X = ibase + in.off, nf.first = 0;
                if (side_b) nf.ld_o = 1, nf.ld_k = in.k_ld, nf.node_stride = in.k_stride;
                else nf.ld_o = in.y_ld, nf.ld_k = 1, nf.node_stride = in.y_stride;
            }
            // level l's rule (per-level rules: each level its own U, V; trees: each parent node
            // its own, coef_stride apart)
            const Algo &al = level_algo(plan, l - 1);
            const bool per = !tab->lucoef.empty();
            nf.nO = side_b ? al.N0 : al.M0, nf.nK = al.K0, nf.side_b = side_b ? 1 : 0, nf.R_ = al.R;
            nf.coef = side_b ? (per ? tab->lvcoef[(size_t)l - 1] : tab->vcoef) : (per ? tab->lucoef[(size_t)l - 1] : tab->ucoef);
            nf.coef_stride = plan->tree.empty() ? 0 : (int64_t)nf.nO * nf.nK * al.R;
            nf.last = 0;
            if (l == s.L) {
                nf.cb_o = side_b ? s.nb : s.mb, nf.cb_k = s.kb;
                if (side_b) {
                    nf.Y = ws + w.xb, nf.y_ld = wd.xb_ld, nf.y_stride = s.kb * wd.xb_ld, nf.kmajor = 1;
                } else {
                    nf.Y = ws + w.xa, nf.y_ld = wd.xa_ld, nf.y_stride = s.mb * wd.xa_ld;
                }
            } else {
                const InnerLevel &out = lv[l - 1];
                nf.cb_o = out.cb_o, nf.cb_k = out.cb_k;
                nf.Y = ibase + out.off, nf.y_ld = out.y_ld, nf.y_stride = out.y_stride;
                if (l == upto && side_b) {  // the fused kernel's B operand: k-major, unpadded
                    nf.y_ld = out.cb_o, nf.y_stride = out.cb_k * out.cb_o, nf.kmajor = 1;
                } else if (side_b) {
                    nf.y_ld = out.k_ld, nf.y_stride = out.k_stride, nf.kmajor = 1;
                }
            }
            if (nodes > 65535) return hipErrorInvalidValue;
            hipError_t er = launch_form_node(plan->prec, nf, (int)nodes, st);
            if (er != hipSuccess) return er;
            nodes *= al.R;
        }
        return hipSuccess;
    };
    hipError_t e = form_side(false);
    return e != hipSuccess ? e : form_side(true);
}

// ---- scaling at every level
// From depth 2, a plan with per-level scaling runs the first level itself: the scaling steps
// on op(A), op(B); the node operands S_r, T_r of eq. (2) written out with those factors
// applied; each node product by the plan of the remaining levels (which scales S_r, T_r in
// turn); the W-combination with the factors D_A, D_B of the first step.
bool every_level(const fastmm_plan_s *p, const Shape &s) {
    return p->sc.per_level && p->sc.mode != FASTMM_SCALE_NONE && s.L >= 2;
}

// The plan of the node products of a depth-L call: levels 2 .. L of p, same cutoff, scaling,
// precision and fusion.
fastmm_status node_plan(fastmm_plan_s *p, int L, fastmm_plan_s **out) {
    std::lock_guard<std::mutex> g(p->mu);
    std::unique_ptr<fastmm_plan_s> &q = p->node_plans[L];
    if (!q) {
        q.reset(new (std::nothrow) fastmm_plan_s());
        if (!q) return fail(FASTMM_ENOMEM, "plan allocation");
        q->algo = p->algo, q->depth = L - 1, q->cutoff = p->cutoff, q->sc = p->sc, q->prec = p->prec;
        q->fuse = p->fuse, q->tile = p->tile;
        if (!p->levels.empty()) q->levels.assign(p->levels.begin() + 1, p->levels.begin() + L);
    }
    *out = q.get();
    return FASTMM_OK;
}

// Workspace: [scaling part] | [S_r nodes][T_r nodes][node products] elems | [workspace of the
// node products' calls, shared by them in turn].
struct EveryLevelWs {
    WsLayout sc;
    size_t sn, tn, mn, sub, sub_bytes, total;
    int64_t mb1, kb1, nb1;
    int nodes;
    fastmm_plan_s *child;
};

fastmm_status every_level_layout(fastmm_plan_s *p, const Shape &s, int64_t m, int64_t k, int64_t n,
                                 EveryLevelWs &w) {
    w = EveryLevelWs{};
    const Algo &a = level_algo(p, 0);
    w.mb1 = s.Mp / a.M0, w.kb1 = s.Kp / a.K0, w.nb1 = s.Np / a.N0;
    w.nodes = leaf_count(a, 1);
    const size_t es = elem_size(p->prec);
    size_t off = scaling_layout(p, m, k, n, w.sc);
    w.sn = off, off = align256(off + es * (size_t)w.nodes * w.mb1 * w.kb1);
    w.tn = off, off = align256(off + es * (size_t)w.nodes * w.kb1 * w.nb1);
    w.mn = off, off = align256(off + es * (size_t)w.nodes * w.mb1 * w.nb1);
    fastmm_status st = node_plan(p, s.L, &w.child);
    if (st != FASTMM_OK) return st;
    if ((st = fastmm_workspace_size(w.child, w.mb1, w.kb1, w.nb1, &w.sub_bytes)) != FASTMM_OK) return st;
    w.sub = off, off = align256(off + w.sub_bytes);
    w.total = off;
    return FASTMM_OK;
}

fastmm_status every_level_total(fastmm_plan_s *p, const Shape &s, int64_t m, int64_t k, int64_t n, size_t *bytes) {
    EveryLevelWs w;
    fastmm_status st = every_level_layout(p, s, m, k, n, w);
    if (st == FASTMM_OK) *bytes = w.total;
    return st;
}

fastmm_status gemm_every_level(fastmm_plan_s *p, const Shape &s, const void *A, int64_t lda, int transA,
                               const void *B, int64_t ldb, int transB, void *C, int64_t ldc, int64_t m, int64_t k,
                               int64_t n, void *workspace, size_t ws_bytes, hipStream_t st) {
    EveryLevelWs w;
    fastmm_status stt = every_level_layout(p, s, m, k, n, w);
    if (stt != FASTMM_OK) return stt;
    if (workspace == nullptr || ws_bytes < w.total)
        return fail(FASTMM_EWORKSPACE, "workspace of " + std::to_string(w.total) + " bytes required");
    if (((uintptr_t)workspace & 255) != 0) return fail(FASTMM_EINVAL, "workspace must be 256-byte aligned");
    Tables *tab = nullptr;
    if ((stt = get_tables(p, 1, &tab)) != FASTMM_OK) return stt;
    if (tab->nleaves != w.nodes) return fail(FASTMM_EUNSUPPORTED, "node count mismatch");
    char *ws = (char *)workspace;
    const size_t es = elem_size(p->prec);
    const Elem el = p->prec == FASTMM_F64 ? Elem::F64 : Elem::F32;
    // The profiler records the node products' calls (each with its own phases, so that the
    // product kernels' durations stay per launch), not this level.
    ScaleExps exps;
    stt = run_scaling(p, A, lda, transA, B, ldb, transB, m, k, n, ws, w.sc, st, &exps);
    if (stt != FASTMM_OK) return stt;
    NodeDense fa{};
    fa.elem = el, fa.X = A, fa.ld_r = transA ? 1 : lda, fa.ld_c = transA ? lda : 1, fa.R = m, fa.K = k;
    fa.rb = w.mb1, fa.cb = w.kb1, fa.nodes = tab->leaves, fa.src = tab->asrc, fa.b_side = 0;
    fa.e_r = exps.ea, fa.e_c = exps.ep, fa.s_r = -1, fa.s_c = 1;  // 2^(ep_kk - ea_i)
    fa.Y = ws + w.sn, fa.y_stride = w.mb1 * w.kb1, fa.y_ld = w.kb1;
    NodeDense fb{};
    fb.elem = el, fb.X = B, fb.ld_r = transB ? 1 : ldb, fb.ld_c = transB ? ldb : 1, fb.R = k, fb.K = n;
    fb.rb = w.kb1, fb.cb = w.nb1, fb.nodes = tab->leaves, fb.src = tab->bsrc, fb.b_side = 1;
    fb.e_r = exps.ep, fb.e_c = exps.eb, fb.s_r = -1, fb.s_c = -1;  // 2^(-ep_kk - eb_j)
    fb.Y = ws + w.tn, fb.y_stride = w.kb1 * w.nb1, fb.y_ld = w.nb1;
    hipError_t e;
    if ((e = launch_node_dense(fa, w.nodes, st)) != hipSuccess || (e = launch_node_dense(fb, w.nodes, st)) != hipSuccess)
        return hip_fail(e, "node operand formation");
    for (int q = 0; q < w.nodes; ++q) {
        stt = fastmm_gemm_ex(w.child, ws + w.sn + es * (size_t)q * w.mb1 * w.kb1, w.kb1, 0,
                             ws + w.tn + es * (size_t)q * w.kb1 * w.nb1, w.nb1, 0,
                             ws + w.mn + es * (size_t)q * w.mb1 * w.nb1, w.nb1, w.mb1, w.kb1, w.nb1,
                             ws + w.sub, w.sub_bytes, st);
        if (stt != FASTMM_OK) return stt;
    }
    CombineLaunch Cb;
    Cb.elem = el;
    Cb.M = ws + w.mn;
    Cb.leaf_stride = w.mb1 * w.nb1;
    Cb.C = C, Cb.ldc = ldc, Cb.m = m, Cb.n = n, Cb.mb = w.mb1, Cb.nb = w.nb1;
    Cb.NB = tab->NB;
    Cb.bdest = tab->bdest, Cb.dest = tab->dest;
    Cb.sc = exps;
    set_kron(p, 1, tab->nleaves, Cb);
    if ((e = launch_combine(Cb, st)) != hipSuccess) return hip_fail(e, "combine kernel");
    return FASTMM_OK;
}

}  // namespace
}  // namespace fastmm

fastmm_status fastmm_gemm_ex(fastmm_plan_t plan, const void *A, int64_t lda, int transA, const void *B, int64_t ldb,
                             int transB, void *C, int64_t ldc, int64_t m, int64_t k, int64_t n, void *workspace,
                             size_t ws_bytes, void *stream) {
    if (check_plan(plan)) return FASTMM_EINVAL;
    if (m < 0 || k < 0 || n < 0) return fail(FASTMM_EINVAL, "negative size");
    if (m == 0 || n == 0) return FASTMM_OK;
    if (!C) return fail(FASTMM_EINVAL, "null C");
    if (ldc < n) return fail(FASTMM_ESHAPE, "ldc < n");
    const size_t es = elem_size(plan->prec);
    hipStream_t st = (hipStream_t)stream;
    const size_t cbytes = span_bytes(m, n, ldc, es);
    if (k == 0) {
        hipError_t e = launch_zero_elems(plan->prec == FASTMM_F64 ? Elem::F64 : Elem::F32, C, ldc, m, n, st);
        return e == hipSuccess ? FASTMM_OK : hip_fail(e, "zero fill");
    }
    if (!A || !B) return fail(FASTMM_EINVAL, "null A or B");
    // op(A) is m x k: stored m x k (lda >= k) or k x m (lda >= m); likewise op(B).
    if (lda < (transA ? m : k)) return fail(FASTMM_ESHAPE, "lda too small");
    if (ldb < (transB ? k : n)) return fail(FASTMM_ESHAPE, "ldb too small");
    const size_t abytes = transA ? span_bytes(k, m, lda, es) : span_bytes(m, k, lda, es);
    const size_t bbytes = transB ? span_bytes(n, k, ldb, es) : span_bytes(k, n, ldb, es);
    if (ranges_overlap(C, cbytes, A, abytes) || ranges_overlap(C, cbytes, B, bbytes))
        return fail(FASTMM_EALIAS, "C overlaps A or B");
    const Shape s = shape_of(plan, m, k, n);
    if (((uintptr_t)A % es) || ((uintptr_t)B % es) || ((uintptr_t)C % es))
        return fail(FASTMM_EINVAL, "misaligned operand");
    if (every_level(plan, s))
        return gemm_every_level(plan, s, A, lda, transA, B, ldb, transB, C, ldc, m, k, n, workspace, ws_bytes, st);
    const WsLayout w = ws_layout(plan, s, m, k, n);
    if (w.total > 0 && (workspace == nullptr || ws_bytes < w.total))
        return fail(FASTMM_EWORKSPACE, "workspace of " + std::to_string(w.total) + " bytes required");
    if (w.total > 0 && ((uintptr_t)workspace & 255) != 0) return fail(FASTMM_EINVAL, "workspace must be 256-byte aligned");
    Tables *tab = nullptr;
    fastmm_status stt = get_tables(plan, s.L, &tab);
    if (stt != FASTMM_OK) return stt;
    char *ws = (char *)workspace;
    PhaseMarks fin(st);
    ScaleExps exps;
    stt = run_scaling(plan, A, lda, transA, B, ldb, transB, m, k, n, ws, w, st, &exps);
    fin.mark();
    if (stt != FASTMM_OK) return stt;
    const Elem el = plan->prec == FASTMM_F64 ? Elem::F64 : Elem::F32;
    LeafLaunch L;
    L.elem = el;
    L.prec = plan->prec;
    L.A = A, L.B = B;
    L.lda = lda, L.ldb = ldb;
    L.transA = transA ? 1 : 0, L.transB = transB ? 1 : 0;
    L.m = m, L.k = k, L.n = n;
    L.mb = s.mb, L.kb = s.kb, L.nb = s.nb;
    L.nleaves = tab->nleaves;
    L.leaves = tab->leaves, L.asrc = tab->asrc, L.bsrc = tab->bsrc;
    L.sc = exps;
    hipError_t e;
    if (is_split(plan->prec) && fused_split(plan, s)) {
        // Split precisions, innermost level fused into the limb GEMM's loads: node operands,
        // then the fused limb GEMM over all leaves, then (L >= 1) the W-combination.
        const bool f16 = plan->prec == FASTMM_F16 || plan->prec == FASTMM_F16X3;
        const int pre = (f16 && exps.ea && schedule_of(plan->sc).find('O') != std::string::npos) ? 8 : 0;
        LimbFused f;
        if ((e = fused_split_operands(plan, s, A, lda, transA, B, ldb, transB, m, k, n, exps, pre, ws, w, tab, st,
                                      f)) != hipSuccess)
            return hip_fail(e, "node operand formation");
        fin.mark();
        if (s.L == 0) {
            f.out = (float *)C, f.ldo = ldc, f.leaf_stride = 0, f.direct = 1;
        } else {
            f.out = (float *)(ws + w.leaves), f.ldo = s.nb, f.leaf_stride = s.mb * s.nb, f.direct = 0;
        }
        e = launch_limb_fused(plan->prec, f, tab->nleaves, st);
        fin.mark();
        if (e != hipSuccess) return hip_fail(e, "fused limb GEMM kernel");
        if (s.L == 0) return FASTMM_OK;
        CombineLaunch Cb;
        Cb.elem = el;
        Cb.M = ws + w.leaves;
        Cb.leaf_stride = s.mb * s.nb;
        Cb.C = C, Cb.ldc = ldc, Cb.m = m, Cb.n = n, Cb.mb = s.mb, Cb.nb = s.nb;
        Cb.NB = tab->NB;
        Cb.bdest = tab->bdest, Cb.dest = tab->dest;
        Cb.sc = exps;
        if (const fastmm_status cs = set_combine(plan, s, tab, ws, w, Cb)) return cs;
        if ((e = launch_combine(Cb, st)) != hipSuccess) return hip_fail(e, "combine kernel");
        return FASTMM_OK;
    }
    if (is_split(plan->prec)) {
        // Split precisions: limb planes of every S_r and T_r^T (k contiguous, zero-padded to
        // the GEMM tiles), then the limb GEMM, then (L >= 1) the W-combination.
        const SplitDims d = split_dims(plan, s);
        LimbGemm g;
        if ((e = split_form(plan, s, d, A, lda, transA, B, ldb, transB, m, k, n, exps, ws, w, tab, st, g)) != hipSuccess)
            return hip_fail(e, "limb plane formation");
        fin.mark();
        if (s.L == 0) {
            g.out = (float *)C, g.ldo = ldc, g.leaf_stride = 0, g.direct = 1;
        } else {
            g.out = (float *)(ws + w.leaves), g.ldo = s.nb, g.leaf_stride = s.mb * s.nb, g.direct = 0;
        }
        e = launch_limb_gemm(plan->prec, d.bm, g, tab->nleaves, st);
        fin.mark();
        if (e != hipSuccess) return hip_fail(e, "limb GEMM kernel");
        if (s.L == 0) return FASTMM_OK;
        CombineLaunch Cb;
        Cb.elem = el;
        Cb.M = ws + w.leaves;
        Cb.leaf_stride = s.mb * s.nb;
        Cb.C = C, Cb.ldc = ldc, Cb.m = m, Cb.n = n, Cb.mb = s.mb, Cb.nb = s.nb;
        Cb.NB = tab->NB;
        Cb.bdest = tab->bdest, Cb.dest = tab->dest;
        Cb.sc = exps;
        if (const fastmm_status cs = set_combine(plan, s, tab, ws, w, Cb)) return cs;
        if ((e = launch_combine(Cb, st)) != hipSuccess) return hip_fail(e, "combine kernel");
        return FASTMM_OK;
    }
    // FP64 / FP32 outside the written path: scaled plans and transposed operands run on
    // row-major (scaled) copies of the operands (one pass, cheaper than applying the factors to
    // every loaded element: the products kernels re-read each operand element many times)
    const bool written = written_taken(plan, s);
    const bool fw = !written && fused_written(plan, s);  // outer levels written, then fused
    const bool scaled_copy = !written && !fw && exps.ea != nullptr;
    if (!written && !fw && (scaled_copy || transA || transB)) {
        if ((e = prescale_operands(plan, s, A, lda, transA, B, ldb, transB, m, k, n, exps, scaled_copy, ws, w, tab,
                                   st, &A, &lda, &B, &ldb)) != hipSuccess)
            return hip_fail(e, "operand copies");
        transA = transB = 0;
        L.A = A, L.B = B, L.lda = lda, L.ldb = ldb, L.transA = L.transB = 0;
        // the products read scaled copies; a single leaf still scales its output
        if (scaled_copy && s.L >= 1) L.sc = ScaleExps{nullptr, nullptr, nullptr};
        if (scaled_copy && s.L == 0) L.scale_in = 0;
    }
    uint32_t masks[6];
    const bool fused = fw ? fused_path(plan, s, 0, 0, masks) : fused_path(plan, s, transA, transB, masks);
    if (fw) {
        if ((e = form_written(plan, s, A, lda, transA, B, ldb, transB, m, k, n, exps, ws, w, tab, st, s.L - 1)) !=
            hipSuccess)
            return hip_fail(e, "node operand formation");
    }
    if (written) {
        // leaf operands written out level by level, then one launch over the stacked blocks
        // (one source per leaf, unscaled: the formation applied the factors), then the
        // W-combination with D_A, D_B
        if ((e = form_written(plan, s, A, lda, transA, B, ldb, transB, m, k, n, exps, ws, w, tab, st, s.L)) !=
            hipSuccess)
            return hip_fail(e, "leaf operand formation");
        fin.mark();
        const WrittenDims wd = written_dims(s);
        LeafLaunch X = L;
        X.A = ws + w.xa, X.lda = wd.xa_ld, X.transA = 0;
        X.B = ws + w.xb, X.ldb = wd.xb_ld, X.transB = 0;
        X.m = (int64_t)tab->nleaves * s.mb, X.k = (int64_t)tab->nleaves * s.kb, X.n = s.nb;
        X.leaves = tab->wleaves, X.asrc = tab->wsrc, X.bsrc = tab->wsrc;
        X.sc = ScaleExps{nullptr, nullptr, nullptr};
        X.out = ws + w.leaves, X.ldo = s.nb, X.leaf_stride = s.mb * s.nb, X.direct = 0;
        X.one = 1;
        e = launch_leaf(X, st);
        fin.mark();
        if (e != hipSuccess) return hip_fail(e, "leaf kernel");
        CombineLaunch Cb;
        Cb.elem = el;
        Cb.M = ws + w.leaves;
        Cb.leaf_stride = s.mb * s.nb;
        Cb.C = C, Cb.ldc = ldc, Cb.m = m, Cb.n = n, Cb.mb = s.mb, Cb.nb = s.nb;
        Cb.NB = tab->NB;
        Cb.bdest = tab->bdest, Cb.dest = tab->dest;
        Cb.sc = exps;
        if (const fastmm_status cs = set_combine(plan, s, tab, ws, w, Cb)) return cs;
        if ((e = launch_combine(Cb, st)) != hipSuccess) return hip_fail(e, "combine kernel");
        return FASTMM_OK;
    }
    fin.mark();  // no operand formation pass on the other FP64 / FP32 paths
    if (fused) {
        // The innermost level runs fused; the L-1 outer levels supply the node operands and,
        // for L >= 2, the W-combination of the node products.
        Tables *outer = nullptr;
        if ((stt = get_tables(plan, s.L - 1, &outer)) != FASTMM_OK) return stt;
        NodeLaunch N;
        N.elem = el;
        N.A = A, N.B = B;
        N.lda = lda, N.ldb = ldb;
        N.m = m, N.k = k, N.n = n;
        N.mb = s.mb, N.kb = s.kb, N.nb = s.nb;
        N.nnodes = outer->nleaves;
        N.outer = outer->leaves, N.asrc = outer->asrc, N.bsrc = outer->bsrc;
        N.sc = exps;  // the operands are the scaled copies when the plan scales
        if (fw) {
            // node q's operands: rows q cb_o of the stacked A side, rows q cb_k of the k-major B
            // side (one source each, block row q); bounds over the stacks
            const InnerLevel la = inner_levels(plan, s, false)[(size_t)s.L - 2];
            const InnerLevel lb = inner_levels(plan, s, true)[(size_t)s.L - 2];
            N.A = ws + w.ia + la.off, N.lda = la.y_ld;
            N.B = ws + w.ib + lb.off, N.ldb = lb.cb_o;
            N.m = (int64_t)outer->nleaves * la.cb_o, N.k = (int64_t)outer->nleaves * la.cb_k, N.n = lb.cb_o;
            N.outer = outer->wleaves, N.asrc = outer->wsrc, N.bsrc = outer->wsrc;
        }
        for (int i = 0; i < 6; ++i) N.masks[i] = masks[i];
        if (s.L == 1) {
            N.out = C, N.ldo = ldc, N.node_stride = 0;
        } else {
            N.out = ws + w.leaves, N.ldo = 2 * s.nb, N.node_stride = 4 * s.mb * s.nb;
        }
        e = launch_node222(N, st);
        fin.mark();
        if (e != hipSuccess) return hip_fail(e, "fused node kernel");
        if (s.L == 1) return FASTMM_OK;
        CombineLaunch Cb;
        Cb.elem = el;
        Cb.M = ws + w.leaves;
        Cb.leaf_stride = 4 * s.mb * s.nb;
        Cb.C = C, Cb.ldc = ldc, Cb.m = m, Cb.n = n, Cb.mb = 2 * s.mb, Cb.nb = 2 * s.nb;
        Cb.NB = outer->NB;
        Cb.bdest = outer->bdest, Cb.dest = outer->dest;
        Cb.sc = exps;
        set_kron(plan, s.L - 1, outer->nleaves, Cb);
        if ((e = launch_combine(Cb, st)) != hipSuccess) return hip_fail(e, "combine kernel");
        return FASTMM_OK;
    }
    auto leaf_launch = [&]() { return launch_leaf(L, st); };
    if (s.L == 0) {
        L.out = C, L.ldo = ldc, L.leaf_stride = 0, L.direct = 1;
        L.one = 1;  // a single leaf: the operands themselves
        e = leaf_launch();
        fin.mark();
        if (e != hipSuccess) return hip_fail(e, "leaf kernel");
        return FASTMM_OK;
    }
    L.out = ws + w.leaves, L.ldo = s.nb, L.leaf_stride = s.mb * s.nb, L.direct = 0;
    e = leaf_launch();
    fin.mark();
    if (e != hipSuccess) return hip_fail(e, "leaf kernel");
    CombineLaunch Cb;
    Cb.elem = el;
    Cb.M = ws + w.leaves;
    Cb.leaf_stride = s.mb * s.nb;
    Cb.C = C, Cb.ldc = ldc, Cb.m = m, Cb.n = n, Cb.mb = s.mb, Cb.nb = s.nb;
    Cb.NB = tab->NB;
    Cb.bdest = tab->bdest, Cb.dest = tab->dest;
    Cb.sc = exps;
    if (const fastmm_status cs = set_combine(plan, s, tab, ws, w, Cb)) return cs;
    if ((e = launch_combine(Cb, st)) != hipSuccess) return hip_fail(e, "combine kernel");
    return FASTMM_OK;
}

fastmm_status fastmm_gemm(fastmm_plan_t plan, const void *A, const void *B, void *C, int64_t m, int64_t k, int64_t n,
                          void *workspace, size_t ws_bytes, void *stream) {
    return fastmm_gemm_ex(plan, A, k, 0, B, n, 0, C, n, m, k, n, workspace, ws_bytes, stream);
}

namespace fastmm {
namespace {
// Sub-plan of `p` for a gradient product (which = 0: dA = G B^T, a <M0,N0,K0> product; 1:
// dB = A^T G, a <K0,M0,N0> product): every level's (or tree node's) rule replaced by the
// transpose of its rotation (section 3.1), same depth, cutoff, scaling, precision, fusion mode
// and tile.  Rotation and transposition keep the product indices, so a tree keeps its node
// numbering.
fastmm_status grad_plan(fastmm_plan_s *p, int which, fastmm_plan_s **out) {
    const int times = which == 0 ? 2 : 1;
    std::lock_guard<std::mutex> g(p->mu);
    if (!p->grad[which]) {
        const int id = algo_transposed_rotation(p->algo, times);
        if (id < 0) return fail(FASTMM_EUNSUPPORTED, "cannot form the backward rule");
        std::unique_ptr<fastmm_plan_s> q(new (std::nothrow) fastmm_plan_s());
        if (!q) return fail(FASTMM_ENOMEM, "plan allocation");
        q->algo = id, q->depth = p->depth, q->cutoff = p->cutoff, q->sc = p->sc, q->prec = p->prec, q->fuse = p->fuse;
        q->tile = p->tile;
        for (int lid : p->levels) {  // non-stationary: every level's rule transformed alike
            const int r = algo_transposed_rotation(lid, times);
            if (r < 0) return fail(FASTMM_EUNSUPPORTED, "cannot form a level's backward rule");
            q->levels.push_back(r);
        }
        for (int nid : p->tree) {  // non-uniform: every node's rule transformed alike
            const int r = algo_transposed_rotation(nid, times);
            if (r < 0) return fail(FASTMM_EUNSUPPORTED, "cannot form a tree node's backward rule");
            q->tree.push_back(r);
        }
        p->grad[which] = std::move(q);
    }
    *out = p->grad[which].get();
    return FASTMM_OK;
}
}  // namespace
}  // namespace fastmm

namespace fastmm {
namespace {
constexpr int kModes = 4;  // FP32 / FP64 batch items: scaled operands or not x output to C or not
struct BatchLayout {
    std::vector<size_t> ws_off, ws_size;
    std::vector<size_t> copy_a, copy_b;  // FP64 / FP32: row-major copies of transposed operands (offsets
                                         // inside the problem's region; 0 = none)
    size_t descs = 0, first = 0, total = 0;
    int bm = 0;  // split precisions: the limb-GEMM tile shared by the batch
};

fastmm_status batch_layout(const fastmm_plan_t *plans, const fastmm_problem_ex *probs, int count, BatchLayout &bl) {
    if (count < 0 || (count > 0 && (!plans || !probs))) return fail(FASTMM_EINVAL, "bad batch arguments");
    if (count > 65536) return fail(FASTMM_EINVAL, "batch too large");
    size_t off = 0;
    int prec = -1;
    for (int i = 0; i < count; ++i) {
        if (!plans[i]) return fail(FASTMM_EINVAL, "null plan in batch");
        if (check_plan(plans[i])) return FASTMM_EINVAL;
        if (prec < 0) prec = plans[i]->prec;
        if (plans[i]->prec != prec) return fail(FASTMM_EUNSUPPORTED, "batched plans must share one precision");
        const fastmm_problem_ex &q = probs[i];
        if (q.m < 0 || q.k < 0 || q.n < 0) return fail(FASTMM_EINVAL, "negative size in batch");
    }
    if (count > 0 && is_split(prec)) {  // one limb-GEMM tile for the whole batch
        bl.bm = 256;
        for (int i = 0; i < count; ++i) {
            const Shape s = shape_of(plans[i], probs[i].m, probs[i].k, probs[i].n);
            bl.bm = std::min(bl.bm, plan_tile(plans[i], s));
        }
    }
    const size_t es = prec < 0 ? 8 : elem_size(prec);
    for (int i = 0; i < count; ++i) {
        const fastmm_problem_ex &q = probs[i];
        const Shape s = shape_of(plans[i], q.m, q.k, q.n);
        if (every_level(plans[i], s))
            return fail(FASTMM_EUNSUPPORTED, "scaling at every level runs through fastmm_gemm_ex, not in a batch");
        size_t w = ws_layout(plans[i], s, q.m, q.k, q.n, bl.bm, true).total;
        size_t ca = 0, cb = 0;
        if (!is_split(prec) && q.transA) ca = align256(w), w = ca + align256(es * (size_t)q.m * q.k);
        if (!is_split(prec) && q.transB) cb = align256(w), w = cb + align256(es * (size_t)q.k * q.n);
        bl.ws_off.push_back(off);
        bl.ws_size.push_back(w);
        bl.copy_a.push_back(ca);
        bl.copy_b.push_back(cb);
        off = align256(off + w);
    }
    const Elem el = prec == FASTMM_F64 ? Elem::F64 : Elem::F32;
    const size_t db = is_split(prec) ? sizeof(LimbGemm) : leaf_desc_bytes(el);
    bl.descs = off, off = align256(off + db * (size_t)std::max(count, 1));
    bl.first = off, off = align256(off + 8 * (size_t)(count + kModes));  // one prefix array per mode
    bl.total = off;
    return FASTMM_OK;
}

// Contiguous problems as strided ones (leading dimensions = row lengths, no transposes).
void problems_ex(const fastmm_problem *probs, int count, std::vector<fastmm_problem_ex> &v) {
    for (int i = 0; probs && i < count; ++i) {
        const fastmm_problem &q = probs[i];
        v.push_back(fastmm_problem_ex{q.A, q.k, 0, q.B, q.n, 0, q.C, q.n, q.m, q.k, q.n});
    }
}

int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cus = v;
        else
            cus = 256;
    }
    return cus;
}
}  // namespace
}  // namespace fastmm

fastmm_status fastmm_batched_ex_workspace_size(const fastmm_plan_t *plans, const fastmm_problem_ex *probs, int count,
                                               size_t *bytes) {
    if (!bytes) return fail(FASTMM_EINVAL, "null output");
    BatchLayout bl;
    fastmm_status st = batch_layout(plans, probs, count, bl);
    if (st == FASTMM_OK) *bytes = bl.total;
    return st;
}

fastmm_status fastmm_batched_workspace_size(const fastmm_plan_t *plans, const fastmm_problem *probs, int count,
                                            size_t *bytes) {
    if (count < 0 || (count > 0 && !probs)) return fail(FASTMM_EINVAL, "bad batch arguments");
    std::vector<fastmm_problem_ex> ex;
    problems_ex(probs, count, ex);
    return fastmm_batched_ex_workspace_size(plans, ex.data(), count, bytes);
}

fastmm_status fastmm_gemm_batched(const fastmm_plan_t *plans, const fastmm_problem *probs, int count, void *workspace,
                                  size_t ws_bytes, void *stream) {
    if (count < 0 || (count > 0 && !probs)) return fail(FASTMM_EINVAL, "bad batch arguments");
    std::vector<fastmm_problem_ex> ex;
    problems_ex(probs, count, ex);
    return fastmm_gemm_batched_ex(plans, ex.data(), count, workspace, ws_bytes, stream);
}

fastmm_status fastmm_gemm_batched_ex(const fastmm_plan_t *plans, const fastmm_problem_ex *probs, int count,
                                     void *workspace, size_t ws_bytes, void *stream) {
    BatchLayout bl;
    fastmm_status st = batch_layout(plans, probs, count, bl);
    if (st != FASTMM_OK) return st;
    if (count == 0) return FASTMM_OK;
    if (workspace == nullptr || ws_bytes < bl.total) return fail(FASTMM_EWORKSPACE, "batch workspace too small");
    if (((uintptr_t)workspace & 255) != 0) return fail(FASTMM_EINVAL, "workspace must be 256-byte aligned");
    const Elem el = plans[0]->prec == FASTMM_F64 ? Elem::F64 : Elem::F32;
    const size_t es = elem_size(plans[0]->prec);
    const bool split = is_split(plans[0]->prec);
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    // validate every problem before launching anything
    auto a_bytes = [&](const fastmm_problem_ex &q) {
        return q.transA ? span_bytes(q.k, q.m, q.lda, es) : span_bytes(q.m, q.k, q.lda, es);
    };
    auto b_bytes = [&](const fastmm_problem_ex &q) {
        return q.transB ? span_bytes(q.n, q.k, q.ldb, es) : span_bytes(q.k, q.n, q.ldb, es);
    };
    for (int i = 0; i < count; ++i) {
        const fastmm_problem_ex &q = probs[i];
        if (q.m == 0 || q.n == 0) continue;
        if (!q.C || (q.k > 0 && (!q.A || !q.B))) return fail(FASTMM_EINVAL, "null operand in batch");
        if (q.ldc < q.n) return fail(FASTMM_ESHAPE, "ldc < n in batch");
        if (q.k > 0 && (q.lda < (q.transA ? q.m : q.k) || q.ldb < (q.transB ? q.k : q.n)))
            return fail(FASTMM_ESHAPE, "lda or ldb too small in batch");
        const size_t cb = span_bytes(q.m, q.n, q.ldc, es);
        for (int j = 0; j < count; ++j) {
            const fastmm_problem_ex &r = probs[j];
            if (r.k > 0 && r.m > 0 && r.n > 0 &&
                (ranges_overlap(q.C, cb, r.A, a_bytes(r)) || ranges_overlap(q.C, cb, r.B, b_bytes(r))))
                return fail(FASTMM_EALIAS, "a batch output overlaps an input");
            if (j != i && r.m > 0 && r.n > 0 && ranges_overlap(q.C, cb, r.C, span_bytes(r.m, r.n, r.ldc, es)))
                return fail(FASTMM_EALIAS, "batch outputs overlap");
        }
        if (((uintptr_t)q.A % es) || ((uintptr_t)q.B % es) || ((uintptr_t)q.C % es))
            return fail(FASTMM_EINVAL, "misaligned operand in batch");
    }
    struct Item {
        int idx;
        int64_t kb;
        std::vector<char> desc;
        int mode;  // FP32 / FP64: 2 * scaled + direct (one launch per mode); split: 0
        int64_t tiles;
        CombineLaunch cb;
        bool combine;
    };
    std::vector<Item> items;
    hipError_t e;
    PhaseMarks fin(s);
    // every problem's scaling steps, then every problem's operand formation (split precisions)
    std::vector<ScaleExps> exps_all(count);
    for (int i = 0; i < count; ++i) {
        const fastmm_problem_ex &q = probs[i];
        fastmm_plan_s *p = plans[i];
        if (q.m == 0 || q.n == 0 || q.k == 0) continue;
        const Shape sh = shape_of(p, q.m, q.k, q.n);
        const WsLayout w = ws_layout(p, sh, q.m, q.k, q.n, bl.bm, true);
        if ((st = run_scaling(p, q.A, q.lda, q.transA, q.B, q.ldb, q.transB, q.m, q.k, q.n, ws + bl.ws_off[i], w, s,
                              &exps_all[i])) != FASTMM_OK)
            return st;
    }
    fin.mark();
    for (int i = 0; i < count; ++i) {
        const fastmm_problem_ex &q = probs[i];
        fastmm_plan_s *p = plans[i];
        if (q.m == 0 || q.n == 0) continue;
        if (q.k == 0) {
            if ((e = launch_zero_elems(el, q.C, q.ldc, q.m, q.n, s)) != hipSuccess) return hip_fail(e, "zero fill");
            continue;
        }
        const Shape sh = shape_of(p, q.m, q.k, q.n);
        const WsLayout w = ws_layout(p, sh, q.m, q.k, q.n, bl.bm, true);
        char *pws = ws + bl.ws_off[i];
        Tables *tab = nullptr;
        if ((st = get_tables(p, sh.L, &tab)) != FASTMM_OK) return st;
        const ScaleExps exps = exps_all[i];
        if (split) {
            // limb planes now; the products of every problem in the one launch below
            Item it;
            it.idx = i;
            it.kb = sh.kb;
            it.combine = sh.L > 0;
            const SplitDims d = split_dims(p, sh, bl.bm);
            LimbGemm g;
            if ((e = split_form(p, sh, d, q.A, q.lda, q.transA, q.B, q.ldb, q.transB, q.m, q.k, q.n, exps, pws, w,
                                tab, s, g)) != hipSuccess)
                return hip_fail(e, "limb plane formation");
            if (sh.L == 0) {
                g.out = (float *)q.C, g.ldo = q.ldc, g.leaf_stride = 0, g.direct = 1;
            } else {
                g.out = (float *)(pws + w.leaves), g.ldo = sh.nb, g.leaf_stride = sh.mb * sh.nb, g.direct = 0;
                CombineLaunch &c = it.cb;
                c.elem = el;
                c.M = pws + w.leaves;
                c.leaf_stride = sh.mb * sh.nb;
                c.C = q.C, c.ldc = q.ldc, c.m = q.m, c.n = q.n, c.mb = sh.mb, c.nb = sh.nb;
                c.NB = tab->NB, c.bdest = tab->bdest, c.dest = tab->dest, c.sc = exps;
                if (const fastmm_status cs = set_combine(p, sh, tab, pws, w, c)) return cs;
            }
            it.mode = 0;
            it.desc.resize(sizeof(LimbGemm));
            std::memcpy(it.desc.data(), &g, sizeof(LimbGemm));
            it.tiles = (int64_t)tab->nleaves * g.tiles_m * g.tiles_n;
            items.push_back(std::move(it));
            continue;
        }
        // the batched leaf kernel reads row-major operands: a transposed one is copied first
        const void *qa = q.A, *qb = q.B;
        int64_t qlda = q.lda, qldb = q.ldb;
        if (q.transA) {
            if ((e = launch_transpose(el, q.A, q.lda, q.k, q.m, pws + bl.copy_a[i], q.k, s)) != hipSuccess)
                return hip_fail(e, "operand copy");
            qa = pws + bl.copy_a[i], qlda = q.k;
        }
        if (q.transB) {
            if ((e = launch_transpose(el, q.B, q.ldb, q.n, q.k, pws + bl.copy_b[i], q.n, s)) != hipSuccess)
                return hip_fail(e, "operand copy");
            qb = pws + bl.copy_b[i], qldb = q.n;
        }
        LeafLaunch L;
        L.elem = el;
        L.prec = p->prec;
        L.A = qa, L.B = qb, L.lda = qlda, L.ldb = qldb, L.transA = 0, L.transB = 0;
        L.m = q.m, L.k = q.k, L.n = q.n, L.mb = sh.mb, L.kb = sh.kb, L.nb = sh.nb;
        L.nleaves = tab->nleaves;
        L.leaves = tab->leaves, L.asrc = tab->asrc, L.bsrc = tab->bsrc;
        L.sc = exps;
        const bool written = sh.L >= 1 && written_leaves(p, sh);
        if (written) {
            // leaf operands written out now (with the scaling factors); the batched launch
            // multiplies the stacked blocks, one source each, as fastmm_gemm_ex does
            if ((e = form_written(p, sh, qa, qlda, 0, qb, qldb, 0, q.m, q.k, q.n, exps, pws, w, tab, s, sh.L)) !=
                hipSuccess)
                return hip_fail(e, "leaf operand formation");
            const WrittenDims wd = written_dims(sh);
            L.A = pws + w.xa, L.lda = wd.xa_ld, L.B = pws + w.xb, L.ldb = wd.xb_ld;
            L.m = (int64_t)tab->nleaves * sh.mb, L.k = (int64_t)tab->nleaves * sh.kb, L.n = sh.nb;
            L.leaves = tab->wleaves, L.asrc = tab->wsrc, L.bsrc = tab->wsrc;
            L.sc = ScaleExps{nullptr, nullptr, nullptr};
        }
        Item it;
        it.idx = i;
        it.kb = sh.kb;
        it.combine = sh.L > 0;
        if (sh.L == 0) {
            L.out = q.C, L.ldo = q.ldc, L.leaf_stride = 0, L.direct = 1;
        } else {
            L.out = pws + w.leaves, L.ldo = sh.nb, L.leaf_stride = sh.mb * sh.nb, L.direct = 0;
            CombineLaunch &c = it.cb;
            c.elem = el;
            c.M = pws + w.leaves;
            c.leaf_stride = sh.mb * sh.nb;
            c.C = q.C, c.ldc = q.ldc, c.m = q.m, c.n = q.n, c.mb = sh.mb, c.nb = sh.nb;
            c.NB = tab->NB, c.bdest = tab->bdest, c.dest = tab->dest, c.sc = exps;
            if (const fastmm_status cs = set_combine(p, sh, tab, pws, w, c)) return cs;
        }
        // mode bits: one source per leaf (written leaf operands, or a classical product
        // unscaled), scaled loads, output to C
        const bool one = written || (sh.L == 0 && exps.ea == nullptr);
        it.mode = 4 * (one ? 1 : 0) + 2 * (L.sc.ea != nullptr ? 1 : 0) + (L.direct ? 1 : 0);
        it.desc.resize(leaf_desc_bytes(el));
        it.tiles = leaf_desc_build(L, it.desc.data());
        items.push_back(std::move(it));
    }
    fin.mark();
    // largest inner dimension first: the longest work items start earliest
    std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &b) {
        return a.mode != b.mode ? a.mode < b.mode : a.kb > b.kb;
    });
    // Host staging of the descriptor table: kept per thread until the copies of the previous
    // batched call on this thread have completed (an event marks them), so the stream never
    // has to be synchronised.
    thread_local struct Staging {
        std::vector<char> descs;
        std::vector<int64_t> first;
        hipEvent_t done = nullptr;
        bool pending = false;
    } stg;
    if (stg.pending && (e = hipEventSynchronize(stg.done)) != hipSuccess) return hip_fail(e, "staging wait");
    stg.pending = false;
    const size_t db = split ? sizeof(LimbGemm) : leaf_desc_bytes(el);
    stg.descs.assign(db * std::max<size_t>(items.size(), 1), 0);
    stg.first.clear();
    // one group of consecutive items per mode, each with its own prefix array of item offsets
    struct Group {
        size_t begin, end, first_off;
        int64_t total;
        int mode;
    };
    std::vector<Group> groups;
    for (size_t i = 0; i < items.size(); ++i) {
        std::memcpy(stg.descs.data() + i * db, items[i].desc.data(), db);
        if (groups.empty() || groups.back().mode != items[i].mode) {
            groups.push_back(Group{i, i, stg.first.size(), 0, items[i].mode});
            stg.first.push_back(0);
        }
        Group &g = groups.back();
        g.end = i + 1;
        g.total += items[i].tiles;
        stg.first.push_back(g.total);
    }
    if (!groups.empty()) {
        if (!stg.done && (e = hipEventCreateWithFlags(&stg.done, hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "staging event");
        if ((e = hipMemcpyAsync(ws + bl.descs, stg.descs.data(), db * items.size(), hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(ws + bl.first, stg.first.data(), 8 * stg.first.size(), hipMemcpyHostToDevice, s)) != hipSuccess)
            return hip_fail(e, "uploading batch descriptors");
        if ((e = hipEventRecord(stg.done, s)) != hipSuccess) return hip_fail(e, "staging event");
        stg.pending = true;
    }
    for (const Group &g : groups) {
        if (g.total <= 0) continue;
        const char *gd = ws + bl.descs + g.begin * db;
        const int64_t *gf = (const int64_t *)(ws + bl.first) + g.first_off;
        const int gc = (int)(g.end - g.begin);
        if (split) {
            if ((e = launch_limb_gemm_batched(plans[0]->prec, bl.bm, gd, gf, gc, g.total, s)) != hipSuccess)
                return hip_fail(e, "batched limb GEMM kernel");
        } else if ((e = launch_leaf_batched(el, (g.mode >> 1) & 1, g.mode & 1, g.mode >> 2, gd, gf, gc, g.total, s)) != hipSuccess) {
            return hip_fail(e, "batched leaf kernel");
        }
    }
    fin.mark();
    for (const Item &it : items)
        if (it.combine && (e = launch_combine(it.cb, s)) != hipSuccess) return hip_fail(e, "combine kernel");
    return FASTMM_OK;
}

fastmm_status fastmm_backward_workspace_size(fastmm_plan_t plan, int64_t m, int64_t k, int64_t n, size_t *bytes) {
    if (check_plan(plan)) return FASTMM_EINVAL;
    if (!bytes || m < 0 || k < 0 || n < 0) return fail(FASTMM_EINVAL, "bad arguments");
    fastmm_plan_s *ga = nullptr, *gb = nullptr;
    fastmm_status st;
    if ((st = grad_plan(plan, 0, &ga)) != FASTMM_OK || (st = grad_plan(plan, 1, &gb)) != FASTMM_OK) return st;
    size_t wa = 0, wb = 0;
    if ((st = fastmm_workspace_size(ga, m, n, k, &wa)) != FASTMM_OK) return st;  // dA = G B^T
    if ((st = fastmm_workspace_size(gb, k, m, n, &wb)) != FASTMM_OK) return st;  // dB = A^T G
    *bytes = std::max(wa, wb);
    return FASTMM_OK;
}

fastmm_status fastmm_gemm_backward(fastmm_plan_t plan, const void *A, const void *B, const void *G, void *dA,
                                   void *dB, int64_t m, int64_t k, int64_t n, void *workspace, size_t ws_bytes,
                                   void *stream) {
    if (check_plan(plan)) return FASTMM_EINVAL;
    if (m < 0 || k < 0 || n < 0) return fail(FASTMM_EINVAL, "negative size");
    const bool full = m > 0 && k > 0 && n > 0;  // empty products need no inputs (zero or nothing)
    if (full && ((dA && (!G || !B)) || (dB && (!G || !A)))) return fail(FASTMM_EINVAL, "null input");
    fastmm_plan_s *ga = nullptr, *gb = nullptr;
    fastmm_status st;
    if ((st = grad_plan(plan, 0, &ga)) != FASTMM_OK || (st = grad_plan(plan, 1, &gb)) != FASTMM_OK) return st;
    // Both products read their transposed operand through the transpose flags: the split
    // precisions form their limb planes from it directly, FP64 / FP32 copy it once.
    if (dA) {  // dA (m x k) = G (m x n) * B^T, B stored k x n
        st = fastmm_gemm_ex(ga, G, n, 0, B, n, 1, dA, k, m, n, k, workspace, ws_bytes, stream);
        if (st != FASTMM_OK) return st;
    }
    if (dB) {  // dB (k x n) = A^T * G (m x n), A stored m x k
        st = fastmm_gemm_ex(gb, A, k, 1, G, n, 0, dB, n, k, m, n, workspace, ws_bytes, stream);
        if (st != FASTMM_OK) return st;
    }
    return FASTMM_OK;
}

namespace fastmm {
namespace {
// The products of a batched backward pass: dA_i then dB_i for every problem that asks for
// them, with their plans.
fastmm_status grad_products(const fastmm_plan_t *plans, const fastmm_grad_problem *probs, int count,
                            std::vector<fastmm_plan_t> &gp, std::vector<fastmm_problem_ex> &gq) {
    if (count < 0 || (count > 0 && (!plans || !probs))) return fail(FASTMM_EINVAL, "bad batch arguments");
    for (int i = 0; i < count; ++i) {
        const fastmm_grad_problem &q = probs[i];
        if (!plans[i] || check_plan(plans[i])) return fail(FASTMM_EINVAL, "null plan in batch");
        if (q.m < 0 || q.k < 0 || q.n < 0) return fail(FASTMM_EINVAL, "negative size in batch");
        const bool full = q.m > 0 && q.k > 0 && q.n > 0;
        if (full && ((q.dA && (!q.G || !q.B)) || (q.dB && (!q.G || !q.A))))
            return fail(FASTMM_EINVAL, "null input in batch");
        fastmm_plan_s *ga = nullptr, *gb = nullptr;
        fastmm_status st;
        if ((st = grad_plan(plans[i], 0, &ga)) != FASTMM_OK || (st = grad_plan(plans[i], 1, &gb)) != FASTMM_OK)
            return st;
        if (q.dA) gp.push_back(ga), gq.push_back(fastmm_problem_ex{q.G, q.n, 0, q.B, q.n, 1, q.dA, q.k, q.m, q.n, q.k});
        if (q.dB) gp.push_back(gb), gq.push_back(fastmm_problem_ex{q.A, q.k, 1, q.G, q.n, 0, q.dB, q.n, q.k, q.m, q.n});
    }
    return FASTMM_OK;
}
}  // namespace
}  // namespace fastmm

fastmm_status fastmm_backward_batched_workspace_size(const fastmm_plan_t *plans, const fastmm_grad_problem *probs,
                                                     int count, size_t *bytes) {
    if (!bytes) return fail(FASTMM_EINVAL, "null output");
    std::vector<fastmm_plan_t> gp;
    std::vector<fastmm_problem_ex> gq;
    fastmm_status st = grad_products(plans, probs, count, gp, gq);
    if (st != FASTMM_OK) return st;
    return fastmm_batched_ex_workspace_size(gp.data(), gq.data(), (int)gq.size(), bytes);
}

fastmm_status fastmm_gemm_backward_batched(const fastmm_plan_t *plans, const fastmm_grad_problem *probs, int count,
                                           void *workspace, size_t ws_bytes, void *stream) {
    std::vector<fastmm_plan_t> gp;
    std::vector<fastmm_problem_ex> gq;
    fastmm_status st = grad_products(plans, probs, count, gp, gq);
    if (st != FASTMM_OK) return st;
    return fastmm_gemm_batched_ex(gp.data(), gq.data(), (int)gq.size(), workspace, ws_bytes, stream);
}

fastmm_status fastmm_task_table(fastmm_plan_t plan, int levels, int64_t counts[5], int32_t *leaves, int32_t *asrc,
                                double *acoef, int32_t *bsrc, double *bcoef, int32_t *bdest, int32_t *dest_leaf,
                                double *dest_coef) {
    if (check_plan(plan)) return FASTMM_EINVAL;
    if (levels < 0 || levels > 8 || !counts) return fail(FASTMM_EINVAL, "bad arguments");
    if (!plan->levels.empty() && levels > (int)plan->levels.size())
        return fail(FASTMM_EINVAL, "more levels than the plan's per-level rules");
    HostTables ht;
    std::string err;
    if (!build_plan_tables(plan, levels, ht, err)) return fail(FASTMM_EUNSUPPORTED, err);
    counts[0] = (int64_t)ht.leaves.size();
    counts[1] = (int64_t)ht.asrc.size();
    counts[2] = (int64_t)ht.bsrc.size();
    counts[3] = (int64_t)ht.bdest.size();
    counts[4] = (int64_t)ht.dest.size();
    for (size_t i = 0; leaves && i < ht.leaves.size(); ++i) {
        leaves[4 * i] = ht.leaves[i].a_begin, leaves[4 * i + 1] = ht.leaves[i].a_count;
        leaves[4 * i + 2] = ht.leaves[i].b_begin, leaves[4 * i + 3] = ht.leaves[i].b_count;
    }
    for (size_t i = 0; i < ht.asrc.size(); ++i) {
        if (asrc) asrc[2 * i] = ht.asrc[i].br, asrc[2 * i + 1] = ht.asrc[i].bc;
        if (acoef) acoef[i] = ht.asrc[i].coef;
    }
    for (size_t i = 0; i < ht.bsrc.size(); ++i) {
        if (bsrc) bsrc[2 * i] = ht.bsrc[i].br, bsrc[2 * i + 1] = ht.bsrc[i].bc;
        if (bcoef) bcoef[i] = ht.bsrc[i].coef;
    }
    for (size_t i = 0; bdest && i < ht.bdest.size(); ++i) bdest[2 * i] = ht.bdest[i].begin, bdest[2 * i + 1] = ht.bdest[i].count;
    for (size_t i = 0; i < ht.dest.size(); ++i) {
        if (dest_leaf) dest_leaf[i] = ht.dest[i].leaf;
        if (dest_coef) dest_coef[i] = ht.dest[i].coef;
    }
    return FASTMM_OK;
}

fastmm_status fastmm_scaling_exponents(fastmm_plan_t plan, const void *A, const void *B, int64_t m, int64_t k,
                                       int64_t n, int32_t *ea, int32_t *eb, int32_t *ep, void *workspace,
                                       size_t ws_bytes, void *stream) {
    if (check_plan(plan)) return FASTMM_EINVAL;
    if (m <= 0 || k <= 0 || n <= 0 || !A || !B || !ea || !eb || !ep) return fail(FASTMM_EINVAL, "bad arguments");
    if (plan->sc.mode == FASTMM_SCALE_NONE) return fail(FASTMM_EINVAL, "plan has no scaling");
    const Shape s = shape_of(plan, m, k, n);
    const WsLayout w = ws_layout(plan, s, m, k, n);
    if (workspace == nullptr || ws_bytes < w.total) return fail(FASTMM_EWORKSPACE, "workspace too small");
    if (((uintptr_t)workspace & 255) != 0) return fail(FASTMM_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    ScaleExps exps;
    fastmm_status stt = run_scaling(plan, A, k, 0, B, n, 0, m, k, n, (char *)workspace, w, st, &exps);
    if (stt != FASTMM_OK) return stt;
    hipError_t e;
    if ((e = hipMemcpyAsync(ea, exps.ea, 4 * (size_t)m, hipMemcpyDeviceToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(eb, exps.eb, 4 * (size_t)n, hipMemcpyDeviceToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(ep, exps.ep, 4 * (size_t)k, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return hip_fail(e, "copying exponents");
    return FASTMM_OK;
}

}  // extern "C"
