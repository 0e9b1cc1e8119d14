/*
 * fastmm.h -- C ABI of the MI355X (gfx950) fast matrix multiplication library.
 *
 * The library computes C = A B (A is m x k, B is k x n) by a recursive bilinear algorithm
 * <M0,K0,N0;R> given by coefficient matrices [U, V, W] (section 3.1, eq. (1)): at every
 * recursion level it forms S_r = sum_i U_ir A_i and T_r = sum_j V_jr B_j, multiplies the R
 * pairs recursively and accumulates C_k = sum_r W_kr M_r (section 3.2, eq. (2)); after L
 * levels the leaves use the classical algorithm.  Dimensions that are not multiples of
 * M0^L, K0^L, N0^L are zero-padded (section 3.2); padding is virtual (masked loads).
 * Optional diagonal scaling before the multiplication: outside scaling (Algorithm 1),
 * inside scaling (Algorithm 2) and repeated outside-inside scaling (Algorithm 3), with every
 * factor rounded to a power of two so that applying and removing it is exact (section 6).
 *
 * Conventions for every entry point:
 *  - Matrices are dense, row-major, in device memory (HBM of the current HIP device), with
 *    leading dimensions in elements.  The element type follows the plan's precision:
 *    FASTMM_F64 -> double; every other precision -> float (FP32 in and out).
 *  - The caller owns A, B, C and the workspace; the library never frees or retains them.
 *    The library owns plans and their device-side task tables (allocated once per plan and
 *    problem shape, released by fastmm_plan_destroy).
 *  - Calls are stream-ordered on `stream` (a hipStream_t; NULL = the default stream) and do
 *    not synchronise the device, except the first call of a plan at a new recursion depth
 *    on a device, which uploads that depth's task table (a blocking copy).
 *  - Argument errors are detected on the host before any launch; nothing is launched then.
 *    HIP errors map to FASTMM_EHIP.  fastmm_last_error() returns a message for the last
 *    failing call on the calling thread.  The library never aborts or exits.
 *  - Non-finite inputs are not errors; they propagate as IEEE arithmetic does.
 */
#ifndef FASTMM_H
#define FASTMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FASTMM_OK = 0,
    FASTMM_EINVAL = -1,      /* bad argument (null pointer, negative size, bad enum) */
    FASTMM_EBRENT = -2,      /* registered [U,V,W] fails the Brent equations */
    FASTMM_ESHAPE = -3,      /* inconsistent leading dimensions */
    FASTMM_ENOMEM = -4,      /* host or device allocation of plan tables failed */
    FASTMM_EHIP = -5,        /* a HIP runtime call or kernel launch failed */
    FASTMM_EUNSUPPORTED = -6,/* combination not implemented (message says which) */
    FASTMM_EALIAS = -7,      /* C overlaps A or B */
    FASTMM_EWORKSPACE = -8   /* workspace missing or smaller than fastmm_workspace_size */
} fastmm_status;

/* Built-in algorithms.  Coefficients follow the paper's appendices (Appendix A Strassen,
 * Appendix B <3,2,3;15>, Appendix C <4,4,2;26>) with rows relabelled to the stated index
 * convention (A and B blocks column-major, C blocks row-major; section 3.1), their cyclic
 * rotations (Appendices B and C), Winograd's variant of Strassen's algorithm and
 * Laderman's rank-23 <3,3,3> rule (literature; not printed in the paper). */
typedef enum {
    FASTMM_ALGO_CLASSICAL = 0, /* <1,1,1;1>: L levels of it are the classical algorithm */
    FASTMM_ALGO_STRASSEN = 1,  /* <2,2,2;7> */
    FASTMM_ALGO_WINOGRAD = 2,  /* <2,2,2;7>, Winograd's variant */
    FASTMM_ALGO_F323 = 3,      /* <3,2,3;15> */
    FASTMM_ALGO_F332 = 4,      /* <3,3,2;15> = [W,U,V] of <3,2,3> */
    FASTMM_ALGO_F233 = 5,      /* <2,3,3;15> = [V,W,U] of <3,2,3> */
    FASTMM_ALGO_F442 = 6,      /* <4,4,2;26> */
    FASTMM_ALGO_F424 = 7,      /* <4,2,4;26> = [V,W,U] of <4,4,2> */
    FASTMM_ALGO_F244 = 8,      /* <2,4,4;26> = [W,U,V] of <4,4,2> */
    FASTMM_ALGO_LADERMAN333 = 9,/* <3,3,3;23> */
    FASTMM_ALGO_USER0 = 64     /* first id handed out by fastmm_algo_register */
} fastmm_algo;

/* Scaling procedures of section 6.  Every factor is rounded to a power of two:
 * outside factors to the smallest power of two >= the row/column max-abs, inside factors
 * to 2^j with j the nearest integer to log2(max_j|B'_kj| / max_i|A'_ik|)/2 (ties to even).
 * All-zero rows/columns get factor 1. */
typedef enum {
    FASTMM_SCALE_NONE = 0,
    FASTMM_SCALE_OUTSIDE = 1,  /* Algorithm 1: one O step */
    FASTMM_SCALE_INSIDE = 2,   /* Algorithm 2: one I step */
    FASTMM_SCALE_OUT_IN = 3,   /* O step then I step */
    FASTMM_SCALE_IN_OUT = 4,   /* I step then O step */
    FASTMM_SCALE_REPEATED = 5  /* Algorithm 3: `steps` alternating steps starting with O */
} fastmm_scale_mode;

/* Arithmetic of the leaf products.  FP32 accumulation everywhere except FASTMM_F64. */
typedef enum {
    FASTMM_F64 = 0,    /* double in/out; v_mfma_f64_16x16x4f64 leaves */
    FASTMM_F32 = 1,    /* float in/out; v_mfma_f32_16x16x4f32 leaves */
    FASTMM_BF16 = 2,   /* float in/out; operands rounded to bf16 (1 product) */
    FASTMM_F16 = 3,    /* float in/out; operands rounded to fp16 (1 product) */
    FASTMM_BF16X3 = 4, /* float in/out; x = hi + lo in bf16, hi*hi + hi*lo + lo*hi */
    FASTMM_F16X3 = 5,  /* float in/out; x = hi + lo in fp16, hi*hi + hi*lo + lo*hi */
    FASTMM_BF16X6 = 6  /* float in/out; three bf16 limbs, the six products of order <= 2 */
} fastmm_precision;

typedef struct {
    int mode;   /* fastmm_scale_mode */
    int steps;  /* number of O/I steps for FASTMM_SCALE_REPEATED (>= 1) */
    double tau; /* > 0: stop early by the test of the stopping-criterion theorem (section
                   6.3), applied to every step after the first O step on the unrounded factors; evaluated on the device (the
                   remaining steps become no-ops), no host synchronisation; 0: run all steps */
    int per_level; /* 0: the steps run once, on A and B (section 6).  1: also on the operands
                   S_r, T_r of every inner node of the recursion (a reading of scaling "at
                   every level"; the paper scales once): the node scales its operands,
                   multiplies them by one level of eq. (2) whose children do the same, and
                   unscales its product.  Nodes on the last level are not scaled (power-of-two
                   factors commute exactly with the classical product), so plans of depth
                   <= 1 behave as with 0.  From depth 2 the first level's node operands and
                   products are written to the workspace (fastmm_workspace_size accounts for
                   them and for the nested products).  Stationary and uniform non-stationary
                   plans; not with fastmm_plan_set_tree or fastmm_gemm_batched
                   (FASTMM_EUNSUPPORTED). */
    int o_round;   /* fastmm_o_round: the power of two an O step (Algorithm 1) takes for a row
                   or column whose max-abs is x.  Section 6 rounds the factors to powers of
                   two (so that scaling is exact) without fixing which one:
                   FASTMM_O_ROUND_UP (0, default) the smallest power of two >= x (scaled
                   maxima in (1/2, 1]); FASTMM_O_ROUND_NEAREST (1) 2^j with j the integer
                   nearest to log2 x (scaled maxima in [2^-1/2, 2^1/2); never a tie).  The
                   nearer factor keeps rows whose maxima are alike on one factor, so the
                   cancelling cross-block terms of a fast rule are not amplified by the factor
                   ratio 2 when the product is unscaled (N(0,1) inputs: errors of unscaled
                   products instead of about twice those). */
} fastmm_scaling;

/* O-step factor rounding (fastmm_scaling.o_round). */
typedef enum { FASTMM_O_ROUND_UP = 0, FASTMM_O_ROUND_NEAREST = 1 } fastmm_o_round;

typedef struct fastmm_plan_s *fastmm_plan_t;

/* ---- algorithms ------------------------------------------------------------------- */

/* Register a user algorithm <M0,K0,N0;R>: num_U (M0K0 x R), num_V (K0N0 x R), num_W
 * (M0N0 x R), row-major int64 numerators over the common denominator 2^log2_den
 * (0 <= log2_den <= 30).  Index conventions of section 3.1.  The Brent equations are
 * checked exactly; FASTMM_EBRENT if they fail.  *algo_out receives the new id. */
fastmm_status fastmm_algo_register(int M0, int K0, int N0, int R, const int64_t *num_U,
                                   const int64_t *num_V, const int64_t *num_W, int log2_den,
                                   int *algo_out);

/* Dimensions and principal quantities (section 4.1: nnz, Q of Definition 4.1, E of
 * Definition 4.2) of an algorithm.  Any output pointer may be NULL. */
fastmm_status fastmm_algo_info(int algo, int *M0, int *K0, int *N0, int *R, int *nnz,
                               double *Q, double *E);

/* Section 5.3's per-rule figures (Table 1's stability exponent; Figure 2's axes) for `levels`
 * recursion levels: stab_exp = log_N0 E for a square <N0,N0,N0> rule and, for a rectangular
 * one, log_{M0 K0 N0} of the product of E over the rule and its two cyclic rotations (the
 * square rule that three levels of their cyclic use make); flops_frac = (R / (M0 K0 N0))^L, the
 * fraction of classical multiplications; rel_instability = (E / K0^2)^L, the factor by which
 * the leading term of Theorem 4.1 exceeds classical's.  Any output may be NULL.  Errors:
 * FASTMM_EINVAL (unknown id, negative levels), FASTMM_EUNSUPPORTED (a rotation failed). */
fastmm_status fastmm_algo_stability(int algo, int levels, double *stab_exp, double *flops_frac,
                                    double *rel_instability);

/* Copy the algorithm's coefficients as doubles into host arrays U (M0K0 x R), V (K0N0 x R),
 * W (M0N0 x R), row-major.  Any pointer may be NULL. */
fastmm_status fastmm_algo_coeffs(int algo, double *U, double *V, double *W);

/* ---- plans ------------------------------------------------------------------------ */

/* Create a plan: `depth` recursion levels of `algo` (fewer when a child dimension would
 * drop below `cutoff`: recursion continues while levels remain and ceil(dim / base^l) >=
 * cutoff for all three dimensions), the scaling procedure (NULL = none) and the leaf
 * precision.  depth >= 0, cutoff >= 1. */
fastmm_status fastmm_plan_create(fastmm_plan_t *out, int algo, int depth, int cutoff,
                                 const fastmm_scaling *scaling, int precision);

fastmm_status fastmm_plan_destroy(fastmm_plan_t plan);

/* Levels the plan uses for an m x k by k x n product, and the padded sizes. */
fastmm_status fastmm_plan_shape(fastmm_plan_t plan, int64_t m, int64_t k, int64_t n,
                                int *levels, int64_t *Mp, int64_t *Kp, int64_t *Np);

/* Execution paths of one product (fastmm_plan_path). */
typedef enum {
    FASTMM_PATH_LEAF = 0,  /* one launch over all leaf products M_r = S_r T_r (S and T formed
                              while loading, eq. (2)), then one W-combination launch */
    FASTMM_PATH_FUSED = 1, /* the innermost level fused: each work-group forms S_r, T_r, the R
                              products and the W-sums of eq. (1) for one tile of a node of the
                              recursion; from depth 2 the node operands of the outer L-1 levels
                              are written level by level first (with the scaling factors and
                              transposes applied), and their W-combination follows the kernel */
    FASTMM_PATH_EVERY_LEVEL = 2, /* scaling at every level (fastmm_scaling.per_level, depth >= 2):
                              the first level's node operands written out, each node product
                              by a call of the remaining levels, then the W-combination */
    FASTMM_PATH_FUSED_LOADS = 4, /* split precisions with FASTMM_FUSE_ALWAYS, 256 x 256 limb-GEMM
                              tiles, at most two limbs, every product live and at most two
                              nonzeros per column of U and V (Strassen's rule, classical): the
                              outer levels' node operands written out in FP32 level by level
                              (none at depth <= 1), the innermost level's S_r, T_r formed in the
                              limb GEMM's tile loads (no limb planes), then the W-combination */
    FASTMM_PATH_WRITTEN = 3 /* FP64 / FP32 from depth 1 where the fused path is not taken (one
                              rule at every level, every product live): every leaf operand S_r,
                              T_r written out level by level (eq. (2) applied once per level,
                              with the scaling factors and transposes at the first), one launch
                              over the written-out leaves with one source each, then the
                              W-combination */
} fastmm_path;

/* Fusion modes (fastmm_plan_set_fusion). */
typedef enum {
    FASTMM_FUSE_OFF = 0,    /* always the leaf path with composite source lists (neither the
                               fused kernels nor written-out leaf operands; split precisions
                               through limb planes) */
    FASTMM_FUSE_AUTO = 1,   /* the default: the fused path where it applies to an FP32 plan,
                               else written-out leaf operands where FASTMM_PATH_WRITTEN applies
                               (every FP64 plan with a level and one rule), else the leaf path */
    FASTMM_FUSE_ALWAYS = 2, /* the fused path wherever it applies; for the split precisions the
                               innermost level formed in the limb GEMM's loads
                               (FASTMM_PATH_FUSED_LOADS) where it applies */
    FASTMM_FUSE_WRITTEN = 3 /* FP64 / FP32: written-out leaf operands wherever FASTMM_PATH_WRITTEN
                               applies, never the fused kernel (the path every FP64 / FP32
                               product of a batched call takes); split precisions as AUTO */
} fastmm_fusion;

/* Set the fusion mode (fastmm_fusion) of this plan and of the rotated sub-plans of its backward
 * pass; FASTMM_EINVAL for an unknown mode.  The fused path applies to FP64 and FP32 plans with
 * at least one level, row-major (non-transposed) operands, and a <2,2,2;7> rule whose
 * coefficients are all 0 or +-1 and whose sign pattern has a compiled kernel (Strassen's rule,
 * Winograd's variant and their cyclic rotations).  Both paths compute the same result in exact
 * arithmetic; at depth 1 they round identically (bitwise equal results). */
fastmm_status fastmm_plan_set_fusion(fastmm_plan_t plan, int mode);

/* Output tile of the split-precision limb GEMM (a tuning choice, not part of the method): 0 =
 * chosen by the leaf-block shape (256 x 256 for blocks of at least 256 x 256 and at most two
 * limbs, else 128 x 128), or 128 / 256 forced.  256 needs at most two limbs
 * (FASTMM_EUNSUPPORTED otherwise); a nonzero tile on a plan that is not split precision is
 * FASTMM_EUNSUPPORTED; other values FASTMM_EINVAL.  In a batched call the problems share the
 * smallest tile among their plans.  The autotuner sets it per shape. */
fastmm_status fastmm_plan_set_tile(fastmm_plan_t plan, int tile);

/* Non-uniform recursion (section 3.4; the two non-uniform examples of section 5.2): gives every
 * internal node of the plan's recursion tree its own rule.  node_algos[i] is the rule id of
 * node i in breadth-first order: node [l, r_1 .. r_{l-1}] (level l, reached through the 0-based
 * products r_1 .. r_{l-1}) is entry (R^(l-1) - 1) / (R - 1) + (r_1 .. r_{l-1} read as a base-R
 * number), so count = 1 + R + ... + R^(depth-1).  Every rule must have the plan rule's
 * <M0,K0,N0;R> (for instance the permutation variants [U, (P x I) V, (I x P) W] of the
 * non-uniform Strassen example, registered with fastmm_algo_register) and every product live.
 * count = 0 restores the plan's rule at every node.  When the cutoff leaves fewer levels, the
 * tree's first levels apply.  Such plans take the leaf path (and the limb planes of the split
 * precisions), forward, batched and backward.  Must not be called while calls using the plan are in flight
 * (the plan's cached task tables are rebuilt).  Errors: FASTMM_EINVAL (null list, unknown
 * id), FASTMM_ESHAPE (wrong count, a rule of another shape), FASTMM_EUNSUPPORTED (a rule with
 * a product that never reaches C). */
fastmm_status fastmm_plan_set_tree(fastmm_plan_t plan, const int *node_algos, int64_t count);

/* Uniform non-stationary recursion (section 3.3, Theorem 4.2): level l (1-based) of the plan
 * uses rule level_algos[l-1] at every node; count must equal the plan's depth, and the rules
 * may have different base shapes <M0,K0,N0;R> (e.g. <3,2,3;15> above <2,2,2;7>; padding is to
 * multiples of the products of the levels' base sizes).  The cutoff stops the recursion as for
 * a stationary plan, keeping the first levels.  count = 0 restores the plan's rule at every
 * level; setting levels clears a tree (fastmm_plan_set_tree) and vice versa.  Such plans take
 * the leaf path (and the split precisions' two passes); the backward pass rotates every
 * level's rule.  Must not be called while calls using the plan are in flight.  Errors:
 * FASTMM_EINVAL (null list, unknown id, a 1x1x1 rule), FASTMM_ESHAPE (count != depth). */
fastmm_status fastmm_plan_set_levels(fastmm_plan_t plan, const int *level_algos, int count);

/* The path (fastmm_path) fastmm_gemm_ex takes for this shape and these transposition flags. */
fastmm_status fastmm_plan_path(fastmm_plan_t plan, int64_t m, int64_t k, int64_t n, int transA,
                               int transB, int *path);

/* Device workspace bytes fastmm_gemm needs for this shape (enough for either path). */
fastmm_status fastmm_workspace_size(fastmm_plan_t plan, int64_t m, int64_t k, int64_t n,
                                    size_t *bytes);

/* ---- multiplication ---------------------------------------------------------------- */

/* C = A B with contiguous row-major operands (lda = k, ldb = n, ldc = n).  m, k, n >= 0;
 * a zero m or n is a no-op, a zero k writes zeros.  `workspace` is device memory of at least
 * fastmm_workspace_size bytes (may be NULL when that size is 0).  C must not overlap A or B
 * (FASTMM_EALIAS).  `stream` is a hipStream_t (NULL = default stream). */
fastmm_status fastmm_gemm(fastmm_plan_t plan, const void *A, const void *B, void *C, int64_t m,
                          int64_t k, int64_t n, void *workspace, size_t ws_bytes, void *stream);

/* As fastmm_gemm with leading dimensions and transposition flags: op(A) is m x k and
 * op(B) is k x n, where op(X) = X^T when the flag is nonzero (X then stored k x m, resp.
 * n x k, row-major with its own leading dimension).  Used by the backward pass. */
fastmm_status fastmm_gemm_ex(fastmm_plan_t plan, const void *A, int64_t lda, int transA,
                             const void *B, int64_t ldb, int transB, void *C, int64_t ldc,
                             int64_t m, int64_t k, int64_t n, void *workspace, size_t ws_bytes,
                             void *stream);

/* Export the composite task table the plan uses at `levels` recursion levels (host memory,
 * for inspection and testing).  counts[0..4] receive the number of leaves, A-source
 * entries, B-source entries, output blocks and output contributions.  Arrays may be NULL
 * (call once with NULLs to size them):
 *   leaves  4 int32 per leaf: first A entry, A count, first B entry, B count;
 *   asrc    2 int32 per entry (block row, block column) with acoef its coefficient
 *           (the product over levels of U entries, eq. (ST_exact)); bsrc / bcoef likewise;
 *   bdest   2 int32 per output block (row-major over the M0^L x N0^L block grid): first
 *           contribution, count; dest_leaf / dest_coef: leaf index and product of W entries. */
fastmm_status fastmm_task_table(fastmm_plan_t plan, int levels, int64_t counts[5], int32_t *leaves,
                                int32_t *asrc, double *acoef, int32_t *bsrc, double *bcoef,
                                int32_t *bdest, int32_t *dest_leaf, double *dest_coef);

/* ---- batches ---------------------------------------------------------------------- */

/* One product of a batch: C = A B with contiguous row-major A (m x k), B (k x n), C (m x n). */
typedef struct {
    const void *A;
    const void *B;
    void *C;
    int64_t m, k, n;
} fastmm_problem;

/* Workspace bytes for fastmm_gemm_batched with these plans and problems. */
fastmm_status fastmm_batched_workspace_size(const fastmm_plan_t *plans, const fastmm_problem *probs,
                                            int count, size_t *bytes);

/* One product of a batch as fastmm_gemm_ex takes it: C = op(A) op(B) with op(A) m x k and
 * op(B) k x n, op(X) = X^T when the flag is nonzero (A then stored k x m, B n x k), row-major
 * storage with leading dimensions lda, ldb (at least the stored row length) and ldc >= n. */
typedef struct {
    const void *A;
    int64_t lda;
    int transA;
    const void *B;
    int64_t ldb;
    int transB;
    void *C;
    int64_t ldc;
    int64_t m, k, n;
} fastmm_problem_ex;

/* Multiply `count` independent problems, problem i with plans[i] (its own rule, depth,
 * cutoff and scaling; all plans must share one precision).  Each problem's scaling steps run
 * first (and, for the split precisions, its limb-plane formation); then ONE launch computes the
 * leaf tiles of all problems (work items ordered by problem, largest inner dimension first:
 * FP64/FP32 on persistent work-groups assigned round-robin, split precisions one work-group per
 * item with one limb-GEMM tile for the whole batch; deterministic either way), then the
 * W-combinations.  FP64/FP32 problems always take the leaf path (fastmm_plan_path).  Outputs
 * must not overlap any input.  The per-call descriptor table is copied from host memory into
 * the workspace (a staged copy). */
fastmm_status fastmm_gemm_batched(const fastmm_plan_t *plans, const fastmm_problem *probs, int count,
                                  void *workspace, size_t ws_bytes, void *stream);

/* fastmm_gemm_batched for strided and transposed operands (fastmm_problem_ex); the same single
 * launch of the products.  The split precisions form their limb planes from transposed
 * operands directly; FP64 / FP32 copy a transposed operand into the workspace first (the
 * batched leaf kernel reads row-major operands).  Same errors as fastmm_gemm_ex, per problem
 * (FASTMM_ESHAPE for a leading dimension below the stored row length), plus FASTMM_EALIAS when
 * an output overlaps any input or another output of the batch. */
fastmm_status fastmm_batched_ex_workspace_size(const fastmm_plan_t *plans, const fastmm_problem_ex *probs,
                                               int count, size_t *bytes);
fastmm_status fastmm_gemm_batched_ex(const fastmm_plan_t *plans, const fastmm_problem_ex *probs, int count,
                                     void *workspace, size_t ws_bytes, void *stream);

/* ---- a multiplication that allocates nothing ---------------------------------------- */

/* Bytes of the fixed scratch array behind fastmm_gemm_noalloc (256 MiB per GPU). */
#define FASTMM_NOALLOC_SCRATCH_BYTES (256ull << 20)

/* For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Computes exactly what fastmm_gemm computes (same
 * kernels, bitwise the same result), with the workspace taken from a fixed device array inside
 * the library instead of a caller's buffer: FASTMM_NOALLOC_SCRATCH_BYTES bytes on every GPU the
 * library runs on, held from its first use on that GPU until the process ends.  Operands as for
 * fastmm_gemm (contiguous row-major device arrays, C must not overlap A or B); `stream` is a
 * hipStream_t (NULL = default stream).
 * The call itself allocates nothing and creates no HIP objects; phase timing records nothing
 * for it.  Errors, detected before any launch:
 *   FASTMM_EWORKSPACE    the product needs more workspace (fastmm_workspace_size) than the array
 *                        holds; nothing is launched (call fastmm_gemm with a workspace instead);
 *   FASTMM_EUNSUPPORTED  the plan's task tables for this shape's recursion depth are not on
 *                        this device yet: a plan uploads them (an allocation) on its first
 *                        fastmm_gemm / fastmm_gemm_ex call at that depth on the device, so run
 *                        one such call with the plan and shape before using this entry point;
 *   otherwise as fastmm_gemm.
 * Every call on one GPU uses that GPU's one array, which keeps the last call's contents (each
 * call clears what it needs cleared): calls that overlap in time on one GPU (different streams
 * or threads without ordering between them) race on it and must not be issued. */
fastmm_status fastmm_gemm_noalloc(fastmm_plan_t plan, const void *A, const void *B, void *C, int64_t m,
                                  int64_t k, int64_t n, void *stream);

/* ---- differentiation ----------------------------------------------------------------- */

/* Gradients of a loss through C = A B: dA = G B^T and dB = A^T G for G = dLoss/dC (m x n),
 * computed by the same recursion with rules derived from the plan's rule by the symmetries of
 * section 3.1: dA = G B^T is a <M0,N0,K0> product, done by the transpose of the cyclic rotation
 * [V,W,U] (the rule that forms B G^T = dA^T); dB = A^T G is a <K0,M0,N0> product, done by the
 * transpose of [W,U,V] (which forms G^T A = dB^T).  Each product reads its transposed operand
 * (B^T, resp. A^T) through the transpose flags of fastmm_gemm_ex and writes its result in
 * place: nothing is transposed before or after.  Same depth, cutoff, scaling, precision and
 * fusion mode as the plan (for uniform non-stationary plans every level's rule is transformed
 * alike).  A (m x k), B (k x n), G (m x n) are contiguous row-major inputs; dA (m x k) and
 * dB (k x n) outputs, either may be NULL to skip it; with m = 0 (resp. n = 0) the requested
 * dB (dA) is filled with zeros.  Workspace: fastmm_backward_workspace_size bytes.  Plans with
 * a non-uniform tree (fastmm_plan_set_tree) transform every node's rule alike and run on the
 * leaf path. */
fastmm_status fastmm_backward_workspace_size(fastmm_plan_t plan, int64_t m, int64_t k, int64_t n,
                                             size_t *bytes);
fastmm_status fastmm_gemm_backward(fastmm_plan_t plan, const void *A, const void *B, const void *G,
                                   void *dA, void *dB, int64_t m, int64_t k, int64_t n,
                                   void *workspace, size_t ws_bytes, void *stream);

/* One problem of a batched backward pass: inputs A (m x k), B (k x n), G (m x n), outputs dA
 * (m x k) and dB (k x n), contiguous row-major; either output may be NULL. */
typedef struct {
    const void *A;
    const void *B;
    const void *G;
    void *dA;
    void *dB;
    int64_t m, k, n;
} fastmm_grad_problem;

/* The backward pass of a batch (section 3.1 symmetries as in fastmm_gemm_backward), problem i
 * with plans[i]: the 2 x count gradient products (dA_i = G_i B_i^T, dB_i = A_i^T G_i) run as ONE
 * fastmm_gemm_batched_ex call, so their leaf products share one launch.  All plans share one
 * precision.  Outputs must not overlap any input or each other (FASTMM_EALIAS). */
fastmm_status fastmm_backward_batched_workspace_size(const fastmm_plan_t *plans, const fastmm_grad_problem *probs,
                                                     int count, size_t *bytes);
fastmm_status fastmm_gemm_backward_batched(const fastmm_plan_t *plans, const fastmm_grad_problem *probs, int count,
                                           void *workspace, size_t ws_bytes, void *stream);

/* ---- scaling vectors (the reductions of Algorithms 1-3, exposed for verification) ---- */

/* Run the plan's scaling steps on A (m x k) and B (k x n) and write the power-of-two
 * exponents of the cumulative factors to device int32 arrays: ea (m) for D_A, eb (n) for
 * D_B, ep (k) for the product of the inside factors, so that the scaled operands are
 * A' = diag(2^-ea) A diag(2^ep) and B' = diag(2^-ep) B diag(2^-eb).  Needs the workspace of
 * fastmm_workspace_size. */
fastmm_status fastmm_scaling_exponents(fastmm_plan_t plan, const void *A, const void *B,
                                       int64_t m, int64_t k, int64_t n, int32_t *ea,
                                       int32_t *eb, int32_t *ep, void *workspace,
                                       size_t ws_bytes, void *stream);

/* ---- diagnostics ------------------------------------------------------------------- */

/* Phase timing for measurement: while enabled (nonzero), every fastmm_gemm / gemm_ex /
 * gemm_batched call on the calling thread records HIP events on its stream around its four
 * phases (scaling reductions; operand formation, i.e. the limb planes of the split precisions,
 * zero otherwise; the products kernel, for a batch its one launch with the descriptor upload;
 * the W-combination; a batch counts as one call; with scaling at every level the calls that
 * multiply the first level's node operands are the ones recorded, one each, and the first
 * level's own passes are not).  fastmm_profile_read synchronises on the
 * last recorded events and returns the summed milliseconds of each phase and the number of
 * calls since the last read (then resets).  Any output pointer may be NULL. */
fastmm_status fastmm_profile_enable(int enable);
fastmm_status fastmm_profile_read(double *ms_scaling, double *ms_form, double *ms_leaf, double *ms_combine,
                                  int *calls);

const char *fastmm_strerror(fastmm_status status);
const char *fastmm_last_error(void);
int fastmm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FASTMM_H */
