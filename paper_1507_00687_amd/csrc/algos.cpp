// Built-in bilinear rules, user registration, the Brent check and the principal quantities.
//
// Tables are the paper's printed matrices (Appendices A, B, C), relabelled here to the index
// convention of section 3.1 (single indices of A and B blocks column-major, of C blocks
// row-major):
//   * Strassen (Appendix A): rows 2 and 3 of U, V, W exchanged (the printed table is a valid
//     rule with A, B row-major and C column-major).
//   * <3,2,3;15> (Appendix B): used as printed.
//   * <4,4,2;26> (Appendix C): U as printed; V takes printed rows 1,5,2,6,3,7,4,8 and W takes
//     printed rows 1,3,5,7,2,4,6,8.
// Cyclic rotations give <3,3,2>, <2,3,3>, <4,2,4>, <2,4,4> (Appendices B and C: [W,U,V] of
// <M0,K0,N0> is <N0,M0,K0>).  Winograd's variant and Laderman's <3,3,3;23> come from the
// literature.  Every table is checked against the Brent equations when the registry is built.
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>

#include "fastmm_internal.h"

namespace fastmm {

double Algo::ldexp_i(int64_t num, int den) { return std::ldexp((double)num, -den); }

namespace {

static const int kStrassenU_printed[4][7] = {
    { 1,  0,  1,  0,  1, -1,  0},
    { 0,  0,  0,  0,  1,  0,  1},
    { 0,  1,  0,  0,  0,  1,  0},
    { 1,  1,  0,  1,  0,  0, -1},
};
static const int kStrassenV_printed[4][7] = {
    { 1,  1,  0, -1,  0,  1,  0},
    { 0,  0,  1,  0,  0,  1,  0},
    { 0,  0,  0,  1,  0,  0,  1},
    { 1,  0, -1,  0,  1,  0,  1},
};
static const int kStrassenW_printed[4][7] = {
    { 1,  0,  0,  1, -1,  0,  1},
    { 0,  1,  0,  1,  0,  0,  0},
    { 0,  0,  1,  0,  1,  0,  0},
    { 1, -1,  1,  0,  0,  1,  0},
};
static const int k323U[6][15] = {
    { 0,  1,  0,  0, -1,  1,  1,  0,  0,  0, -1,  0,  0,  0, -1},
    { 0,  1,  0,  0,  0,  0,  0, -1,  0, -1,  0,  0,  1, -1,  0},
    { 0,  0,  0,  1,  0,  0,  0, -1,  0, -1,  1,  0,  0, -1,  0},
    {-1,  0,  1,  0,  1,  0,  0,  0,  0,  0,  1,  0,  0,  0,  1},
    {-1,  0,  0,  0,  0,  1,  0,  1,  0,  1,  0,  1, -1,  0,  0},
    { 0,  0, -1,  0,  0,  0,  0,  1,  1,  0, -1,  0,  0,  0, -1},
};
static const int k323V[6][15] = {
    { 0,  0,  1,  1,  0,  0,  0,  0,  0,  0,  1,  0,  0,  1,  1},
    { 0,  0,  1,  0,  0,  0,  0, -1,  1, -1,  0,  0,  0,  1,  0},
    { 0, -1,  0,  0,  0,  1,  0,  0,  0,  1,  0,  1,  1, -1,  0},
    {-1,  0,  0,  0,  0,  0,  0,  1,  0,  1,  0,  1,  0, -1,  0},
    { 0,  1,  1,  0,  0,  0,  1,  0,  0,  0,  1,  0,  0,  0,  1},
    { 1,  0,  1,  0,  1,  1,  1,  0,  0,  0,  0,  0,  0,  0,  1},
};
static const int k323W[9][15] = {
    { 0,  0,  1,  0,  0,  0, -1,  0,  1,  0,  0,  0,  0,  0, -1},
    { 1,  0,  0,  0,  1,  1,  0,  0,  0,  0,  0, -1,  0,  0,  0},
    { 0,  0,  0,  0,  1,  0,  1,  0,  0,  0,  0,  0,  0,  0,  0},
    { 0,  0,  0, -1,  0,  0,  0,  0,  0, -1,  0,  1,  0, -1,  0},
    { 0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  1,  1,  0,  0},
    { 0,  1,  0,  0,  0,  1, -1,  0,  0,  0,  0,  0,  1,  0,  0},
    { 0,  0,  0,  1,  0,  0,  0,  0,  1,  0,  0,  0,  0,  0,  0},
    { 0,  0,  0,  0,  0,  0,  0,  1,  1, -1,  0,  0, -1,  0,  0},
    { 0,  0,  0, -1,  1,  0,  0,  0,  0,  0,  1,  0,  0,  0, -1},
};
static const int k442U2_printed[16][26] = {
    { 2,  0,  0, -2,  0,  0,  0,  0, -2,  0,  0,  0,  0, -2,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0},
    { 0,  0,  0,  0,  0, -2,  0,  0,  0,  0,  2,  2,  2,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0},
    { 0,  0,  2,  0,  0, -2,  0,  0,  0,  0,  2,  2,  2, -2,  0,  0,  0,  0,  0,  0, -2,  0,  0,  2,  0,  0},
    { 0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0, -2,  0,  2,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0},
    { 0,  2,  0,  0,  0,  0,  0,  1,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0, -1,  0,  0,  0,  0,  0,  0,  2},
    { 0,  2,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0, -2,  0,  0,  1,  0,  0,  0,  1,  0, -2,  0,  2, -2,  0},
    { 0,  2,  0,  0,  0,  0,  0,  1,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0, -1,  0,  0, -2,  0,  0,  0,  0},
    { 0,  0,  0,  1,  2,  0, -1, -1,  0, -1, -2,  2,  0, -2, -2,  0,  0,  1,  0,  0,  1,  0,  0,  0,  0,  0},
    { 0,  0,  0,  0,  0,  0,  0,  1,  0,  0,  0,  0,  0,  0,  0, -1,  1,  1,  0,  0,  0,  0,  0,  0,  0,  0},
    { 0,  2,  0,  0, -2,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  1,  0,  0,  0,  1,  0, -2,  2,  0,  2,  0},
    { 0,  2,  0,  0, -2,  0,  0,  1,  0,  0,  0,  0,  0,  0,  0,  0,  0,  1,  0,  0,  0, -2,  2,  0,  2,  0},
    { 0,  0,  0,  1,  0,  0, -1, -1,  0,  1,  0,  0,  0,  0,  0,  0,  0, -1,  0,  0, -1,  0,  0,  0,  0,  0},
    { 0, -2,  0,  0,  0,  0,  0,  0,  2,  0,  0,  0,  0,  0,  0,  1, -1, -1,  1,  0,  0,  0,  0,  0,  0, -2},
    { 0,  0,  0,  0,  2,  0,  0,  0,  0,  0,  0,  0,  2,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0},
    { 0,  0,  0,  0,  2,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0, -1,  1,  0,  0,  0,  0,  0, -2,  0},
    { 0,  0,  0,  0, -2,  0,  0,  0,  0,  0,  2,  0,  0,  2,  2,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0},
};
static const int k442V2_printed[8][26] = {
    { 2,  0, -2,  0,  0, -2,  0,  0,  0,  0, -2,  0,  0, -2, -2,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0},
    { 2,  1,  2,  2,  0,  0,  0,  2,  2,  0,  0,  0,  0,  0,  0,  0,  2, -2, -2,  2,  2,  0,  0, -2,  1,  0},
    {-2,  0, -2, -2,  0, -2, -2,  0,  0, -2,  0, -2,  0,  0,  0,  0,  0,  0,  0,  0, -2,  0,  0,  0,  0,  0},
    {-2,  0,  2, -2,  0,  0, -2,  0, -2,  2,  0,  0,  0,  0,  0, -2, -2,  0,  0,  2,  2,  0, -2, -2,  0,  0},
    { 2,  1, -2,  2,  0,  0,  0,  2,  2,  0,  0,  0,  0,  0,  0,  2,  0,  2,  2,  0, -2,  0,  0,  2, -1,  2},
    { 2,  1, -2,  2,  0,  2,  0,  2,  2,  0,  2,  0, -2,  0,  2,  2,  0,  2, -2,  0, -2,  0,  0,  2, -1,  0},
    {-2, -2, -2, -2,  0,  0, -2,  0, -2, -2,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0, -2,  2,  2,  2,  0, -2},
    {-2,  0, -2, -2, -2,  2, -2,  0, -2, -2,  2,  0, -2,  0,  0,  0,  0,  0,  0,  0, -2,  0, -2,  2, -2,  0},
};
static const int k442W_printed[8][26] = {
    { 1, -1,  0,  1,  0,  0,  1,  1,  0,  0,  0,  0,  0,  0,  0,  1,  1,  0,  0,  1,  0,  1,  0,  0,  0,  1},
    { 0,  1, -1,  0,  0,  0,  0,  0,  0, -1,  0,  0,  0,  0,  0, -1, -1, -1, -1, -1, -1, -1,  0,  0,  0, -1},
    { 0, -1,  0,  1,  0,  0,  1,  1, -1,  0,  0,  0,  0,  0,  0,  1, -1,  0,  0,  1,  0,  1,  0,  0,  0,  0},
    { 0,  0,  0,  0,  0,  0,  0,  0,  0,  1,  0,  0,  0,  0,  0,  1,  1,  1,  0, -1,  1, -1, -1, -1,  1,  0},
    { 0,  0,  1,  0,  1,  0,  0,  0,  0,  1, -1,  0, -1,  0,  1,  1,  1,  1,  0,  1,  1,  0,  0,  0,  1,  0},
    { 1,  0, -1,  1,  0,  0,  1,  0,  0, -1,  0,  0,  0, -1,  1,  0,  0,  0,  0,  0, -1,  0,  0,  0,  0,  0},
    { 0,  0,  0,  0, -1,  1,  0,  0,  0, -1,  1,  0,  0,  0, -1, -1, -1, -1,  0,  1, -1,  0,  0,  1, -1,  0},
    { 0,  0,  0,  0,  0,  1,  1,  0,  0,  1,  1,  1,  0,  0, -1,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0,  0},
};

template <int ROWS, int COLS>
std::vector<int64_t> rows_of(const int (&t)[ROWS][COLS], const std::vector<int> &order1) {
    // order1: 1-based printed row for each output row (empty = printed order).
    std::vector<int64_t> out;
    out.reserve(ROWS * COLS);
    for (int i = 0; i < ROWS; ++i) {
        const int src = order1.empty() ? i : order1[i] - 1;
        for (int c = 0; c < COLS; ++c) out.push_back(t[src][c]);
    }
    return out;
}

Algo make_classical111() {
    Algo a;
    a.name = "classical";
    a.M0 = a.K0 = a.N0 = a.R = 1;
    a.U = {1};
    a.V = {1};
    a.W = {1};
    return a;
}

Algo make_strassen() {
    Algo a;
    a.name = "strassen";
    a.M0 = a.K0 = a.N0 = 2;
    a.R = 7;
    const std::vector<int> swap23 = {1, 3, 2, 4};
    a.U = rows_of(kStrassenU_printed, swap23);
    a.V = rows_of(kStrassenV_printed, swap23);
    a.W = rows_of(kStrassenW_printed, swap23);
    return a;
}

Algo make_323() {
    Algo a;
    a.name = "f323";
    a.M0 = 3, a.K0 = 2, a.N0 = 3, a.R = 15;
    a.U = rows_of(k323U, {});
    a.V = rows_of(k323V, {});
    a.W = rows_of(k323W, {});
    return a;
}

Algo make_442() {
    Algo a;
    a.name = "f442";
    a.M0 = 4, a.K0 = 4, a.N0 = 2, a.R = 26;
    a.U = rows_of(k442U2_printed, {});
    a.V = rows_of(k442V2_printed, {1, 5, 2, 6, 3, 7, 4, 8});
    a.W = rows_of(k442W_printed, {1, 3, 5, 7, 2, 4, 6, 8});
    a.den_U = 1;  // printed as (1/2) * integers
    a.den_V = 1;
    return a;
}

// [U,V,W] for <M0,K0,N0>  ->  [W,U,V] for <N0,M0,K0>.
Algo rotate(const Algo &a, const char *name) {
    Algo b;
    b.name = name;
    b.M0 = a.N0, b.K0 = a.M0, b.N0 = a.K0, b.R = a.R;
    b.U = a.W, b.den_U = a.den_W;
    b.V = a.U, b.den_V = a.den_U;
    b.W = a.V, b.den_W = a.den_V;
    return b;
}

// The transposed rule: applied to (B^T, A^T) it forms (C)^T, so it is a rule for <N0,K0,M0>.
// Under the single-index conventions (A and B blocks column-major, C blocks row-major) its
// product r takes as left operand the transposes of the B blocks that product r of `a` takes,
// as right operand the transposes of a's A blocks, and contributes to the transposed C blocks:
// S'_r = T_r^T, T'_r = S_r^T, M'_r = M_r^T (section 3.1 notation).
Algo transpose_rule(const Algo &a, const char *name) {
    Algo t;
    t.name = name;
    t.M0 = a.N0, t.K0 = a.K0, t.N0 = a.M0, t.R = a.R;
    const int R = a.R;
    t.U.assign((size_t)a.N0 * a.K0 * R, 0);
    t.V.assign((size_t)a.K0 * a.M0 * R, 0);
    t.W.assign((size_t)a.N0 * a.M0 * R, 0);
    t.den_U = a.den_V, t.den_V = a.den_U, t.den_W = a.den_W;
    for (int r = 0; r < R; ++r) {
        for (int p = 0; p < a.N0; ++p)  // A' = B^T: block (p, q) is B's block (q, p) transposed
            for (int q = 0; q < a.K0; ++q) t.U[(size_t)(p + q * a.N0) * R + r] = a.V[(size_t)(q + p * a.K0) * R + r];
        for (int q = 0; q < a.K0; ++q)  // B' = A^T: block (q, s) is A's block (s, q) transposed
            for (int s = 0; s < a.M0; ++s) t.V[(size_t)(q + s * a.K0) * R + r] = a.U[(size_t)(s + q * a.M0) * R + r];
        for (int p = 0; p < a.N0; ++p)  // C' = C^T, row-major blocks
            for (int s = 0; s < a.M0; ++s) t.W[(size_t)(p * a.M0 + s) * R + r] = a.W[(size_t)(s * a.N0 + p) * R + r];
    }
    return t;
}

// Rules written as products of sums of named entries.  An entry "xPQ" is row P, column Q
// (1-based) of the A or B base matrix; outputs "cPQ" list (product number, sign).
struct Term {
    int p, q, c;
};
struct Product {
    std::vector<Term> a, b;
};

Algo from_products(const char *name, int M0, int K0, int N0, const std::vector<Product> &prods,
                   const std::vector<std::vector<Term>> &outs /* per C entry row-major: p=product */) {
    Algo al;
    al.name = name;
    al.M0 = M0, al.K0 = K0, al.N0 = N0;
    al.R = (int)prods.size();
    al.U.assign((size_t)M0 * K0 * al.R, 0);
    al.V.assign((size_t)K0 * N0 * al.R, 0);
    al.W.assign((size_t)M0 * N0 * al.R, 0);
    for (int r = 0; r < al.R; ++r) {
        for (const Term &t : prods[r].a) al.U[(size_t)((t.p - 1) + (t.q - 1) * M0) * al.R + r] += t.c;
        for (const Term &t : prods[r].b) al.V[(size_t)((t.p - 1) + (t.q - 1) * K0) * al.R + r] += t.c;
    }
    for (int k = 0; k < M0 * N0; ++k)
        for (const Term &t : outs[k]) al.W[(size_t)k * al.R + (t.p - 1)] += t.c;
    return al;
}

Algo make_winograd() {
    // s1 = a21+a22, s2 = s1-a11, s3 = a11-a21, s4 = a12-s2; t1 = b12-b11, t2 = b22-t1,
    // t3 = b22-b12, t4 = t2-b21; products a11 b11, a12 b21, s4 b22, a22 t4, s1 t1, s2 t2,
    // s3 t3; c11 = p1+p2, c12 = p1+p6+p5+p3, c21 = p1+p6+p7-p4, c22 = p1+p6+p7+p5.
    std::vector<Product> P = {
        {{{1, 1, 1}}, {{1, 1, 1}}},
        {{{1, 2, 1}}, {{2, 1, 1}}},
        {{{1, 1, 1}, {1, 2, 1}, {2, 1, -1}, {2, 2, -1}}, {{2, 2, 1}}},
        {{{2, 2, 1}}, {{1, 1, 1}, {1, 2, -1}, {2, 1, -1}, {2, 2, 1}}},
        {{{2, 1, 1}, {2, 2, 1}}, {{1, 2, 1}, {1, 1, -1}}},
        {{{2, 1, 1}, {2, 2, 1}, {1, 1, -1}}, {{2, 2, 1}, {1, 2, -1}, {1, 1, 1}}},
        {{{1, 1, 1}, {2, 1, -1}}, {{2, 2, 1}, {1, 2, -1}}},
    };
    std::vector<std::vector<Term>> out = {
        {{1, 0, 1}, {2, 0, 1}},
        {{1, 0, 1}, {6, 0, 1}, {5, 0, 1}, {3, 0, 1}},
        {{1, 0, 1}, {6, 0, 1}, {7, 0, 1}, {4, 0, -1}},
        {{1, 0, 1}, {6, 0, 1}, {7, 0, 1}, {5, 0, 1}},
    };
    return from_products("winograd", 2, 2, 2, P, out);
}

Algo make_laderman() {
    std::vector<Product> P = {
        {{{1, 1, 1}, {1, 2, 1}, {1, 3, 1}, {2, 1, -1}, {2, 2, -1}, {3, 2, -1}, {3, 3, -1}}, {{2, 2, 1}}},
        {{{1, 1, 1}, {2, 1, -1}}, {{1, 2, -1}, {2, 2, 1}}},
        {{{2, 2, 1}}, {{1, 1, -1}, {1, 2, 1}, {2, 1, 1}, {2, 2, -1}, {2, 3, -1}, {3, 1, -1}, {3, 3, 1}}},
        {{{1, 1, -1}, {2, 1, 1}, {2, 2, 1}}, {{1, 1, 1}, {1, 2, -1}, {2, 2, 1}}},
        {{{2, 1, 1}, {2, 2, 1}}, {{1, 1, -1}, {1, 2, 1}}},
        {{{1, 1, 1}}, {{1, 1, 1}}},
        {{{1, 1, -1}, {3, 1, 1}, {3, 2, 1}}, {{1, 1, 1}, {1, 3, -1}, {2, 3, 1}}},
        {{{1, 1, -1}, {3, 1, 1}}, {{1, 3, 1}, {2, 3, -1}}},
        {{{3, 1, 1}, {3, 2, 1}}, {{1, 1, -1}, {1, 3, 1}}},
        {{{1, 1, 1}, {1, 2, 1}, {1, 3, 1}, {2, 2, -1}, {2, 3, -1}, {3, 1, -1}, {3, 2, -1}}, {{2, 3, 1}}},
        {{{3, 2, 1}}, {{1, 1, -1}, {1, 3, 1}, {2, 1, 1}, {2, 2, -1}, {2, 3, -1}, {3, 1, -1}, {3, 2, 1}}},
        {{{1, 3, -1}, {3, 2, 1}, {3, 3, 1}}, {{2, 2, 1}, {3, 1, 1}, {3, 2, -1}}},
        {{{1, 3, 1}, {3, 3, -1}}, {{2, 2, 1}, {3, 2, -1}}},
        {{{1, 3, 1}}, {{3, 1, 1}}},
        {{{3, 2, 1}, {3, 3, 1}}, {{3, 1, -1}, {3, 2, 1}}},
        {{{1, 3, -1}, {2, 2, 1}, {2, 3, 1}}, {{2, 3, 1}, {3, 1, 1}, {3, 3, -1}}},
        {{{1, 3, 1}, {2, 3, -1}}, {{2, 3, 1}, {3, 3, -1}}},
        {{{2, 2, 1}, {2, 3, 1}}, {{3, 1, -1}, {3, 3, 1}}},
        {{{1, 2, 1}}, {{2, 1, 1}}},
        {{{2, 3, 1}}, {{3, 2, 1}}},
        {{{2, 1, 1}}, {{1, 3, 1}}},
        {{{3, 1, 1}}, {{1, 2, 1}}},
        {{{3, 3, 1}}, {{3, 3, 1}}},
    };
    auto plus = [](std::initializer_list<int> ps) {
        std::vector<Term> t;
        for (int p : ps) t.push_back({p, 0, 1});
        return t;
    };
    std::vector<std::vector<Term>> out = {
        plus({6, 14, 19}),
        plus({1, 4, 5, 6, 12, 14, 15}),
        plus({6, 7, 9, 10, 14, 16, 18}),
        plus({2, 3, 4, 6, 14, 16, 17}),
        plus({2, 4, 5, 6, 20}),
        plus({14, 16, 17, 18, 21}),
        plus({6, 7, 8, 11, 12, 13, 14}),
        plus({12, 13, 14, 15, 22}),
        plus({6, 7, 8, 9, 23}),
    };
    return from_products("laderman333", 3, 3, 3, P, out);
}

struct Registry {
    std::mutex mu;
    std::vector<Algo> builtin;  // index = fastmm_algo id
    std::vector<Algo> user;     // id = FASTMM_ALGO_USER0 + index
    std::map<std::pair<int, int>, int> rotations;  // (id, times) -> id of the rotated rule
    std::map<std::pair<int, int>, int> transposed;  // (id, times) -> id of the transposed rotation
    bool ok = false;
    Registry() {
        builtin.resize(10);
        builtin[FASTMM_ALGO_CLASSICAL] = make_classical111();
        builtin[FASTMM_ALGO_STRASSEN] = make_strassen();
        builtin[FASTMM_ALGO_WINOGRAD] = make_winograd();
        builtin[FASTMM_ALGO_F323] = make_323();
        builtin[FASTMM_ALGO_F332] = rotate(builtin[FASTMM_ALGO_F323], "f332");
        builtin[FASTMM_ALGO_F233] = rotate(builtin[FASTMM_ALGO_F332], "f233");
        builtin[FASTMM_ALGO_F442] = make_442();
        builtin[FASTMM_ALGO_F244] = rotate(builtin[FASTMM_ALGO_F442], "f244");
        builtin[FASTMM_ALGO_F424] = rotate(builtin[FASTMM_ALGO_F244], "f424");
        builtin[FASTMM_ALGO_LADERMAN333] = make_laderman();
        ok = true;
        for (const Algo &a : builtin) ok = ok && brent_violations(a) == 0;
    }
};

Registry &registry() {
    static Registry r;
    return r;
}

}  // namespace

long brent_violations(const Algo &a) {
    const int M0 = a.M0, K0 = a.K0, N0 = a.N0, R = a.R;
    const int dsum = a.den_U + a.den_V + a.den_W;
    long bad = 0;
    for (int p = 0; p < M0; ++p)
        for (int q = 0; q < K0; ++q)
            for (int q2 = 0; q2 < K0; ++q2)
                for (int s = 0; s < N0; ++s)
                    for (int p2 = 0; p2 < M0; ++p2)
                        for (int s2 = 0; s2 < N0; ++s2) {
                            const int ia = p + q * M0, ib = q2 + s * K0, ic = p2 * N0 + s2;
                            __int128 t = 0;
                            for (int r = 0; r < R; ++r)
                                t += (__int128)a.U[(size_t)ia * R + r] * a.V[(size_t)ib * R + r] *
                                     a.W[(size_t)ic * R + r];
                            const __int128 want =
                                (p == p2 && q == q2 && s == s2) ? ((__int128)1 << dsum) : 0;
                            if (t != want) ++bad;
                        }
    return bad;
}

Quantities quantities(const Algo &a) {
    const int R = a.R;
    std::vector<int> alpha(R, 0), beta(R, 0);
    std::vector<double> av(R, 0.0), bv(R, 0.0);
    int nnz = 0;
    for (int r = 0; r < R; ++r) {
        for (int i = 0; i < a.M0 * a.K0; ++i)
            if (a.U[(size_t)i * R + r]) ++alpha[r], av[r] += std::fabs(a.u(i, r));
        for (int j = 0; j < a.K0 * a.N0; ++j)
            if (a.V[(size_t)j * R + r]) ++beta[r], bv[r] += std::fabs(a.v(j, r));
        nnz += alpha[r] + beta[r];
    }
    double Q = 0, E = 0;
    for (int k = 0; k < a.M0 * a.N0; ++k) {
        int gamma = 0, mx = 0;
        double e = 0;
        for (int r = 0; r < R; ++r)
            if (a.W[(size_t)k * R + r]) {
                ++gamma;
                mx = std::max(mx, alpha[r] + beta[r]);
                e += av[r] * bv[r] * std::fabs(a.w(k, r));
            }
        nnz += gamma;
        Q = std::max(Q, (double)(gamma + mx));
        E = std::max(E, e);
    }
    return {nnz, Q, E};
}

const Algo *algo_get(int id) {
    Registry &reg = registry();
    if (!reg.ok) return nullptr;
    std::lock_guard<std::mutex> g(reg.mu);
    if (id >= 0 && id < (int)reg.builtin.size()) return &reg.builtin[id];
    if (id >= FASTMM_ALGO_USER0 && id - FASTMM_ALGO_USER0 < (int)reg.user.size())
        return &reg.user[id - FASTMM_ALGO_USER0];
    return nullptr;
}

namespace {
int register_locked(Registry &reg, Algo &&a) {
    reg.user.reserve(256);  // keep pointers handed out by algo_get stable
    if (reg.user.size() >= 256) return -1;
    reg.user.push_back(std::move(a));
    return FASTMM_ALGO_USER0 + (int)reg.user.size() - 1;
}
}  // namespace

int algo_register(Algo &&a) {
    Registry &reg = registry();
    std::lock_guard<std::mutex> g(reg.mu);
    return register_locked(reg, std::move(a));
}

int algo_rotated(int id, int times) {
    times = ((times % 3) + 3) % 3;
    if (times == 0) return id;
    const Algo *a = algo_get(id);
    if (!a) return -1;
    Registry &reg = registry();
    std::lock_guard<std::mutex> g(reg.mu);
    auto it = reg.rotations.find({id, times});
    if (it != reg.rotations.end()) return it->second;
    Algo r = rotate(*a, "rotation");
    if (times == 2) r = rotate(r, "rotation");
    if (brent_violations(r) != 0) return -1;
    const int nid = register_locked(reg, std::move(r));
    if (nid >= 0) reg.rotations[{id, times}] = nid;
    return nid;
}

int algo_transposed_rotation(int id, int times) {
    times = ((times % 3) + 3) % 3;
    const Algo *a = algo_get(id);
    if (!a) return -1;
    Registry &reg = registry();
    std::lock_guard<std::mutex> g(reg.mu);
    auto it = reg.transposed.find({id, times});
    if (it != reg.transposed.end()) return it->second;
    Algo r = *a;
    for (int t = 0; t < times; ++t) r = rotate(r, "rotation");
    r = transpose_rule(r, "transposed rotation");
    if (brent_violations(r) != 0) return -1;
    const int nid = register_locked(reg, std::move(r));
    if (nid >= 0) reg.transposed[{id, times}] = nid;
    return nid;
}

}  // namespace fastmm
