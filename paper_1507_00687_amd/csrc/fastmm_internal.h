// Internal declarations shared by the host-side translation units of the library.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "fastmm.h"

namespace fastmm {

// A bilinear rule <M0,K0,N0;R> (section 3.1) with exact dyadic coefficients: entry x of U is
// num_U[x] / 2^den_U, likewise V and W.  Row-major (rows = single block index, cols = r).
struct Algo {
    std::string name;
    int M0 = 0, K0 = 0, N0 = 0, R = 0;
    std::vector<int64_t> U, V, W;
    int den_U = 0, den_V = 0, den_W = 0;

    double u(int i, int r) const { return ldexp_i(U[(size_t)i * R + r], den_U); }
    double v(int j, int r) const { return ldexp_i(V[(size_t)j * R + r], den_V); }
    double w(int k, int r) const { return ldexp_i(W[(size_t)k * R + r], den_W); }
    static double ldexp_i(int64_t num, int den);
};

// Registry access; returns nullptr for an unknown id.
const Algo *algo_get(int id);
int algo_register(Algo &&a);  // returns the new id
// Id of the cyclic rotation of rule `id` applied `times` times: once gives [W,U,V] (a rule for
// <N0,M0,K0>), twice [V,W,U] (<K0,N0,M0>).  Registered on first use; -1 on failure.
int algo_rotated(int id, int times);
// Id of the transpose of that rotation: times = 2 gives a rule for <M0,N0,K0> that forms
// G B^T (the transpose of [V,W,U] applied to (B, G^T)), times = 1 a rule for <K0,M0,N0> that
// forms A^T G (the transpose of [W,U,V] applied to (G^T, A)).  Registered on first use; -1 on
// failure.
int algo_transposed_rotation(int id, int times);
// Number of (a, b, c) index triples violating the Brent equations under the convention
// A, B column-major and C row-major (exact integer arithmetic).
long brent_violations(const Algo &a);
struct Quantities {
    int nnz;
    double Q, E;
};
Quantities quantities(const Algo &a);

// Per-thread error message for fastmm_last_error().
void set_error(const std::string &msg);

// While set on the calling thread, the library allocates no device memory and creates no HIP
// objects: a call that would upload a plan's task tables (its first call at a recursion depth
// on a device) fails with FASTMM_EUNSUPPORTED instead, and phase timing records nothing.
void set_no_alloc(bool on);
bool no_alloc();

}  // namespace fastmm
