// Host-side tables (see tables.cpp).
#pragma once

#include <array>
#include <cstdint>
#include <utility>
#include <vector>

namespace sb {

struct Lam { int l[3]; };
struct QuadTermH { int ma, mb, mc; double c; };

struct Full4Plan {
    std::vector<Lam> out_lams;                    // output order (Alg. 6 loops, one parity)
    std::vector<Lam> canon;                       // computed orderings (la, lb, lc)
    std::vector<std::vector<QuadTermH>> terms;    // per canonical: (ma, mb, mc >= 0, weighted 3j)
    std::vector<int> out_canon;                   // per output Lambda: canonical index
    std::vector<std::array<int, 3>> out_pos;      // canonical position k <- output position out_pos[k]
    std::vector<int> out_sign;                    // odd parity: sign of that permutation (3j columns)
};

bool exact_floor_square(double e, int64_t *out);
double ylm_norm(int l, int m);
double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3);
std::vector<Lam> full4_lambdas(int lmax, bool even);
Full4Plan make_full4_plan(int lmax, int nbins, bool even = true, bool mfma = false);
std::vector<std::pair<int, int>> proj4_pairs(int mmax);

// Projected 4PCF symmetry (Alg. 8): the summand c^b1_m1 c^b2_m2 c^b3_m3, m3 = -(m1 + m2), is
// symmetric under permutations of the three (m, bin) slots and goes to its complex conjugate
// under m -> -m.  Every (m1, m2) maps to one canonical triple: the sorted (m1, m2, m3) or the
// sorted negated triple, whichever is lexicographically smaller (the un-negated one when they
// are equal).  Output bins (b1, b2, b3) read the canonical sums at position k <- b[pos[k]];
// neg: conjugate.
struct P4Canon {
    int m[3];
    int pos[3];
    bool neg;
};
P4Canon p4_canonical(int m1, int m2);

}  // namespace sb
