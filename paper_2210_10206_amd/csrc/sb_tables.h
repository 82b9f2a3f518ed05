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
Full4Plan make_full4_plan(int lmax, int nbins, bool even = true);
std::vector<std::pair<int, int>> proj4_pairs(int mmax);

}  // namespace sb
