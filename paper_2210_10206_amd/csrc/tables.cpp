// Host tables of the library: exact bin thresholds, Y_lm normalisation, Wigner 3j
// symbols, the canonical Lambda list of the full 4PCF and the (m1, m2) pair list of the
// projected 4PCF.
#include "sb_tables.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace sb {

// floor(e^2) exactly: e = M 2^E with an integer 53-bit mantissa M, e^2 = M^2 2^(2E).
bool exact_floor_square(double e, int64_t *out) {
    if (!(e >= 0.0) || !std::isfinite(e)) return false;
    if (e == 0.0) { *out = 0; return true; }
    int ex = 0;
    const double mant = std::frexp(e, &ex);                 // e = mant 2^ex, mant in [0.5, 1)
    const uint64_t M = (uint64_t)std::ldexp(mant, 53);       // exact
    const int E = ex - 53;
    const unsigned __int128 M2 = (unsigned __int128)M * M;   // < 2^106
    unsigned __int128 f;
    if (2 * E >= 0) {
        if (2 * E > 20) return false;                        // e^2 beyond any supported grid
        f = M2 << (2 * E);
    } else {
        const int sh = -2 * E;
        f = sh >= 128 ? 0 : (M2 >> sh);
    }
    if (f > (unsigned __int128)INT64_MAX) return false;
    *out = (int64_t)f;
    return true;
}

double ylm_norm(int l, int m) {
    // sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
    double r = 1.0;
    for (int k = l - m + 1; k <= l + m; ++k) r /= (double)k;
    return std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * r);
}

// Racah's closed form, evaluated in long double.
double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3) {
    if (m1 + m2 + m3 != 0) return 0.0;
    if (j3 < std::abs(j1 - j2) || j3 > j1 + j2) return 0.0;
    if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(m3) > j3) return 0.0;
    auto fact = [](int n) {
        long double r = 1.0L;
        for (int k = 2; k <= n; ++k) r *= (long double)k;
        return r;
    };
    const long double tri = fact(j1 + j2 - j3) * fact(j1 - j2 + j3) * fact(-j1 + j2 + j3) / fact(j1 + j2 + j3 + 1);
    const long double pre = std::sqrt(tri * fact(j1 + m1) * fact(j1 - m1) * fact(j2 + m2) * fact(j2 - m2) *
                                      fact(j3 + m3) * fact(j3 - m3));
    const int kmin = std::max({0, j2 - j3 - m1, j1 - j3 + m2});
    const int kmax = std::min({j1 + j2 - j3, j1 - m1, j2 + m2});
    long double s = 0.0L;
    for (int k = kmin; k <= kmax; ++k) {
        const long double den = fact(k) * fact(j3 - j2 + k + m1) * fact(j3 - j1 + k - m2) * fact(j1 + j2 - j3 - k) *
                                fact(j1 - k - m1) * fact(j2 - k + m2);
        s += ((k & 1) ? -1.0L : 1.0L) / den;
    }
    const int ph = j1 - j2 - m3;
    const long double sign = (ph % 2 != 0) ? -1.0L : 1.0L;
    return (double)(sign * pre * s);
}

// Lambda list in the loop order of Alg. 6 (l1, l2 over 0..lmax, l3 from |l1-l2| to min(l1+l2, lmax)).
std::vector<Lam> full4_lambdas(int lmax, bool even) {
    std::vector<Lam> out;
    for (int l1 = 0; l1 <= lmax; ++l1)
        for (int l2 = 0; l2 <= lmax; ++l2)
            for (int l3 = std::abs(l1 - l2); l3 <= std::min(l1 + l2, lmax); ++l3) {
                const bool odd = ((l1 + l2 + l3) & 1) != 0;
                if (odd == even) continue;
                out.push_back({l1, l2, l3});
            }
    return out;
}

// Terms of one ordering (la, lb, lc) with mc >= 0: (ma, mb = -ma - mc, mc, weight * 3j).
static void terms_of(int la, int lb, int lc, std::vector<QuadTermH> *t) {
    for (int mc = 0; mc <= lc; ++mc)
        for (int ma = -la; ma <= la; ++ma) {
            const int mb = -ma - mc;
            if (std::abs(mb) > lb) continue;
            // zero symbols are kept: the matrix-core kernels walk the same (mc, ma) order at
            // compile time and index this table by position
            const double w = wigner3j(la, lb, lc, ma, mb, mc);
            t->push_back({ma, mb, mc, (mc == 0 ? 1.0 : 2.0) * w});
        }
}

// Odd Lambda: permuting the 3j columns multiplies the symbol by (-1)^(l1+l2+l3) for each
// transposition, so an output Lambda is its canonical ordering's sums times the sign of the
// permutation; the product of the three coefficients is symmetric.
// Issue cycles per 4-cell step of the matrix-core kernel for the ordering (la, lb, lc): the
// vector coupling (2 multiplies + 4 FMAs per M tile for a general term, less where an m is 0,
// the mc = 0 pairing, the weighting of the b1 operands) and the 16x16x4 MFMAs (32 cycles,
// 2 per mc > 0 and M tile); la == lb computes 3 M tiles instead of 4 (pairs b1 <= b2).
static double mfma_cost(int la, int lb, int lc, const std::vector<QuadTermH> &t, bool even) {
    const int nmt = la == lb ? 3 : 4;
    double valu = 2.0 * nmt * (la + 1);
    for (const QuadTermH &q : t) {
        if (q.mc == 0) {
            if (q.ma < 0 || (!even && q.ma == 0)) continue;
            valu += q.ma == 0 ? 1 + nmt : 2 + 2 * nmt;
        } else {
            valu += (q.ma == 0 || q.mb == 0) ? 2 + 2 * nmt : 2 + 4 * nmt;
        }
    }
    const double mfma = nmt * (2.0 * lc + 1.0);
    return std::max(4.0 * valu, 32.0 * mfma) + 0.01 * (4.0 * valu + 32.0 * mfma);
}

Full4Plan make_full4_plan(int lmax, int nbins, bool even, bool mfma) {
    Full4Plan p;
    p.out_lams = full4_lambdas(lmax, even);
    // canonical = sorted triples; pick the cheapest ordering: fewest flops per cell for the
    // vector kernel, fewest issue cycles (mfma_cost) for the matrix-core kernels
    std::vector<Lam> sorted;
    for (const Lam &L : p.out_lams) {
        Lam s = L;
        std::sort(s.l, s.l + 3);
        bool seen = false;
        for (const Lam &q : sorted) seen |= (q.l[0] == s.l[0] && q.l[1] == s.l[1] && q.l[2] == s.l[2]);
        if (!seen) sorted.push_back(s);
    }
    const double nb2 = (double)nbins * nbins, nb3 = nb2 * nbins;
    for (const Lam &s : sorted) {
        int perm[3] = {0, 1, 2};
        double best = 1e300;
        Lam bestL = s;
        std::vector<QuadTermH> bestT;
        do {
            const int la = s.l[perm[0]], lb = s.l[perm[1]], lc = s.l[perm[2]];
            std::vector<QuadTermH> t;
            terms_of(la, lb, lc, &t);
            const double cost = mfma ? mfma_cost(la, lb, lc, t, even)
                                     : (double)t.size() * nb2 * 8.0 + (double)(lc + 1) * nb3 * 4.0;
            if (cost < best) { best = cost; bestL = {la, lb, lc}; bestT = t; }
        } while (std::next_permutation(perm, perm + 3));
        p.canon.push_back(bestL);
        p.terms.push_back(bestT);
    }
    // each output Lambda: its canonical index and position map
    for (const Lam &L : p.out_lams) {
        int found = -1, pos[3] = {0, 1, 2};
        for (size_t c = 0; c < p.canon.size() && found < 0; ++c) {
            int perm[3] = {0, 1, 2};
            do {
                if (L.l[perm[0]] == p.canon[c].l[0] && L.l[perm[1]] == p.canon[c].l[1] &&
                    L.l[perm[2]] == p.canon[c].l[2]) {
                    found = (int)c;
                    std::memcpy(pos, perm, sizeof(pos));
                    break;
                }
            } while (std::next_permutation(perm, perm + 3));
        }
        p.out_canon.push_back(found);
        // canonical position k holds original position pos[k]
        p.out_pos.push_back({pos[0], pos[1], pos[2]});
        int inv = 0;
        for (int i = 0; i < 3; ++i)
            for (int j = i + 1; j < 3; ++j) inv += pos[i] > pos[j];
        p.out_sign.push_back(even || (inv % 2 == 0) ? 1 : -1);
    }
    return p;
}

P4Canon p4_canonical(int m1, int m2) {
    const int mo[3] = {m1, m2, -(m1 + m2)};
    int t[3] = {mo[0], mo[1], mo[2]}, n[3] = {-mo[0], -mo[1], -mo[2]};
    std::sort(t, t + 3);
    std::sort(n, n + 3);
    P4Canon c{};
    c.neg = std::lexicographical_compare(n, n + 3, t, t + 3);
    const int *rep = c.neg ? n : t;
    bool used[3] = {false, false, false};
    for (int k = 0; k < 3; ++k) {
        c.m[k] = rep[k];
        for (int i = 0; i < 3; ++i)
            if (!used[i] && (c.neg ? -mo[i] : mo[i]) == rep[k]) {
                used[i] = true;
                c.pos[k] = i;
                break;
            }
    }
    return c;
}

std::vector<std::pair<int, int>> proj4_pairs(int mmax) {
    std::vector<std::pair<int, int>> out;
    for (int m1 = -mmax; m1 <= mmax; ++m1)
        for (int m2 = -mmax; m2 <= mmax; ++m2)
            if (std::abs(m1 + m2) <= mmax) out.push_back({m1, m2});
    return out;
}

}  // namespace sb
