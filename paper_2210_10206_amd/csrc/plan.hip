// C ABI of the SARABANDE HIP library: plan creation, workspace layout, kernel
// generation (Alg. 1 / Alg. 2) and the forward pass (Alg. 3 / Alg. 4 by FFT
// correlation, then the contractions of Alg. 5 - Alg. 8).
#include "sarabande_hip.h"
#include "sb_kgen.h"
#include "sb_plan.h"
#include "sb_tables.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

namespace sb {

thread_local std::string g_last_error;

sb_status fail(sb_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

sb_status hip_fail(hipError_t e, const char *what) {
    return fail(SB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static bool supported_edge(int64_t n) {
    return n >= 8 && n <= 1024 && fft_supported((int)n);
}

// Half kernel store: the kernels Y*_lm Phi_b have parity (-1)^l under r -> -r (Sec. 2, the
// spherical-harmonic basis), so the stored planes c_0 = 0 .. r0 give the planes c_0 < 0 -- as
// long as no axis truncates the support (2 r0 < N on every axis, where the zero-centred offsets
// cover +-r0 whole).  3D grids only: the 2D planes are small, and there the mirrored rounding
// moved the smallest projected-4PCF blocks past the float32 bound.  The plan takes it where the
// full store would not fit (want = true), since it saves memory but no traffic: the mirrored
// planes are read all the same.
bool half_store(const ShapeGroup &G, int ndim, int64_t r0, bool want) {
    if (!want || ndim != 3) return false;
    for (int d = 0; d < ndim; ++d)
        if (2 * r0 >= G.n[d]) return false;
    return true;
}

// Axis-0 planes stored per kernel for support radius r0.
int stored_planes(const ShapeGroup &G, int ndim, int64_t r0, bool want) {
    const int64_t r = std::min<int64_t>(r0, G.n[0]);
    return half_store(G, ndim, r0, want) ? (int)r + 1 : support_planes(G.n[0], r);
}

// The half-store fields of an axis-0 launch whose kernel group 0 is global group kgroup0.
void mirror_args(const sb_plan *p, const ShapeGroup &G, int kgroup0, Axis0Args &a) {
    a.half = G.half ? 1 : 0;
    a.nflip = p->nlm;   // (l, m) or m groups; the packed m = 0 pairs (3D) come after them
    a.kgroup0 = kgroup0;
    a.odd_lo = a.odd_hi = 0;
    for (int g = 0; g < p->nlm && g < 128; ++g) {
        int l = g;   // 2D: group g is m = g
        if (p->prob.ndim == 3) {
            l = 0;
            while ((l + 1) * (l + 2) / 2 <= g) ++l;
        }
        if (l & 1) (g < 64 ? a.odd_lo : a.odd_hi) |= (uint64_t)1 << (g & 63);
    }
    a.n1 = G.n[1];
    a.n2 = p->prob.ndim == 3 ? G.n[2] : 1;
}

// ------------------------------------------------------------------ plan creation

static sb_status build_gather(sb_plan *p, std::vector<int> &gptr, std::vector<int> &gidx, std::vector<double> &gcoef) {
    const int NB = p->prob.nbins;
    gptr.assign(1, 0);
    auto add = [&](int src, double c) { gidx.push_back(src); gcoef.push_back(c); };
    auto close = [&]() { gptr.push_back((int)gidx.size()); };
    const int NP = NB * (NB + 1) / 2;
    auto pidx = [&](int b1, int b2) {
        if (b1 > b2) std::swap(b1, b2);
        return b1 * NB - b1 * (b1 - 1) / 2 + (b2 - b1);
    };
    if (p->prob.ndim == 3 && p->prob.npcf == 3) {
        for (int l = 0; l <= p->prob.lmax; ++l)
            for (int b1 = 0; b1 < NB; ++b1)
                for (int b2 = 0; b2 < NB; ++b2) {
                    for (int m = 0; m <= l; ++m) add((l * (l + 1) / 2 + m) * NP + pidx(b1, b2), m == 0 ? 1.0 : 2.0);
                    close();
                }
    } else if (p->prob.ndim == 2 && p->prob.npcf == 3) {
        for (int m = 0; m <= p->prob.lmax; ++m)
            for (int b1 = 0; b1 < NB; ++b1)
                for (int b2 = 0; b2 < NB; ++b2) {
                    add(m * 2 * NP + pidx(b1, b2), 1.0);
                    close();
                    if (b1 != b2) add(m * 2 * NP + NP + pidx(b1, b2), b1 < b2 ? 1.0 : -1.0);
                    close();
                }
    } else if (p->prob.ndim == 3 && p->prob.npcf == 4) {
        const int NV = NB * NB * NB;
        for (size_t L = 0; L < p->f4.out_lams.size(); ++L) {
            const int c = p->f4.out_canon[L];
            const auto &pos = p->f4.out_pos[L];
            for (int b1 = 0; b1 < NB; ++b1)
                for (int b2 = 0; b2 < NB; ++b2)
                    for (int b3 = 0; b3 < NB; ++b3) {
                        const int b[3] = {b1, b2, b3};
                        add(c * NV + (b[pos[0]] * NB + b[pos[1]]) * NB + b[pos[2]], (double)p->f4.out_sign[L]);
                        close();
                    }
        }
    } else {
        const int NV2 = 2 * NB * NB * NB;
        for (const auto &pr : p->p4_pairs) {
            const P4Canon cn = p4_canonical(pr.first, pr.second);
            const int key = p->p4_canon_index.at({cn.m[0], cn.m[1]});
            for (int b1 = 0; b1 < NB; ++b1)
                for (int b2 = 0; b2 < NB; ++b2)
                    for (int b3 = 0; b3 < NB; ++b3) {
                        const int b[3] = {b1, b2, b3};
                        const int f = (b[cn.pos[0]] * NB + b[cn.pos[1]]) * NB + b[cn.pos[2]];
                        add(key * NV2 + 2 * f, 1.0);
                        close();
                        add(key * NV2 + 2 * f + 1, cn.neg ? -1.0 : 1.0);
                        close();
                    }
        }
    }
    return SB_OK;
}

// cpb: cells per workgroup (0: the plan's current choice)
static void contraction_shape(const sb_plan *p, int64_t ng, int *groups, int *nvals, int *nblocks, int cpb = 0) {
    const int NB = p->prob.nbins;
    if (cpb == 0) cpb = p->contract_tile();
    if (p->prob.npcf == 3) {
        *groups = p->nlm;
        *nvals = NB * (NB + 1) / 2 * (p->prob.ndim == 2 ? 2 : 1);
    } else if (p->prob.ndim == 3) {
        *groups = (int)p->f4.canon.size();
        *nvals = NB * NB * NB;
    } else {
        *groups = (int)p->p4_canon.size();
        *nvals = 2 * NB * NB * NB;
    }
    *nblocks = (int)((ng + cpb - 1) / cpb);
}


// Scratch layout.  A 3PCF plan whose full set of kernel arrays exceeds coef_limit runs its
// passes over chunks of kernel groups (the fused contraction and the adjoint only need one
// group's bins at a time); every other plan keeps all arrays at once.
void layout_scratch(sb_plan *p) {
    const sb_problem *prob = &p->prob;
    const int NB = prob->nbins;
    const uint64_t per_group = (uint64_t)NB * p->max_ng * sizeof(float2);
    p->chunk_groups = p->nlm;
    p->kept = false;
    const bool chunkable = prob->npcf == 3 && (prob->flags & SB_FLAG_KEEP_COEFFS) == 0 && !p->keep;
    if (chunkable && per_group * p->nlm > p->coef_limit)
        p->chunk_groups = (int)std::max<uint64_t>(1, std::min<uint64_t>(p->nlm, p->coef_limit / per_group));
    // fields per batch (the region of each per-field buffer below is fbatch fields long)
    int maxf = 1;
    for (const auto &G : p->groups) maxf = std::max<int>(maxf, (int)G.fields.size());
    p->fbatch = 1;
    if (p->chunk_groups == p->nlm && !p->regen && (prob->flags & SB_FLAG_KEEP_COEFFS) == 0) {
        const double per_field = (double)per_group * p->nlm;
        p->fbatch = p->fbatch_req > 0 ? std::min(maxf, p->fbatch_req)
                                      : std::max(1, std::min(maxf, (int)(kBatchBytes / per_field)));
    }
    const size_t FB = (size_t)p->fbatch;
    size_t sc = 0;
    p->off_w = sc; sc += align256(FB * p->max_ng * sizeof(float));
    p->off_dhat = sc; sc += align256(FB * p->max_ng * sizeof(float2));
    const bool adjoint = prob->ndim == 3 && prob->npcf == 3 && !p->regen;
    // the adjoint's v arrays directly before the coefficient arrays: its fused pass writes the v
    // of each group into the slot before that group's coefficients
    if (adjoint) { p->off_vtmp = sc; sc += align256((size_t)NB * p->max_ng * sizeof(float2)); }
    p->off_coef = sc;
    if (p->keep) {
        // one region per field: the forward's array groups (packed m = 0 pairs first) of all bins
        const int nag = p->npack > 0 ? p->nag : p->nlm;
        p->keep_off.assign(p->batch, 0);
        size_t k = 0;
        for (const auto &G : p->groups)
            for (const int f : G.fields) {
                p->keep_off[f] = k;
                k += (size_t)nag * NB * G.ng * sizeof(float2);
            }
        // at least the region the recomputing backward uses (one field of every (l, m) group)
        sc += align256(std::max(k, (size_t)p->nlm * NB * p->max_ng * sizeof(float2)));
        p->off_vkeep = sc;
        sc += align256((size_t)nag * NB * p->max_ng * sizeof(float2));
    } else {
        sc += align256(FB * p->chunk_groups * NB * p->max_ng * sizeof(float2));
    }
    if (p->regen) {   // the stored axis-0 planes of one chunk's kernels
        int64_t kc = 0;
        for (const auto &G : p->groups) kc = std::max<int64_t>(kc, (int64_t)G.np * G.plane);
        p->off_kc = sc; sc += align256((size_t)p->chunk_groups * NB * kc * sizeof(float2));
    }
    int groups = 0, nvals = 0, nblocks = 0, tile_lo = 0, tile_hi = 0;
    p->contract_tile_range(&tile_lo, &tile_hi);
    contraction_shape(p, p->max_ng, &groups, &nvals, &nblocks, tile_lo);
    for (const auto &G : p->groups)
        if (G.rows > 0 && prob->npcf == 3) {
            const int64_t nrows = G.ng / G.n[prob->ndim - 1];
            nblocks = std::max<int>(nblocks, (int)((nrows + G.rows_per_block - 1) / G.rows_per_block));
        }
    p->off_part = sc;
    sc += align256(std::max<size_t>(FB * groups * nvals * nblocks, kNormParts) * sizeof(double));
    p->off_tot = sc; sc += align256(FB * groups * nvals * sizeof(double));
    p->off_grad = sc; sc += align256((size_t)p->max_ng * sizeof(float2));
    p->off_flag = sc; sc += 256;
    p->off_zt = sc; sc += align256((size_t)p->zeta_doubles * sizeof(double));
    if (adjoint) {
        p->off_dsum = sc; sc += align256((size_t)p->max_ng * sizeof(float));
        p->off_gtab = sc; sc += align256((size_t)(prob->lmax + 1) * 256 * sizeof(float));   // G_l, 16 x 16
    }
    p->scratch_need = sc;
}

// Device addresses of the tables in the bound persistent buffer (filled by sb_prepare).
static void table_pointers(sb_plan *p) {
    char *base = p->persist;
    p->tw.clear();
    for (auto &kv : p->tw_off) p->tw[kv.first] = reinterpret_cast<const float2 *>(base + kv.second);
    if (p->prob.npcf == 4 && p->prob.ndim == 3) {
        p->d_terms = reinterpret_cast<const QuadTerm *>(base + p->off_terms);
        p->d_term_ptr = reinterpret_cast<const int *>(base + p->off_tptr);
        p->d_lam_l = reinterpret_cast<const int *>(base + p->off_laml);
        p->d_stage = reinterpret_cast<const int *>(base + p->off_stage);
        p->d_coefw = reinterpret_cast<const float *>(base + p->off_coefw);
    }
    if (p->prob.npcf == 4 && p->prob.ndim == 2) p->d_pairs = reinterpret_cast<const int *>(base + p->off_pairs);
    if (p->npack > 0) {
        p->d_kmap = reinterpret_cast<const int *>(base + p->off_kmap);
        p->d_rowmap = reinterpret_cast<const int *>(base + p->off_rowmap);
        p->d_lmsrc = reinterpret_cast<const int *>(base + p->off_lmsrc);
    }
    p->d_gptr = reinterpret_cast<const int *>(base + p->off_gptr);
    p->d_gidx = reinterpret_cast<const int *>(base + p->off_gidx);
    p->d_gcoef = reinterpret_cast<const double *>(base + p->off_gcoef);
}

sb_status plan_create(const sb_problem *prob, int32_t batch, const int64_t *shapes, sb_plan **out) {
    if (!prob || !shapes || !out) return fail(SB_EINVAL, "null argument");
    *out = nullptr;
    if (prob->ndim != 2 && prob->ndim != 3) return fail(SB_EINVAL, "ndim must be 2 or 3");
    if (prob->npcf != 3 && prob->npcf != 4) return fail(SB_EINVAL, "npcf must be 3 or 4");
    if (prob->nbins < 1) return fail(SB_EINVAL, "nbins must be >= 1");
    if (prob->nbins > kMaxBins) return fail(SB_EUNSUPPORTED, "nbins > 16");
    if (prob->npcf == 4 && prob->nbins > 10) return fail(SB_EUNSUPPORTED, "4PCF supports nbins <= 10");
    if (!prob->bin_edges) return fail(SB_EINVAL, "bin_edges is null");
    if (prob->lmax < 0) return fail(SB_EINVAL, "lmax must be >= 0");
    if (prob->ndim == 3 && prob->lmax > kMaxL) return fail(SB_EINVAL, "lmax > 10");
    if (prob->ndim == 2 && prob->lmax > kMaxM) return fail(SB_EINVAL, "mmax > 16");
    if ((prob->flags & SB_FLAG_ODD_PARITY) && !(prob->npcf == 4 && prob->ndim == 3))
        return fail(SB_EINVAL, "odd parity applies to the full 4PCF only");
    if (prob->precision != SB_PREC_FP32 && prob->precision != SB_PREC_SPLIT_BF16)
        return fail(SB_EINVAL, "unknown precision");
    if (prob->input_dtype != SB_IN_F32 && prob->input_dtype != SB_IN_F64)
        return fail(SB_EINVAL, "unknown input dtype");
    if (batch < 1) return fail(SB_EINVAL, "batch must be >= 1");
    for (int b = 0; b <= prob->nbins; ++b) {
        const double e = prob->bin_edges[b];
        if (!std::isfinite(e) || e < 0.0) return fail(SB_EINVAL, "bin edges must be finite and >= 0");
        if (b > 0 && !(e > prob->bin_edges[b - 1])) return fail(SB_EINVAL, "bin edges must increase strictly");
    }
    sb_plan *p = new (std::nothrow) sb_plan();
    if (!p) return fail(SB_ENOMEM, "plan allocation");
    p->prob = *prob;
    p->edges.assign(prob->bin_edges, prob->bin_edges + prob->nbins + 1);
    p->prob.bin_edges = p->edges.data();
    for (int b = 0; b <= prob->nbins; ++b)
        if (!exact_floor_square(p->edges[b], &p->thr[b])) {
            delete p;
            return fail(SB_EUNSUPPORTED, "bin edge too large");
        }
    p->batch = batch;
    p->max_ng = 0;
    for (int f = 0; f < batch; ++f) {
        std::array<int64_t, 3> sh = {1, 1, 1};
        int64_t ng = 1;
        for (int d = 0; d < prob->ndim; ++d) {
            sh[d] = shapes[(int64_t)f * prob->ndim + d];
            if (sh[d] < 1) { delete p; return fail(SB_EINVAL, "grid extents must be positive"); }
            if (!supported_edge(sh[d])) {
                delete p;
                return fail(SB_EUNSUPPORTED, "grid edge " + std::to_string(sh[d]) +
                                                 " not in {8,12,16,24,32,48,64,96,128,160,192,256,512,1024}");
            }
            ng *= sh[d];
        }
        p->shapes.push_back(sh);
        int gid = -1;
        for (size_t g = 0; g < p->groups.size(); ++g)
            if (p->groups[g].n[0] == sh[0] && p->groups[g].n[1] == sh[1] && p->groups[g].n[2] == sh[2]) gid = (int)g;
        if (gid < 0) {
            ShapeGroup G;
            G.n[0] = sh[0]; G.n[1] = sh[1]; G.n[2] = sh[2];
            G.ng = ng;
            p->groups.push_back(G);
            gid = (int)p->groups.size() - 1;
        }
        p->groups[gid].fields.push_back(f);
        p->field_group.push_back(gid);
        p->max_ng = std::max(p->max_ng, ng);
    }
    const int NB = prob->nbins;
    p->nlm = prob->ndim == 3 ? (prob->lmax + 1) * (prob->lmax + 2) / 2 : prob->lmax + 1;
    p->nk = p->nlm * NB;
    // array groups of the fused 3D 3PCF forward path: the real m = 0 kernels go two to a
    // complex transform (the kernel Y*_{l0} Phi_b of eq. almconv is real), packed pairs first, then one (l, m) per group
    // Kernel spectra regenerated per call instead of cached (fused 3PCF plans only): on request, or
    // when the compact cache of every shape would exceed kKernelCacheCap (1024^3 at 10 bins and
    // lmax 6 would need about 169 GB).
    {
        int64_t r0c = 0;
        while ((r0c + 1) * (r0c + 1) <= p->thr[NB]) ++r0c;
        auto cache = [&](bool half) {
            double c = 0.0;
            for (const auto &G : p->groups)
                c += (double)p->nlm * NB * stored_planes(G, prob->ndim, r0c, half) * (double)(G.ng / G.n[0]) *
                     sizeof(float2);
            return c;
        };
        const bool fused3 = prob->npcf == 3 && (prob->flags & (SB_FLAG_UNFUSED | SB_FLAG_KEEP_COEFFS)) == 0;
        if ((prob->flags & SB_FLAG_REGEN_KERNELS) && !fused3) {
            delete p;
            return fail(SB_EUNSUPPORTED, "kernel regeneration applies to the fused 3PCF path only");
        }
        // half store on request or where the full one would pass the cap; regeneration where even
        // the half store would (and then the half store too: it halves the planes generated)
        p->half = (prob->flags & SB_FLAG_HALF_KERNELS) || cache(false) > kKernelCacheCap;
        p->regen = fused3 && ((prob->flags & SB_FLAG_REGEN_KERNELS) || cache(p->half) > kKernelCacheCap);
        if (p->regen) p->half = true;
    }
    {
        // 3PCF: the fused path (forward and adjoint); 4PCF: the coefficients the contraction reads
        // (its kernels take each m = 0 column from its packed array through lm_src)
        bool pack = prob->ndim == 3 && prob->lmax >= 1 && (prob->flags & (SB_FLAG_KEEP_COEFFS | SB_FLAG_NO_PACK)) == 0;
        if (prob->npcf == 3) {
            if (prob->flags & SB_FLAG_UNFUSED) pack = false;
            if (p->regen) pack = false;
            for (const auto &G : p->groups)
                if (fused_last_rows((int)G.n[prob->ndim - 1], NB) <= 0) pack = false;
        }
        if (pack) {
            p->npack = (prob->lmax + 1) / 2;
            for (int i = 0; i < p->npack; ++i) {
                const int la = 2 * i, lb = 2 * i + 1;
                p->pack_l[2 * i] = la;
                p->pack_l[2 * i + 1] = lb;
                p->ag_kmap.push_back(p->nlm + i);
                p->ag_rowmap.push_back(la * (la + 1) / 2);
                p->ag_rowmap.push_back(lb * (lb + 1) / 2);
            }
            for (int l = 0; l <= prob->lmax; ++l)
                for (int m = 0; m <= l; ++m) {
                    if (m == 0 && l < 2 * p->npack) continue;   // in a packed pair
                    const int lm = l * (l + 1) / 2 + m;
                    p->ag_kmap.push_back(lm);
                    p->ag_rowmap.push_back(lm);
                    p->ag_rowmap.push_back(-1);
                }
            p->nag = (int)p->ag_kmap.size();
            // (array group, part) of every (l, m): part 1 / 2 for the real / imaginary part of a pair
            p->lm_src.assign(2 * p->nlm, 0);
            for (int g = 0; g < p->nag; ++g)
                for (int part = 0; part < 2; ++part) {
                    const int lm = p->ag_rowmap[2 * g + part];
                    if (lm < 0) continue;
                    p->lm_src[2 * lm] = g;
                    p->lm_src[2 * lm + 1] = g < p->npack ? part + 1 : 0;
                }
        }
    }
    // bin counts per group (host enumeration of the same integer test as the kernels)
    for (auto &G : p->groups) {
        for (int b = 0; b < NB; ++b) G.counts[b] = 0;
        int64_t lim[3];
        for (int d = 0; d < 3; ++d) lim[d] = d < prob->ndim ? G.n[d] : 1;
        const int64_t rmax = (int64_t)std::floor(p->edges[NB]) + 1;
        for (int64_t i = 0; i < lim[0]; ++i) {
            const int64_t ci = (2 * i < lim[0]) ? i : i - lim[0];
            if (std::llabs(ci) > rmax) continue;
            for (int64_t j = 0; j < lim[1]; ++j) {
                const int64_t cj = prob->ndim >= 2 ? ((2 * j < lim[1]) ? j : j - lim[1]) : 0;
                if (std::llabs(cj) > rmax) continue;
                for (int64_t k = 0; k < lim[2]; ++k) {
                    const int64_t ck = prob->ndim == 3 ? ((2 * k < lim[2]) ? k : k - lim[2]) : 0;
                    const int64_t s = ci * ci + cj * cj + ck * ck;
                    if (s == 0) continue;
                    for (int b = 0; b < NB; ++b)
                        if (p->thr[b] < s && s <= p->thr[b + 1]) { G.counts[b]++; break; }
                }
            }
        }
    }
    // result layout
    const int L = prob->lmax;
    if (prob->npcf == 3) {
        p->zeta_doubles = (int64_t)(L + 1) * NB * NB * (prob->ndim == 2 ? 2 : 1);
        p->idx_rows = L + 1;
        p->idx_cols = 1;
        for (int l = 0; l <= L; ++l) p->idx_table.push_back(l);
    } else if (prob->ndim == 3) {
        // the matrix-core kernels cover l <= 4 and <= 8 bins; their canonical orderings are
        // chosen for that kernel
        const bool mfma = (prob->flags & SB_FLAG_NO_MFMA) == 0 && L <= 4 && NB <= 8;
        p->f4 = make_full4_plan(L, NB, (prob->flags & SB_FLAG_ODD_PARITY) == 0, mfma);
        p->zeta_doubles = (int64_t)p->f4.out_lams.size() * NB * NB * NB;
        p->idx_rows = (int32_t)p->f4.out_lams.size();
        p->idx_cols = 3;
        for (const Lam &x : p->f4.out_lams)
            for (int k = 0; k < 3; ++k) p->idx_table.push_back(x.l[k]);
    } else {
        p->p4_pairs = proj4_pairs(L);
        for (const auto &pr : p->p4_pairs) {
            const P4Canon cn = p4_canonical(pr.first, pr.second);
            if (!p->p4_canon_index.count({cn.m[0], cn.m[1]})) {
                p->p4_canon_index[{cn.m[0], cn.m[1]}] = (int)p->p4_canon.size();
                p->p4_canon.push_back({cn.m[0], cn.m[1]});
            }
        }
        p->zeta_doubles = (int64_t)p->p4_pairs.size() * NB * NB * NB * 2;
        p->idx_rows = (int32_t)p->p4_pairs.size();
        p->idx_cols = 2;
        for (const auto &pr : p->p4_pairs) { p->idx_table.push_back(pr.first); p->idx_table.push_back(pr.second); }
    }
    // ---- device tables: twiddles per distinct length, 4PCF terms, gather map.  Built on the
    // host here; sb_prepare copies them into the head of the caller's persistent buffer.
    std::vector<int> lens;
    for (const auto &G : p->groups)
        for (int d = 0; d < prob->ndim; ++d)
            if (std::find(lens.begin(), lens.end(), (int)G.n[d]) == lens.end()) lens.push_back((int)G.n[d]);
    std::vector<char> &host = p->host_tab;
    auto put = [&](const void *src, size_t bytes) {
        const size_t off = align256(host.size());
        host.resize(off + bytes);
        if (bytes) std::memcpy(host.data() + off, src, bytes);
        return off;
    };
    for (int n : lens) {
        std::vector<float2> tw(n);
        for (int j = 0; j < n; ++j) {
            const double ang = -2.0 * M_PI * (double)j / (double)n;
            tw[j] = make_float2((float)std::cos(ang), (float)std::sin(ang));
        }
        p->tw_off[n] = put(tw.data(), tw.size() * sizeof(float2));
    }
    if (prob->npcf == 4 && prob->ndim == 3) {
        std::vector<QuadTerm> terms;
        std::vector<int> tptr(1, 0), laml, stage;
        std::vector<float> coefw;
        p->max_cols = 0;
        for (size_t c = 0; c < p->f4.canon.size(); ++c) {
            const Lam &C = p->f4.canon[c];
            p->coefw_off.push_back((int)coefw.size());
            for (const auto &t : p->f4.terms[c]) {
                coefw.push_back((float)t.c);
                if (t.c == 0.0) continue;   // the generic kernel skips vanishing symbols
                QuadTerm q;
                q.ma = t.ma; q.mb = t.mb; q.mc = t.mc;
                q.c = (float)t.c;
                terms.push_back(q);
            }
            tptr.push_back((int)terms.size());
            for (int k = 0; k < 3; ++k) laml.push_back(C.l[k]);
            // staged columns: distinct l values in the order la, lb, lc; column = offset + m
            std::vector<int> st(kStageStride, 0);
            int ncol = 0;
            int offs[3];
            for (int q = 0; q < 3; ++q) {
                int prev = -1;
                for (int r = 0; r < q; ++r)
                    if (C.l[r] == C.l[q]) prev = r;
                if (prev >= 0) { offs[q] = offs[prev]; continue; }
                offs[q] = ncol;
                for (int m = 0; m <= C.l[q]; ++m) st[4 + ncol + m] = C.l[q] * (C.l[q] + 1) / 2 + m;
                ncol += C.l[q] + 1;
            }
            st[0] = offs[0]; st[1] = offs[1]; st[2] = offs[2]; st[3] = ncol;
            p->max_cols = std::max(p->max_cols, ncol);
            stage.insert(stage.end(), st.begin(), st.end());
        }
        p->off_terms = put(terms.data(), terms.size() * sizeof(QuadTerm));
        p->off_tptr = put(tptr.data(), tptr.size() * sizeof(int));
        p->off_laml = put(laml.data(), laml.size() * sizeof(int));
        p->off_stage = put(stage.data(), stage.size() * sizeof(int));
        p->off_coefw = put(coefw.data(), coefw.size() * sizeof(float));
        p->quad_mfma = (prob->flags & SB_FLAG_NO_MFMA) == 0;
        for (const Lam &C : p->f4.canon) p->quad_mfma &= quad_mfma_available(C.l[0], C.l[1], C.l[2], prob->nbins);
    }
    if (prob->npcf == 4 && prob->ndim == 2) {
        std::vector<int> pr;
        for (const auto &x : p->p4_canon) { pr.push_back(x.first); pr.push_back(x.second); }
        p->off_pairs = put(pr.data(), pr.size() * sizeof(int));
    }
    if (p->npack > 0) {
        p->off_kmap = put(p->ag_kmap.data(), p->ag_kmap.size() * sizeof(int));
        p->off_rowmap = put(p->ag_rowmap.data(), p->ag_rowmap.size() * sizeof(int));
        p->off_lmsrc = put(p->lm_src.data(), p->lm_src.size() * sizeof(int));
    }
    std::vector<int> gptr, gidx;
    std::vector<double> gcoef;
    build_gather(p, gptr, gidx, gcoef);
    p->gather_nout = (int)gptr.size() - 1;
    p->off_gptr = put(gptr.data(), gptr.size() * sizeof(int));
    p->off_gidx = put(gidx.data(), gidx.size() * sizeof(int));
    p->off_gcoef = put(gcoef.data(), gcoef.size() * sizeof(double));
    p->tab_bytes = align256(host.size());
    // ---- kernel support along axis 0, fused-pass tiling, workspace layout
    int64_t r0 = 0;
    while ((r0 + 1) * (r0 + 1) <= p->thr[NB]) ++r0;      // largest |c_0| with c_0^2 <= e_max^2
    p->fused = (prob->flags & (SB_FLAG_UNFUSED | SB_FLAG_KEEP_COEFFS)) == 0;
    p->adj_fused = (prob->flags & SB_FLAG_UNFUSED) == 0;
    if (prob->flags & SB_FLAG_KEEP_FOR_ADJOINT) {
        if (prob->ndim != 3 || prob->npcf != 3 || !p->fused || p->regen) {
            delete p;
            return fail(SB_EUNSUPPORTED, "keeping the arrays for the adjoint applies to fused 3D 3PCF plans that "
                                         "cache their kernel spectra");
        }
        p->keep = true;
    }
    // an offset coordinate of magnitude r0 with 2 r0 >= N does not fit the zero-centred box
    for (const auto &G : p->groups)
        for (int d = 0; d < prob->ndim; ++d)
            if (2 * r0 >= G.n[d]) p->warnings |= SB_WARN_BOX_TRUNCATED;
    size_t pers = p->tab_bytes;
    for (auto &G : p->groups) {
        G.plane = G.ng / G.n[0];
        G.r0 = (int)std::min<int64_t>(r0, G.n[0]);
        G.half = half_store(G, prob->ndim, r0, p->half);
        G.np = stored_planes(G, prob->ndim, r0, p->half);
        G.khat_off = pers;
        if (!p->regen) pers += align256((size_t)p->kernel_groups() * NB * G.np * G.plane * sizeof(float2));
        // fused last pass: rows per tile fixed by the kernel's compile-time tile shape
        const int nl = (int)G.n[prob->ndim - 1];
        G.rows = NB <= kMaxBins ? fused_last_rows(nl, NB) : 0;
        if (G.rows > 0) {
            const int64_t nrows = G.ng / nl;
            int64_t rpb = (nrows + 1023) / 1024;
            rpb = std::max<int64_t>(rpb, 16);
            rpb = (rpb + G.rows - 1) / G.rows * G.rows;
            G.rows_per_block = rpb;
        }
    }
    p->persist_need = pers;
    // split-BF16 exists for the contractions on the matrix cores only
    if (prob->precision == SB_PREC_SPLIT_BF16) {
        bool ok = true;
        if (prob->npcf == 3) {
            ok = p->fused;
            for (const auto &G : p->groups) ok &= G.rows > 0;
        } else if (prob->ndim == 3) {
            ok = p->quad_mfma;
        } else {
            ok = (prob->flags & SB_FLAG_NO_MFMA) == 0;
        }
        if (!ok) {
            delete p;
            return fail(SB_EUNSUPPORTED, "split-BF16 applies to the contractions on the matrix cores; this path has "
                                         "no split form");
        }
    }
    layout_scratch(p);
    *out = p;
    return SB_OK;
}

// ------------------------------------------------------------------ passes

sb_status fft_axes(sb_plan *p, const int64_t *n, int ndim, int64_t ncell, const int *axes, int naxes, int sign,
                   int first_load, const void *in, int64_t in_bs, float2 *out, int64_t out_bs, int batch,
                   hipStream_t s, int store, const float2 *mul, int64_t mul_bs, float2 *final_out) {
    for (int i = 0; i < naxes; ++i) {
        const int d = axes[i];
        FftPass a{};
        a.n = (int)n[d];
        int64_t stride = 1;
        for (int k = d + 1; k < ndim; ++k) stride *= n[k];
        a.stride = stride;
        a.ng = ncell;
        a.sign = sign;
        a.batch = batch;
        a.tw = p->tw.at(a.n);
        a.variant = p->fft_variant(a.n, d);
        a.out = out;
        a.out_bs = out_bs;
        if (i == 0) {
            a.load = first_load;
            a.in = in;
            a.in_bs = in_bs;
        } else {
            a.load = LOAD_C;
            a.in = out;
            a.in_bs = out_bs;
        }
        const bool last = i == naxes - 1;
        a.store = last ? store : STORE_C;
        a.mul = mul;
        a.mul_bs = mul_bs;
        if (last && final_out) a.out = final_out;
        // algorithmic traffic: read + write of every transformed array
        double bytes = 16.0 * (double)ncell * batch;
        if (a.store == STORE_MACC) bytes += 16.0 * (double)ncell * batch;
        const hipError_t e = p->timed_launch(STAGE_FFT, K_FFT, s, [&]() { return launch_fft_pass(a, s); }, a.n, sign,
                                             batch, bytes);
        if (e != hipSuccess) return hip_fail(e, "fft pass");
    }
    return SB_OK;
}

sb_status fft_all_axes(sb_plan *p, const ShapeGroup &G, int sign, int first_load, const void *in, int64_t in_bs,
                       float2 *out, int64_t out_bs, int batch, hipStream_t s) {
    const int axes[3] = {0, 1, 2};
    return fft_axes(p, G.n, p->prob.ndim, G.ng, axes, p->prob.ndim, sign, first_load, in, in_bs, out, out_bs, batch, s);
}

// Kernel groups [g0, g0 + count) of shape G (Alg. 1 / Alg. 2: the stored axis-0 planes of the
// binned kernels), transformed along every axis but 0, written to out (count * nbins arrays of
// np * plane cells); axis 0 is transformed on the fly by the first inverse pass.
static sb_status gen_kernels(sb_plan *p, const ShapeGroup &G, int g0, int count, float2 *out, hipStream_t s) {
    const int nd = p->prob.ndim;
    const int64_t ncell = (int64_t)G.np * G.plane;
    KgenArgs a{};
    a.ndim = nd;
    for (int d = 0; d < 3; ++d) a.n[d] = G.n[d];
    a.ng = ncell;
    a.np = G.np;
    a.r0 = G.r0;
    a.nbins = p->prob.nbins;
    for (int b = 0; b <= p->prob.nbins; ++b) a.thr[b] = p->thr[b];
    a.lmax = p->prob.lmax;
    a.nlm = p->nlm;
    a.npack = p->npack;
    for (int i = 0; i < 2 * p->npack; ++i) a.pack_l[i] = p->pack_l[i];
    if (nd == 3)
        for (int l = 0; l <= p->prob.lmax; ++l)
            for (int m = 0; m <= l; ++m) a.norm[l * (l + 1) / 2 + m] = ylm_norm(l, m);
    a.scale = (float)(1.0 / (double)G.ng);
    a.gfirst = g0;
    a.gcount = count;
    a.out = out;
    hipError_t e = launch_kgen(a, s);
    if (e != hipSuccess) return hip_fail(e, "kernel generation");
    const int64_t cn[3] = {G.np, G.n[1], G.n[2]};
    const int axes[2] = {1, 2};
    return fft_axes(p, cn, nd, ncell, axes, nd - 1, -1, LOAD_C, out, ncell, out, ncell, count * p->prob.nbins, s);
}

sb_status prepare(sb_plan *p, hipStream_t s) {
    if (!p->persist) return fail(SB_EWORKSPACE, "workspace not bound");
    // the plan's tables go to the head of the persistent buffer (the host copy stays with the plan)
    hipError_t te = hipMemcpyAsync(p->persist, p->host_tab.data(), p->host_tab.size(), hipMemcpyHostToDevice, s);
    if (te != hipSuccess) return hip_fail(te, "table upload");
    if (!p->regen)
        for (auto &G : p->groups) {
            float2 *kc = reinterpret_cast<float2 *>(p->persist + G.khat_off);
            const sb_status st = gen_kernels(p, G, 0, p->kernel_groups(), kc, s);
            if (st != SB_OK) return st;
        }
    p->prepared = true;
    return SB_OK;
}

// First inverse pass: axis-0 correlation of every kernel group with the density spectrum.
// kmap (optional): kernel group of each of the ngr output groups, else groups g0 .. g0 + ngr - 1.
static sb_status axis0_corr(sb_plan *p, const ShapeGroup &G, const float2 *dhat, float2 *out, int g0, int ngr,
                            hipStream_t s, const int *kmap = nullptr, const float2 *kstore = nullptr, int nf = 1) {
    const int NB = p->prob.nbins;
    Axis0Args a{};
    a.n = (int)G.n[0];
    a.plane = G.plane;
    a.ng = G.ng;
    a.np = G.np;
    a.r0 = G.r0;
    a.mode = 0;
    a.dhat = dhat;
    // kstore: the planes of exactly these ngr groups (regenerated); else the cached store
    a.kc = kstore ? kstore
                  : reinterpret_cast<const float2 *>(p->persist + G.khat_off) + (kmap ? 0 : (int64_t)g0 * NB * G.np * G.plane);
    a.kmap = kmap;
    mirror_args(p, G, kmap ? 0 : g0, a);   // kc's group 0 is the store's (with kmap) or group g0
    a.out = out;
    a.nb = NB;
    a.groups = ngr;
    a.tw = p->tw.at(a.n);
    // nf fields of this shape in one launch: field i's spectrum at dhat + i ng, its arrays after
    // the previous field's ngr * NB arrays
    a.fields = nf;
    a.dhat_fs = G.ng;
    a.out_fs = (int64_t)ngr * NB * G.ng;
    // traffic: stored kernel planes read, outputs written, density spectrum read once per group
    const int nk = ngr * NB * nf;
    const double bytes = (double)nk * (8.0 * G.np * G.plane + 8.0 * G.ng) + (double)ngr * nf * 8.0 * G.ng;
    const hipError_t e = p->timed_launch(STAGE_FFT, K_AXIS0, s, [&]() { return launch_axis0(a, s); }, a.n, 1, nk, bytes);
    if (e != hipSuccess) return hip_fail(e, "axis-0 correlation pass");
    return SB_OK;
}

// Density ingest and spectrum (the first step of Alg. 3 / Alg. 4) of nf fields of shape G:
// field i's density at w + i ng, its spectrum at dhat + i ng.
sb_status density_spectrum(sb_plan *p, const ShapeGroup &G, const void *const *deltas, int nf, hipStream_t s) {
    float *w = reinterpret_cast<float *>(p->scratch + p->off_w);
    float2 *dhat = reinterpret_cast<float2 *>(p->scratch + p->off_dhat);
    for (int i = 0; i < nf; ++i) {
        const hipError_t e = launch_to_f32(deltas[i], p->prob.input_dtype, G.ng, w + (int64_t)i * G.ng, s);
        if (e != hipSuccess) return hip_fail(e, "density ingest");
    }
    return fft_all_axes(p, G, -1, LOAD_R32, w, G.ng, dhat, G.ng, nf, s);
}

sb_status density_spectrum(sb_plan *p, const ShapeGroup &G, const void *delta, hipStream_t s) {
    return density_spectrum(p, G, &delta, 1, s);
}

// Coefficients of kernel groups [g0, g0 + ngr) of one field into scratch (Alg. 3 / Alg. 4
// as a correlation); the density spectrum is already in scratch.
sb_status coefficients(sb_plan *p, int f, int g0, int ngr, hipStream_t s, bool last_axis, const int *kmap, int nf) {
    const ShapeGroup &G = p->groups[p->field_group[f]];
    float2 *dhat = reinterpret_cast<float2 *>(p->scratch + p->off_dhat);
    float2 *coef = reinterpret_cast<float2 *>(p->scratch + p->off_coef);
    sb_status st = axis0_corr(p, G, dhat, coef, g0, ngr, s, kmap, nullptr, nf);
    if (st != SB_OK) return st;
    const int axes[2] = {1, 2};
    const int naxes = p->prob.ndim - 1 - (last_axis ? 0 : 1);
    if (naxes == 0) {
        p->last_ng = G.ng;
        return SB_OK;
    }
    st = fft_axes(p, G.n, p->prob.ndim, G.ng, axes, naxes, +1, LOAD_C, coef, G.ng, coef, G.ng,
                  nf * ngr * p->prob.nbins, s);
    if (st != SB_OK) return st;
    p->last_ng = G.ng;
    return SB_OK;
}

// 3PCF of one field with the contraction fused into the last inverse pass (the
// coefficient arrays are never written).
// nf fields of shape G in one launch per pass (nf > 1 only when every array group fits the scratch
// at once); field i's result goes to zout[i].
// coef_off: byte offset of the batch's coefficient arrays past off_coef (a kept field's region).
static sb_status fused_3pcf(sb_plan *p, const ShapeGroup &G, const void *const *deltas, double *const *zout, int nf,
                            size_t coef_off, hipStream_t s) {
    const int nd = p->prob.ndim, NB = p->prob.nbins;
    float2 *dhat = reinterpret_cast<float2 *>(p->scratch + p->off_dhat);
    float2 *coef = reinterpret_cast<float2 *>(p->scratch + p->off_coef + coef_off);
    const float *w = reinterpret_cast<const float *>(p->scratch + p->off_w);
    double *part = reinterpret_cast<double *>(p->scratch + p->off_part);
    double *tot = reinterpret_cast<double *>(p->scratch + p->off_tot);
    if (nf > 1 && p->chunk_groups < p->nlm) return fail(SB_EUNSUPPORTED, "fields batched with chunked kernel groups");
    sb_status st = density_spectrum(p, G, deltas, nf, s);
    if (st != SB_OK) return st;
    // bin counts without a fused last pass (more than 12 bins on a 1024-point last axis) run the
    // plain last pass and the pair contraction
    const bool fused_last = G.rows > 0;
    const int64_t nrows = G.ng / G.n[nd - 1];
    const int nblocks = fused_last ? (int)((nrows + G.rows_per_block - 1) / G.rows_per_block)
                                   : (int)((G.ng + p->cpb_pair - 1) / p->cpb_pair);
    const int nv = NB * (NB + 1) / 2 * (nd == 2 ? 2 : 1);
    const int64_t part_fs = (int64_t)p->nlm * nv * nblocks;   // one field's block partials
    hipError_t e = hipSuccess;
    // array groups: (l, m) groups, or with packing the packed m = 0 pairs and then the rest
    const bool packing = p->npack > 0;
    const int nag = packing ? p->nag : p->nlm;
    float2 *kstore = p->regen ? reinterpret_cast<float2 *>(p->scratch + p->off_kc) : nullptr;
    for (int g0 = 0; g0 < nag; g0 += p->chunk_groups) {
        const int ngr = std::min(p->chunk_groups, nag - g0);
        if (p->regen) {   // this chunk's kernel planes (Alg. 1 / Alg. 2), regenerated into scratch
            st = gen_kernels(p, G, g0, ngr, kstore, s);
            if (st != SB_OK) return st;
        }
        st = axis0_corr(p, G, dhat, coef, g0, ngr, s, packing ? p->d_kmap + g0 : nullptr, kstore, nf);
        if (st != SB_OK) return st;
        if (nd == 3) {
            const int axes[1] = {1};
            st = fft_axes(p, G.n, nd, G.ng, axes, 1, +1, LOAD_C, coef, G.ng, coef, G.ng, nf * ngr * NB, s);
            if (st != SB_OK) return st;
        }
        if (!fused_last) {
            const int axes[1] = {nd - 1};
            st = fft_axes(p, G.n, nd, G.ng, axes, 1, +1, LOAD_C, coef, G.ng, coef, G.ng, nf * ngr * NB, s);
            if (st != SB_OK) return st;
            PairArgs a{};
            a.coef = coef;
            a.gstride = (int64_t)NB * G.ng;
            a.w = w;
            a.ng = G.ng;
            a.nbins = NB;
            a.ngroups = ngr;
            a.cells_per_block = p->cpb_pair;
            a.want_imag = nd == 2;
            a.partial = part + (int64_t)g0 * nv * nblocks;
            a.nblocks = nblocks;
            a.fields = nf;
            a.coef_fs = (int64_t)ngr * NB * G.ng;
            a.w_fs = G.ng;
            a.part_fs = part_fs;
            const double fl = (double)nf * G.ng * ngr * (2.0 + NB * (NB + 1) / 2.0 * (nd == 2 ? 8.0 : 4.0));
            const double by = (double)nf * G.ng * (8.0 * ngr * NB + 4.0);
            e = p->timed_launch(STAGE_CONTRACT, K_PAIR, s, [&]() { return launch_pair_contract(a, s); }, 0, 0, ngr,
                                by, fl);
            if (e != hipSuccess) return hip_fail(e, "pair contraction");
            continue;
        }
        // last pass over array groups [gs, gs + cnt) of this chunk (all packed or none)
        auto last = [&](int gs, int cnt, bool packed) -> hipError_t {
            LastArgs a{};
            a.n = (int)G.n[nd - 1];
            a.ng = G.ng;
            a.in = coef + (int64_t)(gs - g0) * NB * G.ng;
            a.w = w;
            a.nb = NB;
            a.groups = cnt;
            a.rows = G.rows;
            a.rows_per_block = G.rows_per_block;
            a.nblocks = nblocks;
            a.want_imag = nd == 2;
            a.packed = packed;
            a.prec = p->prob.precision == SB_PREC_SPLIT_BF16 ? 1 : 0;
            // with packing the row map places each part's partials at its (l, m) row
            a.rowmap = packing ? p->d_rowmap + 2 * gs : nullptr;
            a.partial = packing ? part : part + (int64_t)gs * nv * nblocks;
            a.tw = p->tw.at(a.n);
            a.fields = nf;
            a.in_fs = (int64_t)ngr * NB * G.ng;
            a.w_fs = G.ng;
            a.part_fs = part_fs;
            const double bytes = nf * ((double)cnt * NB * 8.0 * G.ng + (double)cnt * 4.0 * G.ng);
            const double flops = (double)nf * G.ng * cnt * (2.0 * NB + NB * (NB + 1) / 2.0 * (nd == 2 ? 8.0 : 4.0));
            return p->timed_launch(STAGE_CONTRACT, K_LAST, s, [&]() { return launch_last_contract(a, s); }, a.n, 1,
                                   nf * cnt * NB, bytes, flops);
        };
        if (packing) {
            const int pe = std::min(g0 + ngr, p->npack);
            if (pe > g0) e = last(g0, pe - g0, true);
            const int us = std::max(g0, p->npack);
            if (e == hipSuccess && g0 + ngr > us) e = last(us, g0 + ngr - us, false);
        } else {
            e = last(g0, ngr, false);
        }
        if (e != hipSuccess) return hip_fail(e, "fused last pass");
    }
    e = launch_block_sum(part, nf * p->nlm, nblocks, nv, tot, s);
    if (e != hipSuccess) return hip_fail(e, "block sum");
    for (int i = 0; i < nf && e == hipSuccess; ++i)
        e = launch_gather(tot + (int64_t)i * p->nlm * nv, p->d_gptr, p->d_gidx, p->d_gcoef, p->gather_nout, zout[i], s);
    if (e != hipSuccess) return hip_fail(e, "gather");
    return SB_OK;
}

// Cell-parallel contraction of nf fields of shape G whose coefficient arrays are in scratch (field
// i after the previous field's arrays); field i's result goes to zout[i].
sb_status contract(sb_plan *p, const ShapeGroup &G, double *const *zout, int nf, hipStream_t s) {
    const float *w = reinterpret_cast<const float *>(p->scratch + p->off_w);
    const float2 *coef = reinterpret_cast<const float2 *>(p->scratch + p->off_coef);
    double *part = reinterpret_cast<double *>(p->scratch + p->off_part);
    double *tot = reinterpret_cast<double *>(p->scratch + p->off_tot);
    int groups = 0, nvals = 0, nblocks = 0;
    contraction_shape(p, G.ng, &groups, &nvals, &nblocks);
    hipError_t e = hipSuccess;
    const int NB = p->prob.nbins;
    // field strides: every array group of a field, its density, its block partials
    const int64_t coef_fs = (int64_t)(p->npack > 0 ? p->nag : p->nlm) * NB * G.ng;
    const int64_t part_fs = (int64_t)groups * nvals * nblocks;
    if (p->prob.npcf == 3) {
        PairArgs a{};
        a.coef = coef;
        a.gstride = (int64_t)NB * G.ng;
        a.w = w;
        a.ng = G.ng;
        a.nbins = NB;
        a.ngroups = groups;
        a.cells_per_block = p->cpb_pair;
        a.want_imag = p->prob.ndim == 2;
        a.partial = part;
        a.nblocks = nblocks;
        a.fields = nf;
        a.coef_fs = coef_fs;
        a.w_fs = G.ng;
        a.part_fs = part_fs;
        const double np_ = NB * (NB + 1) / 2.0;
        const double fl = (double)nf * G.ng * groups * (2.0 + np_ * (a.want_imag ? 8.0 : 4.0));
        const double by = (double)nf * G.ng * (8.0 * p->nk + 4.0);
        e = p->timed_launch(STAGE_CONTRACT, K_PAIR, s, [&]() { return launch_pair_contract(a, s); }, 0, 0, groups, by, fl);
    } else if (p->prob.ndim == 3) {
        QuadArgs a{};
        a.coef = coef;
        a.w = w;
        a.ng = G.ng;
        a.nbins = NB;
        a.nlam = groups;
        a.lam_l = p->d_lam_l;
        a.term_ptr = p->d_term_ptr;
        a.terms = p->d_terms;
        a.stage = p->d_stage;
        a.max_cols = p->max_cols;
        a.cells_per_block = p->cpb_quad;
        a.tile = p->quad_tile;
        a.nlm = p->nlm;
        a.partial = part;
        a.nblocks = nblocks;
        a.odd = (p->prob.flags & SB_FLAG_ODD_PARITY) != 0;
        a.lm_src = p->npack > 0 ? p->d_lmsrc : nullptr;
        a.fields = nf;
        a.coef_fs = coef_fs;
        a.w_fs = G.ng;
        a.part_fs = part_fs;
        // flops per cell and canonical Lambda of the plain kernel: per bin pair, 8 per nonzero
        // coupling term, then per mc the weight (2) and the b3 contraction (4 per bin)
        auto lam_flops = [&](size_t c) {
            double nt = 0.0;
            for (const auto &t : p->f4.terms[c]) nt += t.c != 0.0 ? 1.0 : 0.0;
            return (double)NB * NB * (nt * 8.0 + (p->f4.canon[c].l[2] + 1) * (2.0 + 4.0 * NB));
        };
        // flops per cell and canonical Lambda the matrix-core kernel executes on real bins (padding
        // excluded): per computed bin pair (NB^2, or NB (NB + 1) / 2 when la = lb) the coupling FMAs
        // (mc = 0: the +-ma terms paired, 1 FMA for ma = 0 and 2 per ma > 0 for even Lambda, 2 per
        // ma > 0 for odd; mc > 0: 4 per term, 2 when ma or mb is 0) and the b3 contraction (per mc
        // and b3: 1 FMA for mc = 0, 2 above), 2 flops per FMA; then the weight times the b3
        // coefficients (2 per mc and bin)
        auto lam_flops_mfma = [&](size_t c) {
            const Lam &C = p->f4.canon[c];
            const int la = C.l[0], lb = C.l[1], lc = C.l[2];
            const bool odd = ((la + lb + lc) & 1) != 0;
            const double pairs = la == lb ? NB * (NB + 1) / 2.0 : (double)NB * NB;
            double fma = 0.0;
            for (int ma = 0; ma <= std::min(la, lb); ++ma) fma += ma == 0 ? (odd ? 0.0 : 1.0) : 2.0;
            for (int mc = 1; mc <= lc; ++mc)
                for (int ma = -la; ma <= la; ++ma) {
                    const int mb = -ma - mc;
                    if (mb < -lb || mb > lb) continue;
                    fma += (ma == 0 || mb == 0) ? 2.0 : 4.0;
                }
            fma += NB * (1.0 + 2.0 * lc);
            return pairs * 2.0 * fma + 2.0 * NB * (lc + 1);
        };
        if (p->quad_mfma) {
            // one launch per canonical Lambda: its coefficients stay in registers
            double by = 0.0;
            for (size_t c = 0; c < p->f4.canon.size() && e == hipSuccess; ++c) {
                const Lam &C = p->f4.canon[c];
                QuadMArgs m{};
                m.coef = coef;
                m.w = w;
                m.ng = G.ng;
                m.nbins = NB;
                m.lam = (int)c;
                m.coefw = p->d_coefw + p->coefw_off[c];
                m.cells_per_block = p->cpb_quad;
                m.nblocks = nblocks;
                m.precision = p->prob.precision == SB_PREC_SPLIT_BF16 ? 1 : 0;
                m.partial = part;
                m.lm_src = a.lm_src;
                m.fields = nf;
                m.coef_fs = coef_fs;
                m.w_fs = G.ng;
                m.part_fs = part_fs;
                int ncol = 0;
                for (int q = 0; q < 3; ++q) {
                    bool dup = false;
                    for (int r = 0; r < q; ++r) dup |= C.l[r] == C.l[q];
                    if (!dup) ncol += C.l[q] + 1;
                }
                by = (double)nf * G.ng * (8.0 * NB * ncol + 4.0);
                e = p->timed_launch(STAGE_CONTRACT, K_QUAD_MFMA, s,
                                    [&]() { return launch_quad_mfma(C.l[0], C.l[1], C.l[2], m, s); }, 0, 0, nf, by,
                                    (double)nf * G.ng * lam_flops_mfma(c));
            }
        } else {
            double fl = 0.0;
            for (size_t c = 0; c < p->f4.canon.size(); ++c) fl += lam_flops(c);
            fl *= (double)nf * G.ng;
            const double by = (double)nf * G.ng * (8.0 * p->nk + 4.0);
            e = p->timed_launch(STAGE_CONTRACT, K_QUAD, s, [&]() { return launch_quad_contract(a, s); }, 0, 0, groups, by, fl);
        }
    } else {
        Proj4Args a{};
        a.coef = coef;
        a.w = w;
        a.ng = G.ng;
        a.nbins = NB;
        a.npairs = groups;
        a.pairs = p->d_pairs;
        a.mmax = p->prob.lmax;
        a.cells_per_block = p->cpb_proj4;
        a.tile = p->proj4_tile;
        a.partial = part;
        a.nblocks = nblocks;
        a.mfma = (p->prob.flags & SB_FLAG_NO_MFMA) == 0;
        a.precision = p->prob.precision == SB_PREC_SPLIT_BF16 ? 1 : 0;
        a.fields = nf;
        a.coef_fs = coef_fs;
        a.w_fs = G.ng;
        a.part_fs = part_fs;
        const double fl = (double)nf * G.ng * groups * NB * NB * (8.0 + 8.0 * NB);
        const double by = (double)nf * G.ng * (8.0 * p->nk + 4.0);
        e = p->timed_launch(STAGE_CONTRACT, K_PROJ4, s, [&]() { return launch_proj4_contract(a, s); }, 0, 0, groups, by, fl);
    }
    if (e != hipSuccess) return hip_fail(e, "contraction");
    e = launch_block_sum(part, nf * groups, nblocks, nvals, tot, s);
    if (e != hipSuccess) return hip_fail(e, "block sum");
    for (int i = 0; i < nf && e == hipSuccess; ++i)
        e = launch_gather(tot + (int64_t)i * groups * nvals, p->d_gptr, p->d_gidx, p->d_gcoef, p->gather_nout, zout[i], s);
    if (e != hipSuccess) return hip_fail(e, "gather");
    return SB_OK;
}

sb_status check_finite(sb_plan *p, int count, const void *const *in, const int64_t *n, const int *dtype,
                       hipStream_t s) {
    if ((p->prob.flags & SB_FLAG_CHECK_FINITE) == 0) return SB_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return fail(SB_ESTATE, "the finite-value scan waits for the stream and cannot be captured");
    unsigned int *cnt = reinterpret_cast<unsigned int *>(p->scratch + p->off_flag);
    hipError_t e = launch_zero_u32(cnt, 1, s);
    for (int i = 0; i < count && e == hipSuccess; ++i) e = launch_count_nonfinite(in[i], dtype[i], n[i], cnt, s);
    unsigned int host = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&host, cnt, sizeof(host), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "finite-value scan");
    if (host) return fail(SB_ENONFINITE, std::to_string(host) + " NaN / Inf input values");
    return SB_OK;
}

// The densities of every field as scan inputs (plus one extra array when extra != nullptr).
static sb_status check_fields_finite(sb_plan *p, const void *const *delta, hipStream_t s,
                                     const void *extra = nullptr, int64_t extra_n = 0) {
    if ((p->prob.flags & SB_FLAG_CHECK_FINITE) == 0) return SB_OK;
    std::vector<const void *> in(delta, delta + p->batch);
    std::vector<int64_t> n;
    std::vector<int> dt(p->batch, p->prob.input_dtype);
    for (int f = 0; f < p->batch; ++f) n.push_back(p->groups[p->field_group[f]].ng);
    if (extra) {
        in.push_back(extra);
        n.push_back(extra_n);
        dt.push_back(1);
    }
    return check_finite(p, (int)in.size(), in.data(), n.data(), dt.data(), s);
}

sb_status forward(sb_plan *p, const void *const *delta, double *zeta, hipStream_t s) {
    if (!p) return fail(SB_EINVAL, "null plan");
    if (!delta || !zeta) return fail(SB_EINVAL, "null pointer");
    if (!p->persist || !p->scratch) return fail(SB_EWORKSPACE, "workspace not bound");
    if (!p->prepared) return fail(SB_ESTATE, "sb_prepare has not run on the bound workspace");
    for (int f = 0; f < p->batch; ++f)
        if (!delta[f]) return fail(SB_EINVAL, "null field pointer");
    p->kept = false;   // also when the scan below rejects the fields
    if (sb_status st = check_fields_finite(p, delta, s); st != SB_OK) return st;
    // fields of one shape go through the passes together, fbatch at a time (one launch per pass
    // for the whole batch); with fbatch = 1 the fields run one by one in their order
    auto run = [&](const ShapeGroup &G, const int *fidx, int nf) -> sb_status {
        std::vector<const void *> dl(nf);
        std::vector<double *> zo(nf);
        for (int i = 0; i < nf; ++i) {
            dl[i] = delta[fidx[i]];
            zo[i] = zeta + (int64_t)fidx[i] * p->zeta_doubles;
        }
        if (p->chunk_groups < p->nlm && !(p->prob.npcf == 3 && p->fused))
            return fail(SB_EUNSUPPORTED, "this path needs every kernel array at once; raise the scratch limit");
        if (p->prob.npcf == 3 && p->fused)
            return fused_3pcf(p, G, dl.data(), zo.data(), nf, p->keep ? p->keep_off[fidx[0]] : 0, s);
        sb_status st = density_spectrum(p, G, dl.data(), nf, s);
        if (st == SB_OK)   // array groups (packed m = 0 pairs first) where the plan packs
            st = p->npack > 0 ? coefficients(p, fidx[0], 0, p->nag, s, true, p->d_kmap, nf)
                              : coefficients(p, fidx[0], 0, p->nlm, s, true, nullptr, nf);
        if (st == SB_OK) st = contract(p, G, zo.data(), nf, s);
        return st;
    };
    if (p->fbatch <= 1) {
        for (int f = 0; f < p->batch; ++f) {
            const sb_status st = run(p->groups[p->field_group[f]], &f, 1);
            if (st != SB_OK) return st;
        }
    } else {
        for (const auto &G : p->groups)
            for (size_t b0 = 0; b0 < G.fields.size(); b0 += p->fbatch) {
                const int nf = (int)std::min<size_t>(p->fbatch, G.fields.size() - b0);
                const sb_status st = run(G, G.fields.data() + b0, nf);
                if (st != SB_OK) return st;
            }
    }
    if (p->keep) {   // every field's arrays now sit in its region for sb_backward
        p->kept = true;
        p->kept_delta.assign(delta, delta + p->batch);
    }
    return SB_OK;
}

}  // namespace sb

// ====================================================================== C ABI
using namespace sb;

extern "C" {

sb_status sb_plan_create(const sb_problem *prob, int32_t batch, const int64_t *shapes, sb_plan **out) {
    return plan_create(prob, batch, shapes, out);
}

void sb_plan_destroy(sb_plan *plan) {
    if (!plan) return;
    plan->release_graph();
    plan->release_timing();
    delete plan;
}

sb_status sb_plan_workspace(const sb_plan *p, size_t *persistent_bytes, size_t *scratch_bytes) {
    if (!p || !persistent_bytes || !scratch_bytes) return fail(SB_EINVAL, "null argument");
    *persistent_bytes = p->persist_need;
    *scratch_bytes = p->scratch_need;
    return SB_OK;
}

sb_status sb_plan_set_scratch_limit(sb_plan *p, uint64_t bytes) {
    if (!p) return fail(SB_EINVAL, "null plan");
    if (p->persist) return fail(SB_ESTATE, "the scratch limit must be set before sb_plan_bind");
    if (bytes == 0) return fail(SB_EINVAL, "limit must be positive");
    p->coef_limit = bytes;
    layout_scratch(p);
    return SB_OK;
}

sb_status sb_plan_bind(sb_plan *p, void *persistent, size_t persistent_bytes, void *scratch, size_t scratch_bytes) {
    if (!p) return fail(SB_EINVAL, "null plan");
    if (!persistent) return fail(SB_EINVAL, "null persistent workspace");
    // scratch may be left out (NULL, 0 bytes) by callers that only run sb_forward_noalloc
    if (!scratch && scratch_bytes != 0) return fail(SB_EINVAL, "null scratch with a nonzero size");
    if (persistent_bytes < p->persist_need || (scratch && scratch_bytes < p->scratch_need))
        return fail(SB_EWORKSPACE, "workspace smaller than sb_plan_workspace requires");
    if ((reinterpret_cast<uintptr_t>(persistent) & 255) || (reinterpret_cast<uintptr_t>(scratch) & 255))
        return fail(SB_EINVAL, "workspace must be 256-byte aligned");
    p->persist = static_cast<char *>(persistent);
    p->scratch = static_cast<char *>(scratch);
    p->kept = false;
    table_pointers(p);
    p->prepared = false;
    p->release_graph();
    return SB_OK;
}

sb_status sb_prepare(sb_plan *p, void *stream) {
    if (!p) return fail(SB_EINVAL, "null plan");
    return prepare(p, static_cast<hipStream_t>(stream));
}

sb_status sb_zeta_size(const sb_plan *p, int64_t *doubles_per_field) {
    if (!p || !doubles_per_field) return fail(SB_EINVAL, "null argument");
    *doubles_per_field = p->zeta_doubles;
    return SB_OK;
}

sb_status sb_zeta_index(const sb_plan *p, int32_t *rows, int32_t *cols, const int32_t **table) {
    if (!p || !rows || !cols || !table) return fail(SB_EINVAL, "null argument");
    *rows = p->idx_rows;
    *cols = p->idx_cols;
    *table = p->idx_table.data();
    return SB_OK;
}

sb_status sb_bin_counts(const sb_plan *p, int32_t field, int64_t *counts) {
    if (!p || !counts) return fail(SB_EINVAL, "null argument");
    if (field < 0 || field >= p->batch) return fail(SB_EINVAL, "field index out of range");
    const ShapeGroup &G = p->groups[p->field_group[field]];
    for (int b = 0; b < p->prob.nbins; ++b) counts[b] = G.counts[b];
    return SB_OK;
}

sb_status sb_forward(sb_plan *p, const void *const *delta, double *zeta, void *stream) {
    return forward(p, delta, zeta, static_cast<hipStream_t>(stream));
}

sb_status sb_normalize(sb_plan *p, const void *const *delta, double *zeta, double *norm, void *stream) {
    if (!p || !delta || !zeta) return fail(SB_EINVAL, "null argument");
    if (!p->scratch) return fail(SB_EWORKSPACE, "workspace not bound");
    for (int f = 0; f < p->batch; ++f)
        if (!delta[f]) return fail(SB_EINVAL, "null field pointer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (sb_status st = check_fields_finite(p, delta, s); st != SB_OK) return st;
    NormArgs a{};
    a.nbins = p->prob.nbins;
    a.order = p->prob.npcf - 1;
    a.parts = p->prob.ndim == 2 ? 2 : 1;
    int64_t ntup = 1;
    for (int k = 0; k < a.order; ++k) ntup *= a.nbins;
    double *partial = reinterpret_cast<double *>(p->scratch + p->off_part);
    for (int f = 0; f < p->batch; ++f) {
        const ShapeGroup &G = p->groups[p->field_group[f]];
        for (int b = 0; b < a.nbins; ++b) a.vbin[b] = (double)G.counts[b];
        const hipError_t e = launch_normalize(delta[f], p->prob.input_dtype, G.ng, a, partial,
                                              zeta + (int64_t)f * p->zeta_doubles, p->zeta_doubles,
                                              norm ? norm + (int64_t)f * ntup : nullptr, s);
        if (e != hipSuccess) return hip_fail(e, "normalization");
    }
    return SB_OK;
}

sb_status sb_plan_set_field_batch(sb_plan *p, int32_t max_fields) {
    if (!p) return fail(SB_EINVAL, "null plan");
    if (p->persist) return fail(SB_ESTATE, "the field batch must be set before sb_plan_bind");
    if (max_fields < 0) return fail(SB_EINVAL, "max_fields must be >= 0");
    p->fbatch_req = max_fields;
    layout_scratch(p);
    return SB_OK;
}

sb_status sb_plan_get_field_batch(const sb_plan *p, int32_t *fields) {
    if (!p || !fields) return fail(SB_EINVAL, "null argument");
    *fields = p->fbatch;
    return SB_OK;
}

sb_status sb_plan_warnings(const sb_plan *p, uint32_t *bits) {
    if (!p || !bits) return fail(SB_EINVAL, "null argument");
    *bits = p->warnings;
    return SB_OK;
}

sb_status sb_coeffs(const sb_plan *p, int32_t k, const void **ptr) {
    if (!p || !ptr) return fail(SB_EINVAL, "null argument");
    if (k < 0 || k >= p->nk) return fail(SB_EINVAL, "kernel index out of range");
    if (!p->scratch) return fail(SB_EWORKSPACE, "workspace not bound");
    *ptr = p->scratch + p->off_coef + (size_t)k * p->last_ng * sizeof(float2);
    return SB_OK;
}

const char *sb_status_str(sb_status s) {
    switch (s) {
        case SB_OK: return "ok";
        case SB_EINVAL: return "invalid argument";
        case SB_EUNSUPPORTED: return "unsupported";
        case SB_EWORKSPACE: return "workspace missing or too small";
        case SB_EHIP: return "HIP runtime error";
        case SB_ENOMEM: return "out of host memory";
        case SB_ENONFINITE: return "non-finite input";
        case SB_ESTATE: return "call out of order";
        default: return "unknown status";
    }
}

const char *sb_last_error(void) { return g_last_error.c_str(); }

int32_t sb_version(void) { return 1; }

}  // extern "C"
