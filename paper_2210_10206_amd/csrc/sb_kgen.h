// Launch descriptors of the kernel-generation, contraction and reduction passes.
#pragma once

#include "sb_common.h"

namespace sb {

constexpr int kMaxBins = 16;
constexpr int kMaxL = 10;                                   // 3D lmax
constexpr int kMaxM = 16;                                   // 2D mmax
constexpr int kMaxLM = (kMaxL + 1) * (kMaxL + 2) / 2;       // (l, m >= 0) pairs at lmax 10
constexpr int kMaxPack = (kMaxL + 1) / 2;                   // pairs of real m = 0 kernels

struct KgenArgs {
    int ndim;
    int64_t n[3];
    int64_t ng;                  // cells written per kernel: np * (product of the extents after axis 0)
    int np, r0;                  // stored axis-0 planes: index p <= r0 -> p, above -> n0 - (np - p)
    int nbins;
    int64_t thr[kMaxBins + 1];   // floor(e_b^2), exact
    int lmax;                    // 3D lmax or 2D mmax
    int nlm;                     // kernels per bin: (lmax+1)(lmax+2)/2 in 3D, mmax+1 in 2D
    double norm[kMaxLM];         // N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), index l(l+1)/2 + m
    float scale;                 // 1 / N_g
    int npack;                   // 3D: packed m = 0 pairs written after the nlm groups
    int pack_l[2 * kMaxPack];    // (l_a, l_b) of each pair: K_{l_a 0} + i K_{l_b 0}
    int gfirst, gcount;          // kernel groups written: gfirst .. gfirst + gcount - 1 of the
                                 // (nlm + npack) groups, group g to arrays (g - gfirst) * nbins + b
    float2 *out;                 // gcount * nbins arrays of ng cells
};
// Axis-0 planes kept for a kernel support of radius r0 (|c_0| <= r0) on an axis of n cells.
inline int support_planes(int64_t n, int64_t r0) { return (int)((2 * r0 + 1 >= n) ? n : 2 * r0 + 1); }
hipError_t launch_kgen(const KgenArgs &a, hipStream_t s);

// ---- two-coefficient contraction (3PCF): block partials of
//      sum_x w(x) A^b1(x) conj(A^b2(x)) for b1 <= b2 and every coefficient group g.
struct PairArgs {
    const float2 *coef;   // [group][bin][ng] (group stride gstride, bin stride ng)
    int64_t gstride;
    const float *w;       // per-cell weight (the density), ng
    int64_t ng;
    int nbins;
    int ngroups;
    int cells_per_block;
    int want_imag;        // also accumulate the imaginary part (projected 3PCF)
    double *partial;      // [group][block][npairs * (want_imag ? 2 : 1)]
    int nblocks;
    int fields;           // fields of one shape in the launch (grid.z; 0 counts as 1)
    int64_t coef_fs, w_fs, part_fs;   // strides between the fields' coef, w and partial
};
hipError_t launch_pair_contract(const PairArgs &a, hipStream_t s);

// ---- three-coefficient contraction (full 4PCF, canonical Lambda list):
//      block partials of Re sum_x w sum_terms C a^{B1}_{la,ma} a^{B2}_{lb,mb} a^{B3}_{lc,mc}
struct QuadTerm {             // one (m3 >= 0, m1) term of a canonical Lambda
    // All fields are 32-bit: terms are read with scalar loads, which need every field
    // dword aligned (byte-sized fields let the compiler form a base address that is not).
    int32_t ma, mb, mc;       // signed orders of the three coefficients (mc >= 0)
    float c;                  // 3j value times the m3 >= 0 weight (1 or 2)
};
constexpr int kStageStride = 4 + 3 * (kMaxL + 1);
struct QuadArgs {
    const float2 *coef;       // [lm][bin][ng], lm = l(l+1)/2 + m, m >= 0
    const float *w;
    int64_t ng;
    int nbins;
    int nlam;                 // canonical Lambdas
    const int *lam_l;         // 3 per canonical Lambda: (la, lb, lc)
    const int *term_ptr;      // nlam + 1
    const QuadTerm *terms;
    const int *stage;         // per Lambda, kStageStride ints: LDS column of (la,0), (lb,0), (lc,0),
                              // column count, then the global lm index of each column
    int max_cols;             // largest column count over the Lambdas
    int cells_per_block;
    int tile;                 // cells staged in LDS per step
    int nlm;
    double *partial;          // [lam][block][nbins^3]
    int nblocks;
    bool odd;                 // odd Lambda: the imaginary part of the sums (the real part vanishes)
    const int *lm_src;        // optional, 2 per lm: coefficient array and part (0: the complex array,
                              // 1 / 2: the real / imaginary part of a packed m = 0 array)
    int fields;               // fields of one shape in the launch (grid.z; 0 counts as 1)
    int64_t coef_fs, w_fs, part_fs;
};
hipError_t launch_quad_contract(const QuadArgs &a, hipStream_t s);

// Matrix-core form for one ordered Lambda with l <= 4 and at most 8 bins (quad_mfma.h).
struct QuadMArgs {
    const float2 *coef;       // [lm][bin][ng]
    const float *w;
    int64_t ng;
    int nbins;
    int lam;                  // canonical index (partial layout)
    const float *coefw;       // weighted 3j values of this Lambda in table order
    int cells_per_block;
    int nblocks;
    int precision;            // 0 float32 MFMA, 1 split-BF16 MFMA
    double *partial;          // [lam][nbins^3][block]
    const int *lm_src;        // optional, as in QuadArgs
    int fields;               // fields of one shape in the launch (grid.z; 0 counts as 1)
    int64_t coef_fs, w_fs, part_fs;
};
// Returns hipErrorInvalidValue when no kernel exists for (la, lb, lc).
hipError_t launch_quad_mfma(int la, int lb, int lc, const QuadMArgs &a, hipStream_t s);
bool quad_mfma_available(int la, int lb, int lc, int nbins);

// ---- projected 4PCF: block partials of sum_x w c^{b1}_{m1} c^{b2}_{m2} c^{b3}_{m3} (complex)
struct Proj4Args {
    const float2 *coef;       // [m][bin][ng], m >= 0
    const float *w;
    int64_t ng;
    int nbins;
    int npairs;               // canonical (m1, m2) pairs
    const int *pairs;         // 2 per pair
    int mmax;
    int cells_per_block;
    int tile;
    double *partial;          // [pair][block][nbins^3 * 2]
    int nblocks;
    int mfma;                 // 1: the matrix-core kernel (proj4_mfma.hip), 0: the vector kernel
    int precision;            // matrix-core kernel: 0 float32 MFMA, 1 split-BF16 MFMA
    int fields;               // fields of one shape in the launch (grid.z; 0 counts as 1)
    int64_t coef_fs, w_fs, part_fs;
};
hipError_t launch_proj4_contract(const Proj4Args &a, hipStream_t s);
hipError_t launch_proj4_mfma(const Proj4Args &a, hipStream_t s);

// ---- deterministic FP64 reduction of block partials: tot[g][v] = sum_blk partial[g][blk][v]
hipError_t launch_block_sum(const double *partial, int ngroups, int nblocks, int nvals, double *tot,
                            hipStream_t s);

// ---- gather map: out[i] = sum_{t in ptr[i]..ptr[i+1]} coef[t] * src[idx[t]]
hipError_t launch_gather(const double *src, const int *ptr, const int *idx, const double *coef,
                         int nout, double *out, hipStream_t s);

// ---- density ingest: float32 copy of the field (and float64 -> float32 cast)
hipError_t launch_to_f32(const void *in, int dtype, int64_t n, float *out, hipStream_t s);

// ---- input check: count[0] += NaN / Inf values among n float32 (dtype 0) or float64 (1) values
hipError_t launch_count_nonfinite(const void *in, int dtype, int64_t n, unsigned int *count, hipStream_t s);
hipError_t launch_zero_u32(unsigned int *x, int n, hipStream_t s);

// ---- normalization of Sec. 2.5: N_gal = sum (delta + 1) by a float64 reduction in a fixed
//      order (kNormParts block partials, then one block), nbar = N_gal / N_g, and per bin tuple
//      t = (b_1 .. b_order) (b_1 slowest) norm[t] = N_gal prod_i nbar vbin[b_i]; every value of
//      the field's result, taken as rows x tuples x parts, is divided by the norm of its tuple.
constexpr int kNormParts = 1024;
struct NormArgs {
    int nbins;
    int order;                 // npcf - 1 bins per tuple
    int parts;                 // 2 for complex results, else 1
    double vbin[kMaxBins];     // V_bin: offsets per bin (unit cells)
};
hipError_t launch_normalize(const void *delta, int dtype, int64_t ng, const NormArgs &a, double *partial,
                            double *zeta, int64_t nvals, double *norm_out, hipStream_t s);

}  // namespace sb
