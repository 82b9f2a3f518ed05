/*
 * FP64 CPU oracle: direct real-space correlation and grid-sum contractions.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls
 * this file; only tests, the smoke check and the bench's CPU-baseline leg do.
 *
 * Everything here is the plain definition written out:
 *
 *   coefficients (eq. almconv, and the binned c_m of eq. discretize_cmb):
 *       a^b_j(x) = sum over offsets r with bin(r) = b of  B_j(r) * delta((x + r) mod N)
 *   where B_j(r) is the conjugated basis function at offset r (conj Y_lm(r^) in
 *   3D, e^{-i m phi} in 2D), tabulated by the Python side of the oracle;
 *
 *   two-coefficient contraction (eq. alm_to_zeta_clean without its prefactor,
 *   i.e. the sum of Alg. 5; the projected analogue is the sum of Alg. 7):
 *       Z[g][b1][b2] = sum_x delta(x) sum_{j in group g} a^b1_j(x) conj(a^b2_j(x));
 *
 *   three-coefficient contraction (eq. for zeta_{l1 l2 l3}^{b1 b2 b3} of Sec. 2.3
 *   with E(Lambda) C^Lambda_M = 3j, and eq. proj_4pcf_coeff):
 *       Z[t][b1][b2][b3] = sum_x delta(x) sum_{(j1,j2,j3,w) in term list t}
 *                          w * a^b1_j1(x) a^b2_j2(x) a^b3_j3(x).
 *
 * Accumulation is FP64.  Each thread owns a contiguous range of cells and keeps
 * private totals; the totals are added in thread order at the end, so a run is
 * reproducible for a given thread count.
 *
 * Cells are visited in blocks of consecutive indices and, inside a block, the
 * offset loop runs outside the cell loop.  This is a loop interchange only:
 * every a^b_j(x) still receives its terms in the same offset order, so each
 * value is bit-identical to the cell-by-cell loop.  It keeps the basis table
 * from being streamed from memory once per cell.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <complex.h>
#include <omp.h>

#define OC_BLOCK 32 /* = 8 vectors of 4 doubles */
typedef double v4d __attribute__((vector_size(32)));

/* Periodic wrap of c + r for a cell coordinate c in [0, n) and |r| <= n. */
static inline int64_t wrap1(int64_t v, int64_t n) {
    if (v < 0) return v + n;
    if (v >= n) return v - n;
    return v;
}

static inline void cell_coords(int ndim, const int64_t *shape, int64_t cell, int64_t *coord) {
    int64_t rem = cell;
    for (int d = ndim - 1; d >= 0; --d) {
        coord[d] = rem % shape[d];
        rem /= shape[d];
    }
}

/* Linear index of ((x + r) mod N) for a cell with coordinates cx and offset r. */
static inline int64_t shifted_index(int ndim, const int64_t *shape, const int64_t *cx, const int32_t *r) {
    int64_t idx = 0;
    for (int d = 0; d < ndim; ++d) idx = idx * shape[d] + wrap1(cx[d] + r[d], shape[d]);
    return idx;
}

/* a[c][b][j] for the cells cells[0 .. nc), nc <= OC_BIG: direct correlation
 * (eq. almconv).  Complex values are stored as interleaved (re, im) doubles.
 *
 * Offsets are visited in their table order, in runs of at most OC_CHUNK offsets
 * of one bin.  For each run and each group of OC_BLOCK cells, the neighbour
 * values delta(x + r) are gathered first; then every (basis component, cell)
 * total takes the run's terms in offset order.  Each a^b_j(x) therefore sums
 * its terms in table order, exactly as a cell-by-cell loop would. */
#define OC_CHUNK 64
#define OC_BIG 512
static void coeffs_block(int ndim, const int64_t *shape, const double *delta,
                         int64_t n_off, const int32_t *off, const int32_t *bin,
                         int nbins, int nbasis, const double *basis,
                         const int64_t *cells, int nc, double *a /* nc*nbins*nbasis*2 */,
                         double *restrict acc /* nbins * 2*nbasis * OC_BIG scratch */) {
    static __thread int64_t cx[OC_BIG][3];
    double D[OC_CHUNK][OC_BLOCK] __attribute__((aligned(32)));
    for (int c = 0; c < nc; ++c) cell_coords(ndim, shape, cells[c], cx[c]);
    const int nb2 = 2 * nbasis;
    const int nsub = (nc + OC_BLOCK - 1) / OC_BLOCK;
    memset(acc, 0, sizeof(double) * (size_t)nbins * nb2 * OC_BIG);
    int64_t o0 = 0;
    while (o0 < n_off) {
        const int b = bin[o0];
        int64_t o1 = o0;
        while (o1 < n_off && o1 - o0 < OC_CHUNK && bin[o1] == b) ++o1;
        const int no = (int)(o1 - o0);
        for (int s = 0; s < nsub; ++s) {
            const int c0 = s * OC_BLOCK;
            for (int o = 0; o < no; ++o) {
                const int32_t *r = off + (size_t)(o0 + o) * ndim;
                for (int c = 0; c < OC_BLOCK; ++c)
                    D[o][c] = (c0 + c < nc) ? delta[shifted_index(ndim, shape, cx[c0 + c], r)] : 0.0;
            }
            double *restrict ab = acc + (size_t)b * nb2 * OC_BIG + c0;
            for (int jj = 0; jj < nb2; ++jj) {
                /* row[c] += w_o * D[o][c] for o in run order; eight 4-wide
                 * vectors cover the OC_BLOCK = 32 cells. */
                double *restrict row = ab + (size_t)jj * OC_BIG;
                v4d r0, r1, r2, r3, r4, r5, r6, r7;
                memcpy(&r0, row + 0, 32); memcpy(&r1, row + 4, 32); memcpy(&r2, row + 8, 32); memcpy(&r3, row + 12, 32);
                memcpy(&r4, row + 16, 32); memcpy(&r5, row + 20, 32); memcpy(&r6, row + 24, 32); memcpy(&r7, row + 28, 32);
                for (int o = 0; o < no; ++o) {
                    const double w = basis[(size_t)(o0 + o) * nb2 + jj];
                    const v4d wv = {w, w, w, w};
                    const v4d *d = (const v4d *)D[o];
                    r0 += wv * d[0]; r1 += wv * d[1]; r2 += wv * d[2]; r3 += wv * d[3];
                    r4 += wv * d[4]; r5 += wv * d[5]; r6 += wv * d[6]; r7 += wv * d[7];
                }
                memcpy(row + 0, &r0, 32); memcpy(row + 4, &r1, 32); memcpy(row + 8, &r2, 32); memcpy(row + 12, &r3, 32);
                memcpy(row + 16, &r4, 32); memcpy(row + 20, &r5, 32); memcpy(row + 24, &r6, 32); memcpy(row + 28, &r7, 32);
            }
        }
        o0 = o1;
    }
    for (int c = 0; c < nc; ++c)
        for (int bb = 0; bb < nbins; ++bb)
            for (int jj = 0; jj < nb2; ++jj)
                a[((size_t)c * nbins + bb) * nb2 + jj] = acc[((size_t)bb * nb2 + jj) * OC_BIG + c];
}

/* Coefficients at an explicit list of cells: out[c][b][j] (complex, interleaved). */
int oc_coeffs(int ndim, const int64_t *shape, const double *delta,
              int64_t n_off, const int32_t *off, const int32_t *bin, int nbins,
              int nbasis, const double *basis_ri,
              int64_t ncells, const int64_t *cells, double *out_ri, int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
        double *acc = (double *)malloc(sizeof(double) * (size_t)nbins * 2 * nbasis * OC_BIG);
#pragma omp for schedule(dynamic, 1)
        for (int64_t c0 = 0; c0 < ncells; c0 += OC_BIG) {
            int nc = (int)((ncells - c0) < OC_BIG ? (ncells - c0) : OC_BIG);
            coeffs_block(ndim, shape, delta, n_off, off, bin, nbins, nbasis, basis_ri,
                         cells + c0, nc, out_ri + (size_t)2 * c0 * nbins * nbasis, acc);
        }
        free(acc);
    }
    return 0;
}

/*
 * Contraction over the cells cells[0..ncells) (all cells if cells == NULL).
 * mode 3: out[g][b1][b2]       groups: group_ptr[g]..group_ptr[g+1] index term_j (one j per entry)
 * mode 4: out[t][b1][b2][b3]   groups: group_ptr[t]..group_ptr[t+1] index terms (j1,j2,j3) + weight
 * Output is complex (interleaved re, im), FP64.
 */
int oc_zeta(int ndim, const int64_t *shape, const double *delta,
            int64_t n_off, const int32_t *off, const int32_t *bin, int nbins,
            int nbasis, const double *basis_ri,
            int mode, int ngroups, const int32_t *group_ptr, const int32_t *term_j,
            const double *term_w,
            int64_t ncells, const int64_t *cells, double *out_ri, int nthreads) {
    int64_t ng = 1;
    for (int d = 0; d < ndim; ++d) ng *= shape[d];
    if (ncells <= 0) ncells = ng;
    const size_t per = (mode == 3) ? (size_t)nbins * nbins : (size_t)nbins * nbins * nbins;
    const size_t nout = (size_t)ngroups * per;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int nt = omp_get_max_threads();
    double complex *acc = (double complex *)calloc((size_t)nt * nout, sizeof(double complex));
    if (!acc) return -1;
#pragma omp parallel
    {
        const int tid = omp_get_thread_num();
        const int nth = omp_get_num_threads();
        double complex *z = acc + (size_t)tid * nout;
        double complex *a = (double complex *)malloc(sizeof(double complex) * OC_BIG * nbins * nbasis);
        double *a_ri = (double *)a;
        double *scr = (double *)malloc(sizeof(double) * (size_t)nbins * 2 * nbasis * OC_BIG);
        int64_t *blk = (int64_t *)malloc(sizeof(int64_t) * OC_BIG);
        /* contiguous cell range per thread */
        const int64_t lo = ncells * tid / nth, hi = ncells * (tid + 1) / nth;
        for (int64_t c0 = lo; c0 < hi; c0 += OC_BIG) {
            const int nc = (int)((hi - c0) < OC_BIG ? (hi - c0) : OC_BIG);
            for (int c = 0; c < nc; ++c) blk[c] = cells ? cells[c0 + c] : (c0 + c);
            coeffs_block(ndim, shape, delta, n_off, off, bin, nbins, nbasis, basis_ri, blk, nc, a_ri, scr);
            for (int c = 0; c < nc; ++c) {
                const double dx = delta[blk[c]];
                const double complex *ac = a + (size_t)c * nbins * nbasis;
                if (mode == 3) {
                    for (int g = 0; g < ngroups; ++g)
                        for (int e = group_ptr[g]; e < group_ptr[g + 1]; ++e) {
                            const int j = term_j[e];
                            for (int b1 = 0; b1 < nbins; ++b1) {
                                const double complex u = dx * ac[(size_t)b1 * nbasis + j];
                                double complex *zr = z + ((size_t)g * nbins + b1) * nbins;
                                for (int b2 = 0; b2 < nbins; ++b2)
                                    zr[b2] += u * conj(ac[(size_t)b2 * nbasis + j]);
                            }
                        }
                } else {
                    for (int t = 0; t < ngroups; ++t)
                        for (int e = group_ptr[t]; e < group_ptr[t + 1]; ++e) {
                            const int j1 = term_j[3 * e], j2 = term_j[3 * e + 1], j3 = term_j[3 * e + 2];
                            const double w = term_w[e];
                            for (int b1 = 0; b1 < nbins; ++b1) {
                                const double complex u = w * dx * ac[(size_t)b1 * nbasis + j1];
                                for (int b2 = 0; b2 < nbins; ++b2) {
                                    const double complex v = u * ac[(size_t)b2 * nbasis + j2];
                                    double complex *zr = z + (((size_t)t * nbins + b1) * nbins + b2) * nbins;
                                    for (int b3 = 0; b3 < nbins; ++b3)
                                        zr[b3] += v * ac[(size_t)b3 * nbasis + j3];
                                }
                            }
                        }
                }
            }
        }
        free(a);
        free(scr);
        free(blk);
    }
    double complex *out = (double complex *)out_ri;
    memset(out, 0, sizeof(double complex) * nout);
    for (int t = 0; t < nt; ++t)
        for (size_t i = 0; i < nout; ++i) out[i] += acc[(size_t)t * nout + i];
    free(acc);
    return 0;
}

/*
 * Gradient of L = sum_{g,b1,b2} G[g][b1][b2] * Z3[g][b1][b2] with respect to delta(y),
 * for the two-coefficient contraction.  With K^b_j(r) = B_j(r) on bin b:
 *   dZ/d delta(y) = sum_{j in g} a^b1_j(y) conj(a^b2_j(y))
 *                 + sum_x delta(x) sum_{j in g} [ K^b1_j(y - x) conj(a^b2_j(x))
 *                                                + a^b1_j(x) conj(K^b2_j(y - x)) ].
 * The second line is evaluated by visiting every offset r = y - x of the support.
 * a_all holds the coefficients at every cell: a_all[x][b][j].
 * Output: complex gradient per cell (the real part is the gradient of a real L).
 */
/* Gradient at the cells ys[0..ny) (all cells when ys is NULL).  The coefficients of cell x
 * are row amap[x] of a_all (row x when amap is NULL); every x = y - r of a requested y must
 * have a row. */
int oc_grad3(int ndim, const int64_t *shape, const double *delta,
             int64_t n_off, const int32_t *off, const int32_t *bin, int nbins,
             int nbasis, const double *basis_ri,
             int ngroups, const int32_t *group_ptr, const int32_t *term_j,
             const double *G /* ngroups*nbins*nbins real */,
             const double *a_all_ri, const int64_t *amap, int64_t ny, const int64_t *ys,
             double *out_ri, int nthreads) {
    const double complex *basis = (const double complex *)basis_ri;
    const double complex *a_all = (const double complex *)a_all_ri;
    double complex *out = (double complex *)out_ri;
    int64_t ng = 1;
    for (int d = 0; d < ndim; ++d) ng *= shape[d];
    if (!ys) ny = ng;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t iy = 0; iy < ny; ++iy) {
        const int64_t y = ys ? ys[iy] : iy;
        double complex s = 0;
        const double complex *ay = a_all + (size_t)(amap ? amap[y] : y) * nbins * nbasis;
        /* direct term */
        for (int g = 0; g < ngroups; ++g)
            for (int e = group_ptr[g]; e < group_ptr[g + 1]; ++e) {
                const int j = term_j[e];
                for (int b1 = 0; b1 < nbins; ++b1)
                    for (int b2 = 0; b2 < nbins; ++b2)
                        s += G[((size_t)g * nbins + b1) * nbins + b2] * ay[(size_t)b1 * nbasis + j] *
                             conj(ay[(size_t)b2 * nbasis + j]);
            }
        /* terms through the coefficients of the neighbours x = y - r */
        int64_t cy[3];
        cell_coords(ndim, shape, y, cy);
        for (int64_t o = 0; o < n_off; ++o) {
            int32_t mr[3];
            for (int d = 0; d < ndim; ++d) mr[d] = -off[(size_t)o * ndim + d];
            const int64_t x = shifted_index(ndim, shape, cy, mr);
            const double dx = delta[x];
            const int b = bin[o];
            const double complex *ax = a_all + (size_t)(amap ? amap[x] : x) * nbins * nbasis;
            const double complex *K = basis + (size_t)o * nbasis;
            for (int g = 0; g < ngroups; ++g)
                for (int e = group_ptr[g]; e < group_ptr[g + 1]; ++e) {
                    const int j = term_j[e];
                    for (int b2 = 0; b2 < nbins; ++b2)
                        s += G[((size_t)g * nbins + b) * nbins + b2] * dx * K[j] * conj(ax[(size_t)b2 * nbasis + j]);
                    for (int b1 = 0; b1 < nbins; ++b1)
                        s += G[((size_t)g * nbins + b1) * nbins + b] * dx * ax[(size_t)b1 * nbasis + j] * conj(K[j]);
                }
        }
        out[iy] = s;
    }
    return 0;
}

int oc_max_threads(void) { return omp_get_max_threads(); }
