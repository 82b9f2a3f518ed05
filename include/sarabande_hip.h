/*
 * sarabande_hip.h -- C ABI of the MI355X (gfx950) SARABANDE hot path.
 *
 * The library measures 3- and 4-point correlation functions of gridded
 * density fields with the FFT method of Sunseri et al. 2022 (arXiv 2210.10206):
 * radially binned angular kernels (Y_lm in 3D, e^{-i m phi} in projected 2D)
 * are correlated with the density by FFTs to give the expansion coefficients
 * about every cell (a^b_lm, eq. almconv; c^b_m, eq. discretize_cmb), which are
 * then contracted with the density and summed over the grid (Alg. 5-8).
 *
 * Conventions (all sizes in grid cells, unit spacing, periodic boundaries):
 *  - Arrays are C-ordered; 3D axes (x, y, z) = (axis 0, 1, 2), 2D (x, y) = (axis 0, 1),
 *    phi = atan2(y, x).
 *  - Offsets are zero-centred: coordinate c(i) = i for 2i < N, else i - N
 *    (notes to Alg. 1 and Alg. 2).  Offset r is in bin b iff e_b < |r| <= e_{b+1},
 *    decided exactly on the float64 edges (the mask of Alg. 1 / Alg. 2); r = 0 is in no bin.
 *  - a^b_lm(x) = sum_{r in b} conj(Y_lm(r^)) delta(x + r) (a correlation, eq. almconv
 *    and its footnote); c^b_m(x) = sum_{r in b} e^{-i m phi(r)} delta(x + r).  Masks are
 *    unnormalised (the 1/V_b of eq. bin_volume_unity is not applied).
 *  - Results are the raw grid sums of the appendix algorithms, without the
 *    (-1)^l/sqrt(2l+1), 1/(2 pi)^2 and 1/V prefactors (Sec. 2.1, 2.2) and without the
 *    normalisation of Sec. 2.5 (sb_normalize applies it on the device).
 *  - All ordered bin tuples are returned, diagonals included.
 *
 * Output layouts (float64 per field, complex values interleaved re, im):
 *  - full 3PCF  (ndim 3, npcf 3): Z[l][b1][b2], l = 0..lmax, real;
 *        Z = sum_x delta sum_{m=-l..l} a^b1_lm conj(a^b2_lm)          (Alg. 5)
 *  - full 4PCF  (ndim 3, npcf 4): Z[L][b1][b2][b3], real, L over the even-parity
 *        (l1, l2, l3) of Alg. 6's loop order (l1 outer, l2, then l3 from |l1-l2| to
 *        min(l1+l2, lmax));  Z = sum_x delta sum_M 3j(l1 l2 l3; m1 m2 m3) a a a   (Alg. 6, Sec. 2.3);
 *        with SB_FLAG_ODD_PARITY the odd-parity L in the same loop order and Z = Im of that sum
 *  - projected 3PCF (ndim 2, npcf 3): Z[m][b1][b2] complex, m = 0..mmax;
 *        Z = sum_x delta c^b1_m conj(c^b2_m)                           (Alg. 7)
 *  - projected 4PCF (ndim 2, npcf 4): Z[p][b1][b2][b3] complex, p over (m1, m2) with m1
 *        outer in -mmax..mmax, m2 inner, |m1 + m2| <= mmax;
 *        Z = sum_x delta c^b1_m1 c^b2_m2 c^b3_{-(m1+m2)}, c_{-m} = conj(c_m)  (Alg. 8, eq. proj_4pcf_coeff)
 *
 * Memory: every device buffer is owned by the caller; the library allocates no device
 * memory.  The plan owns host metadata only: its device tables (twiddles, 3j terms,
 * layout maps) live at the head of the caller's persistent buffer, where sb_prepare
 * copies them.  sb_forward / sb_backward / sb_normalize / sb_prepare enqueue work on the
 * given stream (a hipStream_t passed as void*, NULL = default stream) and return before it
 * finishes (except with SB_FLAG_CHECK_FINITE, whose scan waits).  A plan must not be used
 * from two threads at once.
 *
 * Errors: every call returns an sb_status; argument checks happen before any
 * launch; sb_last_error() gives a thread-local message for the last failure.  A call that
 * fails before its first launch leaves the caller's buffers untouched.
 */
#ifndef SARABANDE_HIP_H
#define SARABANDE_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SB_OK = 0,
    SB_EINVAL = -1,        /* invalid argument (shape, edges, lmax, npcf, ndim, null pointer) */
    SB_EUNSUPPORTED = -2,  /* valid but not supported by the library (grid edge, bin count) */
    SB_EWORKSPACE = -3,    /* bound workspace too small or not bound */
    SB_EHIP = -4,          /* a HIP runtime call failed (detail in sb_last_error) */
    SB_ENOMEM = -5,        /* host allocation failed */
    SB_ENONFINITE = -6,    /* an input holds NaN or Inf (only with SB_FLAG_CHECK_FINITE) */
    SB_ESTATE = -7         /* call out of order (e.g. forward before sb_prepare) */
} sb_status;

typedef enum { SB_PREC_FP32 = 0, SB_PREC_SPLIT_BF16 = 1 } sb_precision;
typedef enum { SB_IN_F32 = 0, SB_IN_F64 = 1 } sb_input_dtype;

/* Flags */
enum {
    SB_FLAG_KEEP_COEFFS = 1u, /* keep every a / c array of the last field in scratch (sb_coeffs) */
    SB_FLAG_UNFUSED = 2u,     /* 3PCFs: write every coefficient array, then contract in a separate
                                 pass (the plain path; the default fuses the contraction into the
                                 last FFT pass and never writes the coefficients) */
    SB_FLAG_NO_MFMA = 4u,     /* full 4PCF: use the plain float32 vector-ALU contraction even where
                                 the matrix-core one exists (lmax <= 4, nbins <= 8); projected
                                 4PCF: the vector-ALU contraction instead of the matrix cores */
    SB_FLAG_ODD_PARITY = 8u,  /* full 4PCF: the odd-parity Lambda (l1 + l2 + l3 odd, Sec. 2.3, the
                                 ones Alg. 6 skips) instead of the even ones; each value is the
                                 imaginary part of the sum, whose real part vanishes for a real
                                 density */
    SB_FLAG_NO_PACK = 16u,    /* full 3PCF (fused forward and adjoint) and full 4PCF: one complex
                                 transform per (l, m) array.  By default the real m = 0 coefficient
                                 fields a_{l0} (Alg. 5, Alg. 6; eq. almconv: the m = 0 kernels are
                                 real) are carried two to a transform, as real and imaginary part,
                                 which removes floor((lmax + 1) / 2) of the (lmax + 1)(lmax + 2) / 2
                                 arrays per bin */
    SB_FLAG_REGEN_KERNELS = 64u, /* fused 3PCF plans: keep no kernel spectra in the persistent buffer;
                                 every call regenerates the stored axis-0 planes of each chunk of
                                 kernel groups (Alg. 1 / Alg. 2 and the transforms along the other
                                 axes) in scratch before using them.  Chosen automatically when the
                                 cache of every shape would exceed 64 GiB (1024^3 grids); such plans
                                 have no adjoint (sb_backward returns SB_EUNSUPPORTED) and no packed
                                 m = 0 pairs.  SB_EUNSUPPORTED on other paths */
    SB_FLAG_HALF_KERNELS = 128u, /* 3D plans: store only the axis-0 planes c_0 = 0 .. r0 of each kernel
                                 spectrum and take the planes c_0 < 0 from them by parity (the
                                 kernels Y*_lm Phi_b change by (-1)^l under r -> -r, Sec. 2), on
                                 the shapes whose support radius r0 is below half of every edge.
                                 Halves the persistent buffer; each pass still reads as many bytes.
                                 Chosen automatically when the full cache would exceed 64 GiB and
                                 with SB_FLAG_REGEN_KERNELS (it halves the planes generated);
                                 without effect on 2D plans and on the other shapes */
    SB_FLAG_KEEP_FOR_ADJOINT = 256u, /* fused 3D full 3PCF plans: every sb_forward keeps each
                                 field's coefficient arrays before the last axis (the middle pass's
                                 output: N_ag array groups x N_b bins per field) in scratch, one
                                 region per field, and an sb_backward that follows on the same
                                 density pointers reads them instead of running the axis-0 and
                                 middle passes again (about 30 % of its time).  The scratch grows to
                                 every field's arrays at once plus one field's arrays for the
                                 backward (sb_plan_workspace; the scratch limit does not chunk such
                                 plans).  The kept arrays belong to the last sb_forward /
                                 sb_forward_graph on the bound scratch; sb_backward only reads them,
                                 so several may follow, and the caller must not change the density
                                 values in between (the pointers are all that is compared).  An
                                 sb_backward on other density pointers, and one after
                                 sb_forward_noalloc, sb_autotune, a rebind or a layout change,
                                 recomputes them (same result) and drops what was kept.
                                 SB_EUNSUPPORTED on other paths and with SB_FLAG_REGEN_KERNELS */
    SB_FLAG_CHECK_FINITE = 32u /* sb_forward / sb_backward / sb_normalize first scan every input array
                                 (densities, and grad_zeta) for NaN and Inf and return SB_ENONFINITE,
                                 with no other work done, when one holds any.  The scan waits for the
                                 stream, so such a plan cannot be captured in a HIP graph
                                 (sb_forward_graph returns SB_ESTATE) */
};

/* Warning bits of a plan (sb_plan_warnings). */
enum {
    SB_WARN_BOX_TRUNCATED = 1u /* the outer bin edge reaches half a grid edge (an offset coordinate
                                 c with 2|c| >= N exists in the support): the zero-centred offsets of
                                 the notes to Alg. 1 / Alg. 2 then cover the box [-N/2, N/2 - 1] only,
                                 each cell once, so the kernel is truncated by the box and is no
                                 longer symmetric under r -> -r; results stay well defined */
};

/* Problem statement: the grid, bins, lmax, full or projected, 3 or 4 PCF
 * (the measure(**kwargs) of Sec. 3.3: projected, NPCF). */
typedef struct {
    int32_t ndim;              /* 3 = full (Y_lm kernels), 2 = projected (e^{-i m phi} kernels) */
    int32_t npcf;              /* 3 or 4 */
    int32_t nbins;             /* 1 .. 16 */
    const double *bin_edges;   /* host, nbins + 1 values, strictly increasing, edges[0] >= 0 */
    int32_t lmax;              /* 3D: l = 0..lmax (<= 10); 2D: mmax, m = 0..mmax (<= 16) */
    int32_t precision;         /* sb_precision: the arithmetic of the contractions on the matrix
                                  cores.  SB_PREC_FP32: float32 MFMA.  SB_PREC_SPLIT_BF16: bf16
                                  MFMA on hi + lo splits of both operands (hi = bf16(x), lo =
                                  bf16(x - hi); products hi*hi + hi*lo + lo*hi, float32
                                  accumulation, about 2^-16 relative per product) for the fused
                                  pair sums of the 3PCFs (Alg. 5, Alg. 7), the full-4PCF
                                  contraction on the matrix cores (lmax <= 4, nbins <= 8; Alg. 6)
                                  and the projected-4PCF one (Alg. 8).  Paths with no split form
                                  (SB_FLAG_UNFUSED or SB_FLAG_KEEP_COEFFS 3PCFs, the vector-ALU
                                  4PCF kernels) return SB_EUNSUPPORTED from sb_plan_create. */
    int32_t input_dtype;       /* sb_input_dtype of the density arrays */
    uint32_t flags;
} sb_problem;

typedef struct sb_plan sb_plan;

/* Create a plan for a batch of `batch` fields whose shapes are given row by row in
 * `shapes` (host, batch x ndim int64, C order of each field's extents).  Fields may differ
 * in shape (uneven batch); each grid edge must be one of 8, 12, 16, 24, 32, 48, 64, 96,
 * 128, 160, 192, 256, 512, 1024 (lengths whose transforms are built: SB_EUNSUPPORTED otherwise).
 * The problem statement is that of the measure(**kwargs) of Sec. 3.3; bins follow the mask
 * of Alg. 1 / Alg. 2.  `prob` and its edges are copied.  Host memory only; *out is NULL on
 * failure.  Errors: SB_EINVAL (null pointer, ndim not 2 / 3, npcf not 3 / 4, nbins < 1, edges
 * not finite, negative or not strictly increasing, lmax < 0 or > 10 (3D) / 16 (2D), unknown
 * precision, dtype or flag combination), SB_EUNSUPPORTED (grid edge, nbins > 16 or > 10 for a
 * 4PCF, split-BF16 on a path without a split form), SB_ENOMEM. */
sb_status sb_plan_create(const sb_problem *prob, int32_t batch, const int64_t *shapes, sb_plan **out);

/* Release the plan's host memory (NULL is a no-op).  The caller's device buffers are not
 * touched; work already enqueued with the plan must have finished. */
void sb_plan_destroy(sb_plan *plan);

/* Device bytes the caller must provide: `persistent` holds the plan's tables and the kernel
 * spectra of every distinct shape (Alg. 1 / Alg. 2 transformed along all axes but the first;
 * kept between calls; for a fused 3D 3PCF plan also the packed m = 0 pairs, see
 * SB_FLAG_NO_PACK), `scratch` the per-field working arrays (density spectrum, the kernel
 * arrays of eq. almconv between FFT passes, block partials).  Errors: SB_EINVAL (null). */
sb_status sb_plan_workspace(const sb_plan *plan, size_t *persistent_bytes, size_t *scratch_bytes);

/* Cap the scratch a 3PCF plan uses for its kernel arrays (default 48 GiB).  When all
 * N_k = nbins (lmax+1)(lmax+2)/2 arrays of the largest field would exceed `bytes`, sb_forward
 * (fused path) and sb_backward run the three passes over chunks of kernel groups, so that
 * grids such as 512^3 fit next to their kernel cache (the memory regime of Sec. 4.1).  Call
 * between sb_plan_create and sb_plan_bind (SB_ESTATE afterwards); sb_plan_workspace then
 * reports the new scratch size.  Plans that need every array at once (4PCFs,
 * SB_FLAG_KEEP_COEFFS) ignore the cap; SB_FLAG_UNFUSED 3PCF plans return SB_EUNSUPPORTED
 * from sb_forward when chunked.  Errors: SB_EINVAL (null plan, bytes = 0), SB_ESTATE. */
sb_status sb_plan_set_scratch_limit(sb_plan *plan, uint64_t bytes);

/* Fields of one shape run through the passes together, one launch per pass for the whole
 * batch (the field is the launch's third grid dimension), in batches of up to `max_fields`:
 * 0 (the default) takes as many as 32 GiB of kernel arrays allow, 1 runs every field through
 * its own launch sequence in field order.  Plans whose passes run in chunks of kernel groups,
 * and SB_FLAG_KEEP_COEFFS plans, use 1.  Results do not depend on the batch (each field's sums
 * are computed by the same launches in the same order).  Call before sb_plan_bind (SB_ESTATE
 * afterwards); sb_plan_workspace then reports the scratch for the batch.  get: the batch the
 * plan uses.  Errors: SB_EINVAL (null plan, max_fields < 0), SB_ESTATE. */
sb_status sb_plan_set_field_batch(sb_plan *plan, int32_t max_fields);
sb_status sb_plan_get_field_batch(const sb_plan *plan, int32_t *fields);

/* Bind caller-owned device buffers (at least the sizes of sb_plan_workspace, 256-byte
 * aligned, on the device current at sb_plan_create).  The library keeps the pointers until
 * the next bind or sb_plan_destroy and never frees them.  A bind invalidates sb_prepare and
 * the captured graph.  Errors: SB_EINVAL (null plan or buffer, misaligned), SB_EWORKSPACE
 * (too small). */
sb_status sb_plan_bind(sb_plan *plan, void *persistent, size_t persistent_bytes,
                       void *scratch, size_t scratch_bytes);

/* Copy the plan's tables into the persistent buffer, generate every binned kernel (Alg. 1 in
 * 3D: Y*_lm on the bin masks; Alg. 2 in 2D: e^{-i m phi}) and transform it along every axis
 * but the first into the persistent buffer.  Must precede sb_forward; needed again only
 * after a re-bind.  Errors: SB_EINVAL, SB_EWORKSPACE (not bound), SB_EHIP. */
sb_status sb_prepare(sb_plan *plan, void *stream);

/* Number of float64 values per field of the result (complex outputs count 2 per entry).
 * Errors: SB_EINVAL (null). */
sb_status sb_zeta_size(const sb_plan *plan, int64_t *doubles_per_field);

/* Index table of the result's leading axis: for the full 4PCF the (l1, l2, l3) of each
 * L (3 ints per row, Alg. 6 loop order), for the projected 4PCF the (m1, m2) of each p
 * (2 ints per row, Alg. 8 loop order), for the 3PCFs the l or m of each row (1 int per row;
 * Alg. 5, Alg. 7).  Host memory owned by the plan, valid until sb_plan_destroy.
 * Errors: SB_EINVAL (null). */
sb_status sb_zeta_index(const sb_plan *plan, int32_t *rows, int32_t *cols, const int32_t **table);

/* Number of offsets in each bin (the N_cells in bin of eq. radial_binning, Sec. 2.5) for
 * field `field`'s grid; counts is a host array of nbins, written in bin order.  Exact
 * integer enumeration of the mask of Alg. 1 / Alg. 2.  Errors: SB_EINVAL (null, field out
 * of range). */
sb_status sb_bin_counts(const sb_plan *plan, int32_t field, int64_t *counts);

/* Warning bits (SB_WARN_*) of the plan, fixed at creation.  Errors: SB_EINVAL (null). */
sb_status sb_plan_warnings(const sb_plan *plan, uint32_t *bits);

/* Forward pass (Alg. 3 / Alg. 4 as the correlation of eq. almconv, then Alg. 5 - Alg. 8):
 * delta[f] (host array of batch device pointers) is field f (input_dtype, C order, the
 * shape given at creation); zeta is a device array of batch * doubles_per_field float64,
 * written in field order with the layouts above.  Reads the persistent buffer, overwrites
 * the scratch.  Errors: SB_EINVAL (null pointer), SB_EWORKSPACE (not bound), SB_ESTATE (no
 * sb_prepare), SB_ENONFINITE (SB_FLAG_CHECK_FINITE and a NaN / Inf input), SB_EUNSUPPORTED
 * (a path that needs every kernel array at once under a scratch limit), SB_EHIP. */
sb_status sb_forward(sb_plan *plan, const void *const *delta, double *zeta, void *stream);

/* Forward pass for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same work and results
 * as sb_forward, but the per-field working arrays live in a fixed array of the library (one
 * 64 MiB array per device, held until the process ends) instead of the caller's scratch, so
 * only the persistent buffer has to be bound (sb_plan_bind accepts a NULL scratch of size 0).
 * Calls no allocating routine.  The plan's scratch need (sb_plan_workspace) must fit the
 * 64 MiB, else SB_EWORKSPACE (sb_plan_set_scratch_limit can lower it for 3PCF plans).  Every
 * call on one device shares that device's array: calls that overlap on one device (several
 * streams, threads or plans at once) race and must be serialised by the caller.  Errors: as
 * sb_forward, plus SB_ESTATE while per-launch timing is on. */
sb_status sb_forward_noalloc(sb_plan *plan, const void *const *delta, double *zeta, void *stream);

/* Normalization of Sec. 2.5 (eq. num_gals and the N of that section, with unit cells: box
 * side = grid resolution, V_bin = the offsets of the bin from sb_bin_counts), applied on the
 * device: for every field f, N_gal = sum_x (delta_f(x) + 1) by a float64 reduction in a
 * fixed order, nbar = N_gal / N_g, and every value of zeta (as written by sb_forward, in
 * place) is divided by N_gal prod_i nbar V_bin(b_i) over the bins of its tuple (b1, b2) or
 * (b1, b2, b3).  norm (optional, device) receives those factors, batch x nbins^(npcf-1)
 * float64 with b1 slowest.  Uses the plan's scratch; needs sb_plan_bind only.  Errors:
 * SB_EINVAL, SB_EWORKSPACE, SB_ENONFINITE (with SB_FLAG_CHECK_FINITE), SB_EHIP. */
sb_status sb_normalize(sb_plan *plan, const void *const *delta, double *zeta, double *norm, void *stream);

/* Adjoint of the full 3PCF (ndim 3, npcf 3; the derivative of the sum of Alg. 5 /
 * eq. alm_to_zeta_clean with respect to the density): given grad_zeta (device, batch *
 * (lmax+1) * nbins^2 float64, the gradient of a real loss with respect to Z[l][b1][b2]),
 * write grad_delta[f] (device, float32, shape of field f) = d loss / d delta.  Recomputes
 * the coefficients; overwrites the scratch.  Errors: as sb_forward, plus SB_EUNSUPPORTED for
 * other problems. */
sb_status sb_backward(sb_plan *plan, const void *const *delta, const double *grad_zeta,
                      float *const *grad_delta, void *stream);

/* Device pointer to the coefficient array of kernel k of the last forward field
 * (flag SB_FLAG_KEEP_COEFFS; eq. almconv, or the c_m of eq. discretize_cmb): complex
 * float32, field shape, inside the scratch; k = lm * nbins + b with lm = l(l+1)/2 + m (3D,
 * m >= 0) or lm = m (2D).  An sb_backward call overwrites the arrays (it recomputes them
 * only up to the last axis).  Errors: SB_EINVAL (null, k out of range), SB_EWORKSPACE. */
sb_status sb_coeffs(const sb_plan *plan, int32_t k, const void **ptr);

/* Launch-shape autotuner: times the candidate tilings of every FFT pass and
 * contraction of this plan on `stream` (which it synchronises) and keeps the fastest.
 * Requires bound workspace and sb_prepare; writes only the plan's scratch (no allocation).
 * cache_path (optional, host file): a JSON object keyed by the device architecture and the
 * plan's problem and shapes; an entry for this plan is applied without timing, otherwise the
 * choices found are added to the file.  Errors: SB_EINVAL (null plan, malformed entry,
 * unwritable file), SB_EWORKSPACE, SB_ESTATE, SB_EHIP. */
sb_status sb_autotune(sb_plan *plan, void *stream, const char *cache_path);

/* Number of launch shapes ("variants") of the FFT passes of length n (0: unsupported
 * length), and the choice of one for the passes of length n along `axis` of this plan
 * (what sb_autotune sets by timing; e.g. to reuse tuned choices).  Untuned passes take
 * variant 0, except those of length 1024 along a strided axis (variant 6, the register-resident
 * form).  Results do not depend on the variant beyond float32 rounding.  Errors: SB_EINVAL
 * (length, axis or variant). */
int32_t sb_fft_variants(int32_t n);
sb_status sb_plan_set_fft_variant(sb_plan *plan, int32_t n, int32_t axis, int32_t variant);
sb_status sb_plan_get_fft_variant(const sb_plan *plan, int32_t n, int32_t axis, int32_t *variant);

/* Cells per workgroup ("contraction tile") of the cell-parallel contractions: the full
 * 4PCF (Alg. 6), the projected 4PCF (Alg. 8) and the unfused 3PCF pair sums (Alg. 5, 7).
 * A power of two within [lo, hi] = [512, 4096] (full 4PCF), [1024, 8192] (projected
 * 4PCF), [2048, 16384] (3PCF); the workspace of sb_plan_workspace holds the partial sums
 * of lo.  sb_autotune sets it by timing; set returns SB_EINVAL outside the range.  The
 * choice only reorders the FP64 sum of per-workgroup partials.  get: lo and hi may be NULL. */
sb_status sb_plan_set_contract_tile(sb_plan *plan, int32_t cells);
sb_status sb_plan_get_contract_tile(const sb_plan *plan, int32_t *cells, int32_t *lo, int32_t *hi);

/* Forward pass replayed from a HIP graph captured on first use for these exact
 * pointers (re-captured when they change).  Same contract and results as sb_forward; needs a
 * non-default stream.  Errors: as sb_forward, plus SB_ESTATE while per-launch timing is on
 * or with SB_FLAG_CHECK_FINITE. */
sb_status sb_forward_graph(sb_plan *plan, const void *const *delta, double *zeta, void *stream);

/* Per-launch timing: with enable = 1 every FFT-pass and contraction launch of later
 * sb_forward / sb_backward calls is bracketed by HIP events recorded on the stream it
 * runs on; enable = 0 stops it.  Either call clears the records. */
sb_status sb_profile(sb_plan *plan, int32_t enable);

/* Sum of the recorded launch durations (milliseconds) and launch counts per stage:
 * stage 0 = FFT passes, 1 = contractions.  Synchronises on the recorded events. */
sb_status sb_stage_times(sb_plan *plan, double *fft_ms, int32_t *n_fft, double *contract_ms,
                         int32_t *n_contract);

/* One recorded launch.  `bytes` is the algorithmic HBM traffic of the launch (every array
 * it must read or write once: 16 B per complex cell per transformed array for an FFT
 * pass, plus 8 B per cell and array for a fused spectral product); `flops` the
 * floating-point work a contraction executes (its counted products and sums). */
typedef struct {
    int32_t stage;       /* 0 FFT pass, 1 contraction, 2 other */
    int32_t kernel;      /* 0 FFT pass, 1 axis-0 correlation pass, 2 fused last pass + contraction,
                            3 pair contraction, 4 full-4PCF contraction, 5 projected-4PCF contraction,
                            6 adjoint preparation, 7 full-4PCF contraction on the matrix cores */
    int32_t fft_n;       /* transform length (FFT passes) */
    int32_t fft_sign;    /* -1 forward, +1 inverse */
    int32_t batch;       /* arrays in the launch */
    double bytes;
    double flops;
    double ms;           /* event-measured duration */
} sb_launch_record;

/* Copy up to `max` recorded launches (oldest first) into `out`; `count` receives the
 * number of records available.  Synchronises on the recorded events. */
sb_status sb_profile_read(sb_plan *plan, int32_t max, int32_t *count, sb_launch_record *out);

/* Name of a status code, the thread-local detail of the last failure, the ABI version. */
const char *sb_status_str(sb_status s);
const char *sb_last_error(void);
int32_t sb_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SARABANDE_HIP_H */
