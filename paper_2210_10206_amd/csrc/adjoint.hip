// Adjoint of the full 3PCF: d loss / d delta for loss = sum g[l][b1][b2] Z[l][b1][b2].
//
// With G_l = (g_l + g_l^T) / 2, K^b_lm(r) = conj(Y_lm(r^)) on bin b and w_0 = 1, w_m = 2:
//   d loss / d delta(y) = D(y) + C(y),
//   D(y) = sum_{l, m >= 0} w_m sum_b1 Re( a^b1_lm(y) h^b1_lm(y) ),  h^b1 = sum_b2 G_l[b1][b2] conj(a^b2_lm)
//   C(y) = 2 Re sum_{l, m >= 0, b} w_m (K^b_lm * v^b_lm)(y),        v^b = delta h^b
// (the ordinary derivative of the trilinear grid sum of Alg. 5 / eq. alm_to_zeta_clean,
// with the -m terms folded in through a_{l,-m} = (-1)^m conj(a_lm)).  The convolution
// K * v equals the forward correlation applied to the reflected field read back at -y,
// so the forward kernel spectra serve unchanged:  U = IFFT( sum_k FFT(w_m v_k(-.)) Khat_k ),
// C(y) = 2 Re U(-y).
#include "sb_plan.h"
#include "adj_last.h"

#include <vector>

namespace sb {
namespace {

__device__ __forceinline__ int64_t flip_index(int64_t cell, int ndim, const int64_t *n) {
    int64_t idx[3] = {0, 0, 0};
    int64_t rem = cell;
    for (int d = ndim - 1; d >= 0; --d) {
        idx[d] = rem % n[d];
        rem /= n[d];
    }
    int64_t out = 0;
    for (int d = 0; d < ndim; ++d) out = out * n[d] + ((n[d] - idx[d]) % n[d]);
    return out;
}

struct AdjPrepArgs {
    const float2 *coef;     // NB arrays of one (l, m)
    const float *w;         // density
    const double *gz;       // g_l, NB x NB
    int nbins;
    float wm;
    int ndim;
    int64_t n[3];
    int64_t ng;
    float2 *vtmp;           // NB arrays: w_m v^b at the reflected cell
    float *dsum;            // direct term, accumulated over (l, m)
    int first;              // write instead of accumulate
};

__global__ void adj_prep_kernel(AdjPrepArgs a) {
    const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= a.ng) return;
    const int NB = a.nbins;
    float2 av[kMaxBins];
    for (int b = 0; b < NB; ++b) av[b] = a.coef[(int64_t)b * a.ng + y];
    const float dy = a.w[y];
    const int64_t yf = flip_index(y, a.ndim, a.n);
    float dsum = 0.f;
    for (int b1 = 0; b1 < NB; ++b1) {
        float hx = 0.f, hy = 0.f;
        for (int b2 = 0; b2 < NB; ++b2) {
            const float G = (float)(0.5 * (a.gz[b1 * NB + b2] + a.gz[b2 * NB + b1]));
            hx += G * av[b2].x;
            hy -= G * av[b2].y;   // conj(a)
        }
        dsum += a.wm * (av[b1].x * hx - av[b1].y * hy);
        a.vtmp[(int64_t)b1 * a.ng + yf] = make_float2(a.wm * dy * hx, a.wm * dy * hy);
    }
    if (a.first) a.dsum[y] = dsum;
    else a.dsum[y] += dsum;
}

__global__ void adj_finish_kernel(const float2 *U, const float *dsum, int ndim, int64_t n0, int64_t n1, int64_t n2,
                                  int64_t ng, float *out) {
    const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= ng) return;
    const int64_t n[3] = {n0, n1, n2};
    const int64_t yf = flip_index(y, ndim, n);
    out[y] = dsum[y] + 2.f * U[yf].x;
}

// G_l = (g_l + g_l^T) / 2 of every l as float, 16 x 16 with zeros beyond nb
__global__ void adj_weights_kernel(const double *gz, int nl, int nb, float *gt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nl * 256) return;
    const int l = i / 256, b1 = i % 256 / 16, b2 = i % 16;
    const double *g = gz + (int64_t)l * nb * nb;
    gt[i] = (b1 < nb && b2 < nb) ? (float)(0.5 * (g[b1 * nb + b2] + g[b2 * nb + b1])) : 0.f;
}

__global__ void zero_c_kernel(float2 *x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = make_float2(0.f, 0.f);
}

}  // namespace

hipError_t launch_adj_last(const AdjLastArgs &a, hipStream_t s) {
    // register-resident stages where the radix list allows (the forward fused pass uses the same
    // lists), the LDS-staged tile kernel otherwise
    hipError_t e = hipErrorInvalidValue;
    switch (a.n) {
        case 64: e = adjlast::launch_rs<64, 8, 8>(a, s); break;
        case 96: e = adjlast::launch_rs<96, 12, 4, 2>(a, s); break;
        case 128: e = adjlast::launch_rs<128, 16, 8>(a, s); break;
        case 160: e = adjlast::launch_rs<160, 20, 4, 2>(a, s); break;
        case 192: e = adjlast::launch_rs<192, 12, 4, 4>(a, s); break;
        case 256: e = adjlast::launch_rs<256, 16, 16>(a, s); break;
        default: break;
    }
    if (e == hipSuccess) return e;
    switch (a.n) {   // (none at 1024: a tile of every bin of a row would not fit the LDS)
#define SB_X(N, TPP, ...)                                                             \
    case N:                                                                           \
        if constexpr (N <= 512) return adjlast::launch_n<N, TPP, __VA_ARGS__>(a, s); \
        else return hipErrorInvalidValue;
        SB_LAST_CONFIGS(SB_X)
#undef SB_X
        default: return hipErrorInvalidValue;
    }
}

sb_status backward(sb_plan *p, const void *const *delta, const double *grad_zeta, float *const *grad_delta,
                   hipStream_t s) {
    if (!p || !delta || !grad_zeta || !grad_delta) return fail(SB_EINVAL, "null argument");
    if (p->prob.ndim != 3 || p->prob.npcf != 3) return fail(SB_EUNSUPPORTED, "adjoint is implemented for the full 3PCF");
    if (!p->persist || !p->scratch) return fail(SB_EWORKSPACE, "workspace not bound");
    if (!p->prepared) return fail(SB_ESTATE, "sb_prepare has not run on the bound workspace");
    if (p->regen) return fail(SB_EUNSUPPORTED, "the adjoint reads cached kernel spectra; this plan regenerates them");
    if (p->adj_fused)
        for (const auto &G : p->groups)
            if (fused_last_rows((int)G.n[2], p->prob.nbins) <= 0 || G.n[2] > 512)
                return fail(SB_EUNSUPPORTED, "no fused adjoint last pass for a last axis of " + std::to_string(G.n[2]) +
                                                 " (use SB_FLAG_UNFUSED)");
    const int NB = p->prob.nbins;
    float2 *acc = reinterpret_cast<float2 *>(p->scratch + p->off_grad);
    float2 *vtmp = reinterpret_cast<float2 *>(p->scratch + p->off_vtmp);
    float *dsum = reinterpret_cast<float *>(p->scratch + p->off_dsum);
    float2 *coef_w = reinterpret_cast<float2 *>(p->scratch + p->off_coef);
    const float2 *coef = coef_w;
    const float *w = reinterpret_cast<const float *>(p->scratch + p->off_w);
    float *gtab = reinterpret_cast<float *>(p->scratch + p->off_gtab);
    const int nl = p->prob.lmax + 1;
    for (int f = 0; f < p->batch; ++f)
        if (!delta[f] || !grad_delta[f]) return fail(SB_EINVAL, "null field pointer");
    if (p->prob.flags & SB_FLAG_CHECK_FINITE) {
        std::vector<const void *> in(delta, delta + p->batch);
        std::vector<int64_t> n;
        std::vector<int> dt(p->batch, p->prob.input_dtype);
        for (int f = 0; f < p->batch; ++f) n.push_back(p->groups[p->field_group[f]].ng);
        in.push_back(grad_zeta);
        n.push_back((int64_t)p->batch * p->zeta_doubles);
        dt.push_back(1);
        if (sb_status st = check_finite(p, (int)in.size(), in.data(), n.data(), dt.data(), s); st != SB_OK) return st;
    }
    // arrays the last forward kept for these fields (SB_FLAG_KEEP_FOR_ADJOINT) replace the
    // recomputed ones; they are only read, so they stay for another backward.  Recomputing
    // overwrites them.
    bool use_kept = p->keep && p->kept && p->adj_fused && (int)p->kept_delta.size() == p->batch;
    for (int f = 0; use_kept && f < p->batch; ++f) use_kept = p->kept_delta[f] == delta[f];
    if (!use_kept) p->kept = false;
    for (int f = 0; f < p->batch; ++f) {
        const ShapeGroup &G = p->groups[p->field_group[f]];
        const float2 *khat = reinterpret_cast<const float2 *>(p->persist + G.khat_off);
        sb_status st = density_spectrum(p, G, delta[f], s);
        if (st != SB_OK) return st;
        const int nt = 256;
        const unsigned nblk = (unsigned)((G.ng + nt - 1) / nt);
        hipLaunchKernelGGL(zero_c_kernel, dim3(nblk), dim3(nt), 0, s, acc, G.ng);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "adjoint zero");
        const double *gz_f = grad_zeta + (int64_t)f * p->zeta_doubles;
        hipLaunchKernelGGL(adj_weights_kernel, dim3((nl * 256 + 255) / 256), dim3(256), 0, s, gz_f, nl, NB, gtab);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "adjoint weights");
        // groups: one per (l, m), or with the fused pass of a packed plan the forward's array
        // groups (the packed m = 0 pairs first)
        const bool packing = p->npack > 0 && p->adj_fused;
        const int ngrp = packing ? p->nag : p->nlm;
        auto l_of = [](int lm, int *m) {
            int l = 0;
            while ((l + 1) * (l + 2) / 2 <= lm) ++l;
            *m = lm - l * (l + 1) / 2;
            return l;
        };
        // (l, m) of group g; a packed group also has l2 (m = 0)
        auto group_l = [&](int g, int *m, int *l2) {
            int m2 = 0;
            *l2 = -1;
            const int l = l_of(packing ? p->ag_rowmap[2 * g] : g, m);
            if (packing && p->ag_rowmap[2 * g + 1] >= 0) *l2 = l_of(p->ag_rowmap[2 * g + 1], &m2);
            return l;
        };
        // acc += sum_{groups, b} FFT(w_m v_b(-.)) * Khat_b over ngr groups whose v arrays start at
        // vin: the axis-0 pass regenerates each kernel spectrum and adds every group's sum in turn
        auto accumulate = [&](const float2 *vin, int g0, int ngr) -> hipError_t {
            Axis0Args x{};
            x.n = (int)G.n[0];
            x.plane = G.plane;
            x.ng = G.ng;
            x.np = G.np;
            x.r0 = G.r0;
            x.mode = 1;
            x.kc = khat;
            mirror_args(p, G, 0, x);
            x.out = acc;
            x.vin = vin;
            x.nb = NB;
            x.groups = 1;
            x.accgroups = ngr;
            x.kmap = packing ? p->d_kmap + g0 : nullptr;
            x.kfirst = g0 * NB;
            x.tw = p->tw.at(x.n);
            return p->timed_launch(STAGE_FFT, K_AXIS0, s, [&]() { return launch_axis0(x, s); }, x.n, -1, ngr * NB,
                                   (double)ngr * NB * (8.0 * G.ng + 8.0 * G.np * G.plane) + 16.0 * ngr * G.ng);
        };
        for (int g0 = 0; g0 < ngrp; g0 += p->chunk_groups) {
            const int ngr = std::min(p->chunk_groups, ngrp - g0);
            // recompute a for this chunk of groups, unless the forward kept it; with the fused pass
            // it stops before the last axis, which that pass finishes
            const float2 *cf = use_kept ? reinterpret_cast<const float2 *>(p->scratch + p->off_coef + p->keep_off[f])
                                        : coef;
            if (!use_kept) {
                st = coefficients(p, f, g0, ngr, s, !p->adj_fused, packing ? p->d_kmap + g0 : nullptr);
                if (st != SB_OK) return st;
            }
            if (p->adj_fused) {
                // per group: last inverse pass + h, D and v + forward transform of v(-x) along the
                // last axis.  v of group g goes to the slot before its own coefficients (the vtmp
                // arrays for the first group, then the coefficients the previous group consumed),
                // so the chunk's v arrays end up contiguous from vbase; kept arrays stay intact,
                // the v arrays going to a region of their own.
                float2 *vbase = use_kept ? reinterpret_cast<float2 *>(p->scratch + p->off_vkeep)
                                         : coef_w - (int64_t)NB * G.ng;
                for (int g = g0; g < g0 + ngr; ++g) {
                    int m = 0, l2 = -1;
                    const int l = group_l(g, &m, &l2);
                    AdjLastArgs a{};
                    a.n = (int)G.n[2];
                    a.ndim = 3;
                    for (int d = 0; d < 3; ++d) a.shape[d] = G.n[d];
                    a.ng = G.ng;
                    a.in = cf + (int64_t)(g - g0) * NB * G.ng;
                    a.w = w;
                    a.gz = gz_f + (int64_t)l * NB * NB;
                    a.gz2 = l2 >= 0 ? gz_f + (int64_t)l2 * NB * NB : nullptr;
                    a.gt = gtab + (int64_t)l * 256;
                    a.gt2 = l2 >= 0 ? gtab + (int64_t)l2 * 256 : nullptr;
                    a.wm = m == 0 ? 1.f : 2.f;
                    a.nb = NB;
                    const int64_t nrows = G.ng / a.n;
                    // about 4096 workgroups (the small grids need them all to fill the chip),
                    // at most 16 rows each
                    a.rows_per_block = std::max<int64_t>(1, std::min<int64_t>(16, nrows / 4096));
                    a.first = g == 0;
                    a.dsum = dsum;
                    a.out = vbase + (int64_t)(g - g0) * NB * G.ng;
                    a.tw = p->tw.at(a.n);
                    e = p->timed_launch(STAGE_OTHER, K_ADJPREP, s, [&]() { return launch_adj_last(a, s); }, a.n, 0,
                                        NB, 16.0 * NB * G.ng + 8.0 * G.ng);
                    if (e != hipSuccess) return hip_fail(e, "adjoint fused last pass");
                }
                const int axes[1] = {1};
                st = fft_axes(p, G.n, 3, G.ng, axes, 1, -1, LOAD_C, vbase, G.ng, vbase, G.ng, ngr * NB, s);
                if (st != SB_OK) return st;
                e = accumulate(vbase, g0, ngr);
                if (e != hipSuccess) return hip_fail(e, "adjoint axis-0 pass");
            } else {
                for (int g = g0; g < g0 + ngr; ++g) {
                    int m = 0, l2 = -1;
                    const int l = group_l(g, &m, &l2);
                    AdjPrepArgs a{};
                    a.coef = coef + (int64_t)(g - g0) * NB * G.ng;
                    a.w = w;
                    a.gz = gz_f + (int64_t)l * NB * NB;
                    a.nbins = NB;
                    a.wm = m == 0 ? 1.f : 2.f;
                    a.ndim = 3;
                    for (int d = 0; d < 3; ++d) a.n[d] = G.n[d];
                    a.ng = G.ng;
                    a.vtmp = vtmp;
                    a.dsum = dsum;
                    a.first = g == 0;
                    e = p->timed_launch(STAGE_OTHER, K_ADJPREP, s, [&]() {
                        hipLaunchKernelGGL(adj_prep_kernel, dim3(nblk), dim3(nt), 0, s, a);
                        return hipGetLastError();
                    });
                    if (e != hipSuccess) return hip_fail(e, "adjoint prep");
                    // transform v_b(-.) along axes 2..1 in place
                    const int axes[2] = {2, 1};
                    st = fft_axes(p, G.n, 3, G.ng, axes, 2, -1, LOAD_C, vtmp, G.ng, vtmp, G.ng, NB, s);
                    if (st != SB_OK) return st;
                    e = accumulate(vtmp, g, 1);
                    if (e != hipSuccess) return hip_fail(e, "adjoint axis-0 pass");
                }
            }
        }
        st = fft_all_axes(p, G, +1, LOAD_C, acc, 0, acc, 0, 1, s);
        if (st != SB_OK) return st;
        hipLaunchKernelGGL(adj_finish_kernel, dim3(nblk), dim3(nt), 0, s, acc, dsum, 3, G.n[0], G.n[1], G.n[2], G.ng,
                           grad_delta[f]);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "adjoint finish");
    }
    return SB_OK;
}

}  // namespace sb

extern "C" sb_status sb_backward(sb_plan *p, const void *const *delta, const double *grad_zeta,
                                 float *const *grad_delta, void *stream) {
    return sb::backward(p, delta, grad_zeta, grad_delta, static_cast<hipStream_t>(stream));
}
