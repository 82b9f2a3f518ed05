// Binned angular kernels on the grid (Alg. 1 for Y_lm, Alg. 2 for e^{i m phi}).
//
// Every stored cell is visited once.  Only the axis-0 planes that meet the support
// (|c_0| <= r0, at most 2 r0 + 1 planes) are stored; the FFT along the other axes is
// applied afterwards and the axis-0 transform is redone on the fly by the first
// inverse pass.  A cell's offset is the zero-centred coordinate of the *reflected* cell, d_a = c((n_a - i_a) mod n_a), so the array
// written is K(-r): the FFT of that array turns the FFT product of the
// correlation (eq. almconv, a correlation per its footnote) into a plain
// spectral multiplication.  The bin test e_b < |d| <= e_{b+1} is done in
// integers on |d|^2 against floor(e_b^2) (computed exactly on the host), so ties
// on an edge are decided exactly.  Values are evaluated in float64 and stored as
// float32, scaled by 1/N_g so that the unnormalised inverse FFT of the product
// is the correlation itself.
//
//   3D: K^b_lm(d) = conj(Y_lm(d^)) = N_lm Q_l^m(z/r) ((x - i y)/r)^m, m >= 0, with
//       Q_m^m = (-1)^m (2m-1)!!, Q_{m+1}^m = (2m+1) t Q_m^m,
//       (l - m) Q_l^m = (2l - 1) t Q_{l-1}^m - (l + m - 1) Q_{l-2}^m    (t = z / r)
//       (P_l^m = sin^m(theta) Q_l^m with the Condon-Shortley phase).
//   2D: K^b_m(d) = e^{-i m phi} = ((x - i y)/r)^m   (eq. c_m def, kernel K^b_m).
#include "sb_kgen.h"

namespace sb {

__device__ __forceinline__ int64_t centred(int64_t i, int64_t n) { return (2 * i < n) ? i : i - n; }

__global__ void kgen_kernel(KgenArgs a) {
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= a.ng) return;
    // stored cell -> grid index: axes 1.. in full, axis 0 through the plane map
    int64_t idx[3] = {0, 0, 0};
    int64_t rem = cell;
    for (int d = a.ndim - 1; d >= 1; --d) {
        idx[d] = rem % a.n[d];
        rem /= a.n[d];
    }
    {
        const int64_t p = rem;   // stored plane
        idx[0] = (a.np == a.n[0] || p <= a.r0) ? p : a.n[0] - (a.np - p);
    }
    int64_t c[3] = {0, 0, 0};
    for (int d = 0; d < a.ndim; ++d) c[d] = centred((a.n[d] - idx[d]) % a.n[d], a.n[d]);
    const int64_t s = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    int bin = -1;
    if (s > 0) {
        for (int b = 0; b < a.nbins; ++b)
            if (a.thr[b] < s && s <= a.thr[b + 1]) { bin = b; break; }
    }
    const int nb = a.nbins;
    const int64_t ng = a.ng;
    // array base of kernel group g (nullptr: not written by this launch)
    auto group_out = [&](int g) -> float2 * {
        return (g >= a.gfirst && g < a.gfirst + a.gcount) ? a.out + (int64_t)(g - a.gfirst) * nb * ng : nullptr;
    };
    if (bin < 0) {
        for (int k = 0; k < a.gcount * nb; ++k) a.out[(int64_t)k * ng + cell] = make_float2(0.f, 0.f);
        return;
    }
    const double r = sqrt((double)s);
    const double ux = (double)c[0] / r, uy = (double)c[1] / r;
    const double sc = (double)a.scale;
    if (a.ndim == 2) {
        double pr = 1.0, pi = 0.0;  // ((x - i y)/r)^m
        for (int m = 0; m <= a.lmax; ++m) {
            if (float2 *o = group_out(m))
                for (int b = 0; b < nb; ++b)
                    o[(int64_t)b * ng + cell] =
                        (b == bin) ? make_float2((float)(pr * sc), (float)(pi * sc)) : make_float2(0.f, 0.f);
            const double nr = pr * ux + pi * uy;   // (pr + i pi)(ux - i uy)
            const double ni = pi * ux - pr * uy;
            pr = nr; pi = ni;
        }
        return;
    }
    const double t = (double)c[2] / r;
    double pr = 1.0, pi = 0.0;   // ((x - i y)/r)^m
    double qmm = 1.0;            // Q_m^m
    float k0[kMaxL + 1];         // the real m = 0 kernels, for the packed pairs
    for (int m = 0; m <= a.lmax; ++m) {
        double qlm2 = 0.0, qlm1 = qmm;  // Q_{l-2}, Q_{l-1} as l advances
        for (int l = m; l <= a.lmax; ++l) {
            double q;
            if (l == m) q = qmm;
            else if (l == m + 1) q = (2.0 * m + 1.0) * t * qmm;
            else q = ((2.0 * l - 1.0) * t * qlm1 - (double)(l + m - 1) * qlm2) / (double)(l - m);
            if (l > m) { qlm2 = qlm1; qlm1 = q; }
            const int lm = l * (l + 1) / 2 + m;
            const double f = a.norm[lm] * q * sc;
            const float2 v = make_float2((float)(f * pr), (float)(f * pi));
            if (m == 0) k0[l] = v.x;
            if (float2 *o = group_out(lm))
                for (int b = 0; b < nb; ++b) o[(int64_t)b * ng + cell] = (b == bin) ? v : make_float2(0.f, 0.f);
        }
        // advance to m + 1
        qmm = -(2.0 * m + 1.0) * qmm;
        const double nr = pr * ux + pi * uy;
        const double ni = pi * ux - pr * uy;
        pr = nr; pi = ni;
    }
    // packed pairs: K_{l_a 0} + i K_{l_b 0}, both real
    for (int i = 0; i < a.npack; ++i) {
        const float2 v = make_float2(k0[a.pack_l[2 * i]], k0[a.pack_l[2 * i + 1]]);
        if (float2 *o = group_out(a.nlm + i))
            for (int b = 0; b < nb; ++b) o[(int64_t)b * ng + cell] = (b == bin) ? v : make_float2(0.f, 0.f);
    }
}

hipError_t launch_kgen(const KgenArgs &a, hipStream_t s) {
    const int nt = 256;
    hipLaunchKernelGGL(kgen_kernel, dim3((unsigned)((a.ng + nt - 1) / nt)), dim3(nt), 0, s, a);
    return hipGetLastError();
}

}  // namespace sb
