// Mixed-radix Stockham FFT passes for gfx950, LDS-staged.
//
// A launch transforms every pencil of one axis of a batch of C-ordered complex
// arrays.  A workgroup owns P pencils: it stages them in LDS (coalesced: P
// adjacent pencils along the fastest axis for a strided axis, P whole rows for
// the contiguous axis), runs the radix stages in LDS with TPP threads per
// pencil, and writes the tile back.  Loads can fuse the spectral product
// (delta_hat * kernel_hat) or read a real field; stores can fuse a spectral
// multiply-accumulate.  The radix stages are in fft_core.h.
#include <utility>

#include "fft_core.h"

namespace sb {
namespace {
using namespace fftcore;

__device__ __forceinline__ float2 load_elem(const FftPass &a, int y, int64_t idx) {
    switch (a.load) {
        case LOAD_MUL: {
            const float2 x = reinterpret_cast<const float2 *>(a.in)[y * a.in_bs + idx];
            const float2 k = a.in2[y * a.in2_bs + idx];
            return cmul(x, k);
        }
        case LOAD_R32:
            return make_float2(reinterpret_cast<const float *>(a.in)[y * a.in_bs + idx], 0.f);
        case LOAD_R64:
            return make_float2((float)reinterpret_cast<const double *>(a.in)[y * a.in_bs + idx], 0.f);
        default:
            return reinterpret_cast<const float2 *>(a.in)[y * a.in_bs + idx];
    }
}

__device__ __forceinline__ void store_elem(const FftPass &a, int y, int64_t idx, float2 v) {
    float2 *o = a.out + y * a.out_bs + idx;
    if (a.store == STORE_MACC) {
        const float2 m = a.mul[y * a.mul_bs + idx];
        *o = cadd(*o, cmul(v, m));
    } else {
        *o = v;
    }
}

template <int N, int TPP, int NT, int SIGN, int... RAD>
__global__ __launch_bounds__(NT) void fft_pass_kernel(FftPass a) {
    constexpr int P = NT / TPP;
    constexpr int PITCH = P + 1;
    __shared__ float2 sm[N * PITCH];
    __shared__ float2 tw[N];
    __shared__ int64_t base[P];
    const int tid = threadIdx.x;
    const int y = blockIdx.y;
    const int64_t npencil = a.ng / N;
    const int64_t g0 = (int64_t)blockIdx.x * P;
    for (int i = tid; i < N; i += NT) tw[i] = a.tw[i];
    if (tid < P) {
        const int64_t g = g0 + tid;
        base[tid] = (g / a.stride) * (int64_t)N * a.stride + (g % a.stride);
    }
    __syncthreads();
    if (a.stride == 1) {
        for (int f = tid; f < P * N; f += NT) {
            const int p = f / N, j = f % N;
            float2 v = make_float2(0.f, 0.f);
            if (g0 + p < npencil) v = load_elem(a, y, base[p] + j);
            sm[j * PITCH + p] = v;
        }
    } else {
        for (int f = tid; f < P * N; f += NT) {
            const int p = f % P, j = f / P;
            float2 v = make_float2(0.f, 0.f);
            if (g0 + p < npencil) v = load_elem(a, y, base[p] + (int64_t)j * a.stride);
            sm[j * PITCH + p] = v;
        }
    }
    __syncthreads();
    stages<N, TPP, SIGN, 1, RAD...>(sm, tw, tid % P, tid / P, PITCH);
    if (a.stride == 1) {
        for (int f = tid; f < P * N; f += NT) {
            const int p = f / N, j = f % N;
            if (g0 + p < npencil) store_elem(a, y, base[p] + j, sm[j * PITCH + p]);
        }
    } else {
        for (int f = tid; f < P * N; f += NT) {
            const int p = f % P, j = f / P;
            if (g0 + p < npencil) store_elem(a, y, base[p] + (int64_t)j * a.stride, sm[j * PITCH + p]);
        }
    }
}

// ------------------------------------------------------------------------------
// First inverse pass of the correlation, along axis 0, with the kernel spectrum
// regenerated on the fly.  The kernels are stored transformed along the other axes
// and compacted along axis 0 to the np planes of their support (|c_0| <= r0).  For a
// tile of P pencils (P adjacent positions of the (axis 1, axis 2) plane):
//   CORR : for each of the nb kernels of the group: K = FFT_0(stored kernel pencil),
//          T = IFFT_0(delta_hat * K), written out;  delta_hat is read once per group.
//   ADJ  : acc += sum_b FFT_0(v_b) * FFT_0(stored kernel pencil b)   (adjoint)
// Mode 1: kernel index of step t of the flattened (group, bin) loop of an accumulation launch.
__device__ __forceinline__ int64_t acc_kernel(const Axis0Args &a, int t) {
    return a.kmap ? (int64_t)a.kmap[t / a.nb] * a.nb + t % a.nb : (int64_t)a.kfirst + t;
}

// Half store: the in-plane cell of -k for cell g ((i1, i2) -> (-i1, -i2) modulo the extents).
// (The helpers take scalars: a reference to the kernel's argument copy would keep it in scratch.)
__device__ __forceinline__ int64_t mirror_cell(int64_t n1, int64_t n2, int64_t g) {
    const int64_t i1 = g / n2, i2 = g - i1 * n2;
    return ((n1 - i1) % n1) * n2 + (n2 - i2) % n2;
}

// Half store: how a kernel of global group g gives a plane c_0 < 0: 0 the stored plane -c_0 at
// -k, 1 the same negated, 2 the stored plane -c_0 conjugated.
__device__ __forceinline__ int mirror_rule(int g, int nflip, uint64_t odd_lo, uint64_t odd_hi) {
    if (g >= nflip) return 2;
    const uint64_t bits = g < 64 ? odd_lo : odd_hi;
    return (int)((bits >> (g & 63)) & 1);
}

// Where a kernel keeps its planes c_0 < 0 (axis-0 indices j in the upper half of the axis): plane
// pa + pb j, scaled by (sx, sy).  Full store: the stored plane np - n + j as it is (or every plane
// j when the store is dense, np = n).  Half store: plane n - j = -c_0, at -k (rules 0, 1:
// mirrored) or at k (rule 2), with the sign or conjugation of mirror_rule.  All uniform.
struct UpperPlanes {
    int pa, pb;
    bool dense, mirrored;
    float sx, sy;
    // (bit arithmetic on the rule, not selects over its values: those become a lookup table in
    // scratch memory)
    __device__ __forceinline__ UpperPlanes(int half, int rule, int np, int n) {
        const unsigned neg = (unsigned)rule & 1u, conj = (unsigned)rule >> 1;
        pa = half ? n : np - n;
        pb = half ? -1 : 1;
        dense = !half && np == n;
        mirrored = half && !conj;
        sx = __uint_as_float(0x3f800000u | (neg << 31));
        sy = __uint_as_float(0x3f800000u | ((neg | conj) << 31));
    }
};

// Stored-kernel value at axis-0 index j of this thread's cell g (gm: the cell of -k): `upper`
// (compile-time in the callers) says whether j lies in the upper half of the axis.  Zero outside
// the support |c_0| <= r0.
__device__ __forceinline__ float2 kernel_elem(const float2 *kc, int64_t plane, int r0, int j, int n, bool upper, int64_t g,
                                              int64_t gm, const UpperPlanes &u) {
    if (!upper) return (j <= r0 || u.dense) ? ld_stream(&kc[(int64_t)j * plane + g]) : make_float2(0.f, 0.f);
    if (j < n - r0 && !u.dense) return make_float2(0.f, 0.f);
    const float2 v = ld_stream(&kc[(int64_t)(u.pa + u.pb * j) * plane + (u.mirrored ? gm : g)]);
    return make_float2(u.sx * v.x, u.sy * v.y);
}

// The rule of global kernel group grp in an axis-0 launch (0 for a full store).  The groups come
// from 32-bit arithmetic: a 64-bit division would be a call, whose stack frame puts the kernel's
// argument copy in scratch memory.
#define SB_MIRROR_RULE(a, grp) ((a).half ? mirror_rule((grp), (a).nflip, (a).odd_lo, (a).odd_hi) : 0)

// Global kernel group of step t of an accumulation launch (mode 1; see acc_kernel).
__device__ __forceinline__ int acc_group(const Axis0Args &a, int t) {
    return a.kgroup0 + (a.kmap ? a.kmap[t / a.nb] : (a.kfirst + t) / a.nb);
}

template <int N, int TPP, int NT, int... RAD>
__global__ __launch_bounds__(NT) void axis0_kernel(Axis0Args a) {
    // field of the launch (grid.z); local pointers, so the argument struct is never written
    const float2 *dhat0 = a.dhat + (int64_t)blockIdx.z * a.dhat_fs;
    float2 *out0 = a.out + (int64_t)blockIdx.z * a.out_fs;
    constexpr int P = NT / TPP;
    constexpr int PITCH = P + 1;
    constexpr int EPT = N / TPP;      // tile elements per thread: pencil p, rows q0 + e TPP
    __shared__ float2 sm[N * PITCH];
    __shared__ float2 tw[N];
    const int tid = threadIdx.x;
    const int p = tid % P, q0 = tid / P;
    const int64_t g = (int64_t)blockIdx.x * P + p;
    const bool ok = g < a.plane;
    for (int i = tid; i < N; i += NT) tw[i] = a.tw[i];
    const int64_t kstride = (int64_t)a.np * a.plane;
    const int64_t gm = (a.half && ok) ? mirror_cell(a.n1, a.n2, g) : g;
    auto load_kernel = [&](int64_t k, int grp, float2 *dst) {
        const float2 *kc = a.kc + k * kstride;
        const UpperPlanes up(a.half, SB_MIRROR_RULE(a, grp), a.np, N);
#pragma unroll
        for (int e = 0; e < EPT; ++e)   // rows e >= EPT / 2 lie in the upper half of the axis
            dst[e] = ok ? kernel_elem(kc, a.plane, a.r0, q0 + e * TPP, N, 2 * e >= EPT, g, gm, up) : make_float2(0.f, 0.f);
    };
    float2 nx[EPT];
    if (a.mode == 0) {
        float2 dr[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) dr[e] = ok ? dhat0[(int64_t)(q0 + e * TPP) * a.plane + g] : make_float2(0.f, 0.f);
        const int64_t kbase = (int64_t)(a.kmap ? a.kmap[blockIdx.y] : blockIdx.y) * a.nb;   // kernel group
        const int kgrp = a.kgroup0 + (int)(a.kmap ? a.kmap[blockIdx.y] : blockIdx.y);       // its global index
        const int64_t obase = (int64_t)blockIdx.y * a.nb;                                 // output arrays
        load_kernel(kbase, kgrp, nx);
        for (int b = 0; b < a.nb; ++b) {
            __syncthreads();
#pragma unroll
            for (int e = 0; e < EPT; ++e) sm[(q0 + e * TPP) * PITCH + p] = nx[e];
            if (b + 1 < a.nb) load_kernel(kbase + b + 1, kgrp, nx);   // in flight during the transforms
            __syncthreads();
            stages<N, TPP, -1, 1, RAD...>(sm, tw, p, q0, PITCH);
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                float2 *x = &sm[(q0 + e * TPP) * PITCH + p];
                *x = cmul(*x, dr[e]);
            }
            __syncthreads();
            stages<N, TPP, 1, 1, RAD...>(sm, tw, p, q0, PITCH);
            float2 *out = out0 + (obase + b) * a.ng;
            if (ok)
#pragma unroll
                for (int e = 0; e < EPT; ++e) out[(int64_t)(q0 + e * TPP) * a.plane + g] = sm[(q0 + e * TPP) * PITCH + p];
        }
    } else {
        float2 acc[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) acc[e] = make_float2(0.f, 0.f);
        // v of bin b + 1 and its kernel pencil are loaded into registers while bin b is processed
        auto load_v = [&](int b, float2 *dst) {
            const float2 *vb = a.vin + (int64_t)b * a.ng;
#pragma unroll
            for (int e = 0; e < EPT; ++e) dst[e] = ok ? vb[(int64_t)(q0 + e * TPP) * a.plane + g] : make_float2(0.f, 0.f);
        };
        float2 nv[EPT], kx[EPT];
        const int nt = (a.accgroups > 1 ? a.accgroups : 1) * a.nb;   // (group, bin) steps
        load_v(0, nv);
        load_kernel(acc_kernel(a, 0), acc_group(a, 0), nx);
        for (int t = 0; t < nt; ++t) {
            __syncthreads();
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                sm[(q0 + e * TPP) * PITCH + p] = nv[e];
                kx[e] = nx[e];
            }
            if (t + 1 < nt) {
                load_v(t + 1, nv);
                load_kernel(acc_kernel(a, t + 1), acc_group(a, t + 1), nx);
            }
            __syncthreads();
            stages<N, TPP, -1, 1, RAD...>(sm, tw, p, q0, PITCH);
            float2 vr[EPT];
#pragma unroll
            for (int e = 0; e < EPT; ++e) vr[e] = sm[(q0 + e * TPP) * PITCH + p];
            __syncthreads();
#pragma unroll
            for (int e = 0; e < EPT; ++e) sm[(q0 + e * TPP) * PITCH + p] = kx[e];
            __syncthreads();
            stages<N, TPP, -1, 1, RAD...>(sm, tw, p, q0, PITCH);
#pragma unroll
            for (int e = 0; e < EPT; ++e) acc[e] = cadd(acc[e], cmul(vr[e], sm[(q0 + e * TPP) * PITCH + p]));
            if (t % a.nb == a.nb - 1) {   // end of a group: out += its sum, as separate launches would
                if (ok)
#pragma unroll
                    for (int e = 0; e < EPT; ++e) {
                        float2 *o = out0 + (int64_t)(q0 + e * TPP) * a.plane + g;
                        *o = cadd(*o, acc[e]);
                    }
#pragma unroll
                for (int e = 0; e < EPT; ++e) acc[e] = make_float2(0.f, 0.f);
            }
        }
    }
}

// Rows r of a register-resident axis-0 thread (elements q + r2 r, q < r2) that can meet the
// compact kernel support |c_0| <= r0: r <= kr or r >= r1 - kr.  A dense axis returns r1.
inline int support_rows(const Axis0Args &a, int r1, int r2) {
    if (a.np >= a.n) return r1;
    const int pos = a.r0 / r2;                                   // rows holding some j <= r0
    const int first_neg = (a.n - a.r0 - (r2 - 1) + r2 - 1) / r2;   // first row holding some j >= n - r0
    const int neg = r1 - first_neg;
    return pos > neg ? pos : neg;
}

// Axis-0 correlation pass for n = R1 * R2 (R2 divides R1) held in registers: thread q < R2 of a
// pencil owns rows q + R2 s (s < R1).  Those are the inputs of radix-R1 butterfly q of the first
// Stockham stage, and the outputs of butterflies q + R2 t (t < R1 / R2) of the second
// (radix R2), which read positions q + R2 t + R1 r'.  So the forward transform of the kernel
// pencil, the product with the density spectrum and the inverse transform touch LDS only for
// the two stage exchanges (positions R1 q + r written).  One exchange buffer with two barriers
// per exchange keeps the workgroup at 34 KB of LDS, so four of them share a CU.  Loads and
// stores take P adjacent pencils of the contiguous axes per row, as in the LDS-staged kernel.
// A compact kernel is nonzero on rows r <= KR and r >= R1 - KR of each thread at most (KR from
// the support radius, see support_rows; KR >= R1 / 2 for a dense axis): the other rows are
// compile-time zeros, so they are neither loaded nor held, and the first forward stage folds
// them away.
template <int R1, int R2, int P, int MODE, int KR>
__global__ __launch_bounds__(P * R2, MODE == 0 ? (2 * KR < R1 ? 3 : 2) : 1) void axis0_reg_kernel(Axis0Args a) {
    // field of the launch (grid.z); local pointers, so the argument struct is never written
    const float2 *dhat0 = a.dhat + (int64_t)blockIdx.z * a.dhat_fs;
    float2 *out0 = a.out + (int64_t)blockIdx.z * a.out_fs;
    constexpr int N = R1 * R2;
    constexpr int T = R1 / R2;   // second-stage butterflies per thread
    static_assert(R1 % R2 == 0, "R2 must divide R1");
    constexpr int PITCH = P + 1;
    __shared__ float2 ex[N * PITCH];
    __shared__ float2 twl[N];    // [t][r][q]: second-stage twiddles w^{(q + R2 t) r}, w = e^{-2 pi i / N}
    const int tid = threadIdx.x;
    const int p = tid % P, q = tid / P;
    const int64_t g = (int64_t)blockIdx.x * P + p;
    const bool ok = g < a.plane;
    // 32-bit byte offsets within one array (the launcher checks that an array spans less than
    // 4 GiB): element (j, g) of an array is at j * pb + gb
    const uint32_t pb = (uint32_t)a.plane * (uint32_t)sizeof(float2), gb = (uint32_t)g * (uint32_t)sizeof(float2);
    for (int i = tid; i < N; i += P * R2) {
        const int t = i / (R2 * R2), r = i / R2 % R2, qq = i % R2;
        twl[i] = a.tw[((qq + R2 * t) * r) % N];
    }
    const int64_t kstride = (int64_t)a.np * a.plane;
    // kernel planes: uniform row pointers plus 32-bit lane offsets (R2 planes of a kernel span
    // under 4 GiB); the lower rows read plane j = q + R2 r, the upper ones plane pa + pb j at the
    // cell of k or, mirrored, of -k
    const uint32_t lane_lo = (uint32_t)q * pb + gb;
    const uint32_t lane_rev = (uint32_t)(R2 - 1 - q) * pb + gb;
    const uint32_t lane_mir =
        (uint32_t)(R2 - 1 - q) * pb + (uint32_t)((a.half && ok) ? mirror_cell(a.n1, a.n2, g) : g) * (uint32_t)sizeof(float2);
    auto load_kernel = [&](int64_t k, int grp, float2 *dst) {
        const float2 *kc = a.kc + k * kstride;
        const UpperPlanes up(a.half, SB_MIRROR_RULE(a, grp), a.np, N);
        // copies first: a conditional over the captured variables themselves would select their
        // addresses and keep them (and the whole capture) in scratch memory
        const uint32_t llo = lane_lo, lrev = lane_rev, lmir = lane_mir;
        const uint32_t lane_hi = up.pb > 0 ? llo : (up.mirrored ? lmir : lrev);
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            if (r > KR && r < R1 - KR) {
                dst[r] = make_float2(0.f, 0.f);
                continue;
            }
            const int j = q + R2 * r;
            if (2 * r < R1) {
                dst[r] = (ok && (j <= a.r0 || up.dense)) ? ld_stream(at_bytes(kc + (int64_t)(R2 * r) * a.plane, lane_lo))
                                                           : make_float2(0.f, 0.f);
            } else {
                const int p0 = up.pb > 0 ? up.pa + R2 * r : up.pa - R2 * r - (R2 - 1);   // lowest plane of the row
                const float2 v = (ok && (j >= N - a.r0 || up.dense)) ? ld_stream(at_bytes(kc + (int64_t)p0 * a.plane, lane_hi))
                                                                     : make_float2(0.f, 0.f);
                dst[r] = make_float2(up.sx * v.x, up.sy * v.y);
            }
        }
    };
    // one transform: radix-R1 DFT of the own rows, exchange, twiddle, radix-R2 DFTs -> own rows
    auto transform = [&](float2 *v, float2 *buf, auto sign_c) {
        constexpr int SIGN = decltype(sign_c)::value;
        Dft<R1, SIGN>::run(v);
        __syncthreads();                 // the previous exchange has been read
#pragma unroll
        for (int r = 0; r < R1; ++r) buf[(R1 * q + r) * PITCH + p] = v[r];
        __syncthreads();
#pragma unroll
        for (int t = 0; t < T; ++t) {
            float2 u[R2];
#pragma unroll
            for (int r = 0; r < R2; ++r) {
                const float2 x = buf[(q + R2 * t + R1 * r) * PITCH + p];
                const float2 tv = twl[(t * R2 + r) * R2 + q];     // the inverse takes the conjugate
                const float2 w = SIGN < 0 ? tv : make_float2(tv.x, -tv.y);
                u[r] = r == 0 ? x : cmul(x, w);
            }
            Dft<R2, SIGN>::run(u);
#pragma unroll
            for (int r = 0; r < R2; ++r) v[t + T * r] = u[r];   // element q + R2 t + R1 r
        }
    };
    float2 nx[R1];
    if constexpr (MODE == 1) {
        // adjoint: out += sum_b FFT_0(v_b) FFT_0(kernel b); bin b + 1 loads during bin b
        auto load_v = [&](int b, float2 *dst) {
            const float2 *vb = a.vin + (int64_t)b * a.ng;
#pragma unroll
            for (int r = 0; r < R1; ++r) dst[r] = ok ? *at_bytes(vb, (uint32_t)(q + R2 * r) * pb + gb) : make_float2(0.f, 0.f);
        };
        float2 acc[R1], nv[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r) acc[r] = make_float2(0.f, 0.f);
        const int nt = (a.accgroups > 1 ? a.accgroups : 1) * a.nb;   // (group, bin) steps
        load_v(0, nv);
        load_kernel(acc_kernel(a, 0), acc_group(a, 0), nx);
        for (int t = 0; t < nt; ++t) {
            float2 v[R1], k[R1];
#pragma unroll
            for (int r = 0; r < R1; ++r) { v[r] = nv[r]; k[r] = nx[r]; }
            if (t + 1 < nt) { load_v(t + 1, nv); load_kernel(acc_kernel(a, t + 1), acc_group(a, t + 1), nx); }
            transform(v, ex, std::integral_constant<int, -1>{});
            transform(k, ex, std::integral_constant<int, -1>{});
#pragma unroll
            for (int r = 0; r < R1; ++r) acc[r] = cadd(acc[r], cmul(v[r], k[r]));
            if (t % a.nb == a.nb - 1) {   // end of a group: out += its sum, as separate launches would
                if (ok)
#pragma unroll
                    for (int r = 0; r < R1; ++r) {
                        float2 *o = at_bytes(out0, (uint32_t)(q + R2 * r) * pb + gb);
                        *o = cadd(*o, acc[r]);
                    }
#pragma unroll
                for (int r = 0; r < R1; ++r) acc[r] = make_float2(0.f, 0.f);
            }
        }
        return;
    }
    float2 dr[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) dr[r] = ok ? *at_bytes(dhat0, (uint32_t)(q + R2 * r) * pb + gb) : make_float2(0.f, 0.f);
    const int64_t kbase = (int64_t)(a.kmap ? a.kmap[blockIdx.y] : blockIdx.y) * a.nb;   // kernel group
    const int kgrp = a.kgroup0 + (int)(a.kmap ? a.kmap[blockIdx.y] : blockIdx.y);       // its global index
    const int64_t obase = (int64_t)blockIdx.y * a.nb;                                 // output arrays
    load_kernel(kbase, kgrp, nx);
    for (int b = 0; b < a.nb; ++b) {
        float2 v[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r) v[r] = nx[r];
        if (b + 1 < a.nb) load_kernel(kbase + b + 1, kgrp, nx);   // in flight during the transforms
        transform(v, ex, std::integral_constant<int, -1>{});
#pragma unroll
        for (int r = 0; r < R1; ++r) v[r] = cmul(v[r], dr[r]);
        transform(v, ex, std::integral_constant<int, 1>{});
        float2 *out = out0 + (obase + b) * a.ng;
        if (ok)
#pragma unroll
            for (int r = 0; r < R1; ++r) st_stream(at_bytes(out, (uint32_t)(q + R2 * r) * pb + gb), v[r]);
    }
}

// Axis-0 correlation pass on the register-resident Stockham stages of reg_stages (any radix
// list whose last radix divides the first; two or more stages): thread q < T = n / R0 of a
// pencil owns rows q + T s.  P adjacent pencils of the contiguous axes per workgroup.
// KR as in axis0_reg_kernel: rows r <= KR and r >= R0 - KR of a thread are the only ones the
// compact kernel support can reach (KR >= R0 / 2: all rows).
template <int N, int P, int MODE, int KR, bool ONE, int R0, int... REST>
__global__ __launch_bounds__(P * (N / R0)) void axis0_rs_kernel(Axis0Args a) {
    // field of the launch (grid.z); local pointers, so the argument struct is never written
    const float2 *dhat0 = a.dhat + (int64_t)blockIdx.z * a.dhat_fs;
    float2 *out0 = a.out + (int64_t)blockIdx.z * a.out_fs;
    constexpr int T = N / R0;
    constexpr int PITCH = P + 1;
    __shared__ float2 ex[ONE ? 1 : 2][N * PITCH];   // ONE: a single exchange buffer
    float2 *ex1 = ex[ONE ? 0 : 1];
    __shared__ float2 tw[N];
    const int tid = threadIdx.x;
    const int p = tid % P, q = tid / P;
    const int64_t g = (int64_t)blockIdx.x * P + p;
    const bool ok = g < a.plane;
    // element q + T r of a pencil: the uniform row pointer of r plus the lane's 32-bit byte offset
    // (q plane + g) * 8 (under 4 GiB: q < T <= 128 and plane <= 2^20 cells, as the plan's edges are
    // at most 1024)
    const uint32_t lane_off = (uint32_t)(((int64_t)q * a.plane + g) * (int64_t)sizeof(float2));
    auto row = [&](const float2 *base, int r) { return base + (int64_t)(T * r) * a.plane; };
    for (int i = tid; i < N; i += P * T) tw[i] = a.tw[i];
    const int64_t kstride = (int64_t)a.np * a.plane;
    // kernel planes as in axis0_reg_kernel: the lower rows read plane j = q + T r, the upper ones
    // plane pa + pb j, from uniform row pointers plus 32-bit lane offsets
    const uint32_t kpb = (uint32_t)a.plane * (uint32_t)sizeof(float2);
    const uint32_t gbk = (uint32_t)g * (uint32_t)sizeof(float2);
    const uint32_t lane_lo = (uint32_t)q * kpb + gbk;
    const uint32_t lane_rev = (uint32_t)(T - 1 - q) * kpb + gbk;
    const uint32_t lane_mir =
        (uint32_t)(T - 1 - q) * kpb + (uint32_t)((a.half && ok) ? mirror_cell(a.n1, a.n2, g) : g) * (uint32_t)sizeof(float2);
    auto load_kernel = [&](int64_t k, int grp, float2 *dst) {
        const float2 *kc = a.kc + k * kstride;
        const UpperPlanes up(a.half, SB_MIRROR_RULE(a, grp), a.np, N);
        // copies first: a conditional over the captured variables themselves would select their
        // addresses and keep them (and the whole capture) in scratch memory
        const uint32_t llo = lane_lo, lrev = lane_rev, lmir = lane_mir;
        const uint32_t lane_hi = up.pb > 0 ? llo : (up.mirrored ? lmir : lrev);
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            if (r > KR && r < R0 - KR) {
                dst[r] = make_float2(0.f, 0.f);
                continue;
            }
            const int j = q + T * r;
            if (2 * r < R0) {
                dst[r] = (ok && (j <= a.r0 || up.dense)) ? ld_stream(at_bytes(kc + (int64_t)(T * r) * a.plane, lane_lo))
                                                           : make_float2(0.f, 0.f);
            } else {
                const int p0 = up.pb > 0 ? up.pa + T * r : up.pa - T * r - (T - 1);   // lowest plane of the row
                const float2 v = (ok && (j >= N - a.r0 || up.dense)) ? ld_stream(at_bytes(kc + (int64_t)p0 * a.plane, lane_hi))
                                                                     : make_float2(0.f, 0.f);
                dst[r] = make_float2(up.sx * v.x, up.sy * v.y);
            }
        }
    };
    float2 nx[R0];
    if constexpr (MODE == 1) {
        // adjoint: out += sum_b FFT_0(v_b) FFT_0(kernel b); bin b + 1 loads during bin b.  The
        // stage buffers alternate, so consecutive transforms need no barrier between them
        // (odd stage counts: the last stage reads the buffer the next first stage does not write).
        static_assert(sizeof...(REST) % 2 == 0, "odd number of stages");
        auto load_v = [&](int b, float2 *dst) {
            const float2 *vb = a.vin + (int64_t)b * a.ng;
#pragma unroll
            for (int r = 0; r < R0; ++r) dst[r] = ok ? *at_bytes(row(vb, r), lane_off) : make_float2(0.f, 0.f);
        };
        float2 acc[R0], nv[R0];
#pragma unroll
        for (int r = 0; r < R0; ++r) acc[r] = make_float2(0.f, 0.f);
        const int nt = (a.accgroups > 1 ? a.accgroups : 1) * a.nb;   // (group, bin) steps
        load_v(0, nv);
        load_kernel(acc_kernel(a, 0), acc_group(a, 0), nx);
        __syncthreads();   // twiddle table
        for (int t = 0; t < nt; ++t) {
            float2 v[R0], k[R0];
#pragma unroll
            for (int r = 0; r < R0; ++r) { v[r] = nv[r]; k[r] = nx[r]; }
            if (t + 1 < nt) { load_v(t + 1, nv); load_kernel(acc_kernel(a, t + 1), acc_group(a, t + 1), nx); }
            if constexpr (ONE) __syncthreads();   // the previous transform has read the buffer
            reg_stages<N, -1, R0, REST...>(v, ex[0], ex1, tw, q, p, PITCH);
            if constexpr (ONE) __syncthreads();
            reg_stages<N, -1, R0, REST...>(k, ex[0], ex1, tw, q, p, PITCH);
#pragma unroll
            for (int r = 0; r < R0; ++r) acc[r] = cadd(acc[r], cmul(v[r], k[r]));
            if (t % a.nb == a.nb - 1) {   // end of a group: out += its sum, as separate launches would
                if (ok)
#pragma unroll
                    for (int r = 0; r < R0; ++r) {
                        float2 *o = at_bytes(const_cast<float2 *>(row(out0, r)), lane_off);
                        *o = cadd(*o, acc[r]);
                    }
#pragma unroll
                for (int r = 0; r < R0; ++r) acc[r] = make_float2(0.f, 0.f);
            }
        }
        return;
    }
    float2 dr[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) dr[r] = ok ? *at_bytes(row(dhat0, r), lane_off) : make_float2(0.f, 0.f);
    const int64_t kbase = (int64_t)(a.kmap ? a.kmap[blockIdx.y] : blockIdx.y) * a.nb;   // kernel group
    const int kgrp = a.kgroup0 + (int)(a.kmap ? a.kmap[blockIdx.y] : blockIdx.y);       // its global index
    const int64_t obase = (int64_t)blockIdx.y * a.nb;                                 // output arrays
    load_kernel(kbase, kgrp, nx);
    __syncthreads();   // twiddle table
    for (int b = 0; b < a.nb; ++b) {
        float2 v[R0];
#pragma unroll
        for (int r = 0; r < R0; ++r) v[r] = nx[r];
        if (b + 1 < a.nb) load_kernel(kbase + b + 1, kgrp, nx);   // in flight during the transforms
        if constexpr (ONE) __syncthreads();   // the previous transform has read the buffer
        reg_stages<N, -1, R0, REST...>(v, ex[0], ex1, tw, q, p, PITCH);
#pragma unroll
        for (int r = 0; r < R0; ++r) v[r] = cmul(v[r], dr[r]);
        if constexpr (ONE) __syncthreads();
        reg_stages<N, 1, R0, REST...>(v, ex[0], ex1, tw, q, p, PITCH);
        float2 *out = out0 + (obase + b) * a.ng;
        if (ok)
#pragma unroll
            for (int r = 0; r < R0; ++r) st_stream(at_bytes(const_cast<float2 *>(row(out, r)), lane_off), v[r]);
    }
}

template <int N, int TPP, int NT, int... RAD>
hipError_t launch_axis0_t(const Axis0Args &a, hipStream_t s) {
    constexpr int P = NT / TPP;
    dim3 grid((unsigned)((a.plane + P - 1) / P), (unsigned)a.groups, (unsigned)(a.fields > 1 ? a.fields : 1));
    hipLaunchKernelGGL((axis0_kernel<N, TPP, NT, RAD...>), grid, dim3(NT), 0, s, a);
    return hipGetLastError();
}

// Persistent form of the plain pass (complex in, complex out): a workgroup walks
// `tiles` consecutive tiles and loads tile t + 1 into registers while tile t is
// transformed, so the memory pipe stays busy across the LDS stages.
template <int N, int TPP, int NT, int SIGN, int... RAD>
__global__ __launch_bounds__(NT) void fft_pass_pf_kernel(FftPass a, int tiles) {
    constexpr int P = NT / TPP;
    constexpr int PITCH = P + 1;
    constexpr int EPT = N / TPP;
    __shared__ float2 sm[N * PITCH];
    __shared__ float2 tw[N];
    const int tid = threadIdx.x;
    const int y = blockIdx.y;
    const int64_t npencil = a.ng / N;
    const int64_t ntile = (npencil + P - 1) / P;
    const float2 *in = reinterpret_cast<const float2 *>(a.in) + y * a.in_bs;
    float2 *out = a.out + y * a.out_bs;
    for (int i = tid; i < N; i += NT) tw[i] = a.tw[i];
    const bool rows = a.stride == 1;
    // element e of thread tid: f = tid + e NT -> (pencil, column) by the coalesced pattern
    auto elem = [&](int e, int &p, int &j) {
        const int f = tid + e * NT;
        if (rows) { p = f / N; j = f % N; } else { p = f % P; j = f / P; }
    };
    auto addr = [&](int64_t g, int j) -> int64_t {
        return (g / a.stride) * (int64_t)N * a.stride + (g % a.stride) + (int64_t)j * a.stride;
    };
    const int64_t t0 = (int64_t)blockIdx.x * tiles;
    const int64_t t1 = min(t0 + tiles, ntile);
    float2 nx[EPT];
    auto load = [&](int64_t t) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            int p, j;
            elem(e, p, j);
            const int64_t g = t * P + p;
            nx[e] = g < npencil ? in[addr(g, j)] : make_float2(0.f, 0.f);
        }
    };
    if (t0 < t1) load(t0);
    for (int64_t t = t0; t < t1; ++t) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            int p, j;
            elem(e, p, j);
            sm[j * PITCH + p] = nx[e];
        }
        if (t + 1 < t1) load(t + 1);
        __syncthreads();
        stages<N, TPP, SIGN, 1, RAD...>(sm, tw, tid % P, tid / P, PITCH);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            int p, j;
            elem(e, p, j);
            const int64_t g = t * P + p;
            if (g < npencil) st_stream(&out[addr(g, j)], sm[j * PITCH + p]);
        }
    }
}

// Register-resident pass along a strided axis for n = R1 * R2 (R2 divides R1): P adjacent
// pencils of the faster axes per tile (16, 32 or 64: rows of 128, 256 or 512 contiguous bytes),
// thread q < R2 of a pencil owns elements q + R2 s (the inputs of first-stage butterfly q and the
// outputs of second-stage butterflies q + R2 t), so loads and stores are coalesced over the P
// pencils and LDS holds only the one exchange between the two radix stages (130 KB at n = 256,
// P = 64: one 1024-thread workgroup per CU).  A workgroup walks `tiles` consecutive tiles with
// the next one's loads in flight.
template <int R1, int R2, int P, int SIGN>
__global__ __launch_bounds__(P * R2, 3) void mid_reg_kernel(FftPass a, int tiles) {
    constexpr int N = R1 * R2;
    constexpr int T = R1 / R2;   // second-stage butterflies per thread
    static_assert(R1 % R2 == 0, "R2 must divide R1");
    constexpr int PITCH = P + 1;
    __shared__ float2 ex[N * PITCH];
    __shared__ float2 twl[N];    // [t][r][q]: second-stage twiddles w^{(q + R2 t) r}, w = e^{-2 pi i / N}
    const int tid = threadIdx.x;
    const int p = tid % P, q = tid / P;
    for (int i = tid; i < N; i += P * R2) {
        const int t = i / (R2 * R2), r = i / R2 % R2, qq = i % R2;
        twl[i] = a.tw[((qq + R2 * t) * r) % N];
    }
    const int64_t npencil = a.ng / N;
    const int64_t ntile = (npencil + P - 1) / P;
    const float2 *in = reinterpret_cast<const float2 *>(a.in) + blockIdx.y * a.in_bs;
    float2 *out = a.out + blockIdx.y * a.out_bs;
    // P divides the stride, so a tile's pencils share one uniform base; a lane addresses element
    // j of its pencil as the uniform row pointer of j plus its own 32-bit byte offset (the
    // launcher checks that n * stride elements span less than 4 GiB)
    auto tile_base = [&](int64_t t) -> int64_t {
        const int64_t g0 = t * P;
        return (g0 / a.stride) * (int64_t)N * a.stride + (g0 % a.stride);
    };
    const uint32_t es = (uint32_t)a.stride * (uint32_t)sizeof(float2);   // bytes between elements
    const uint32_t lane_off = (uint32_t)p * (uint32_t)sizeof(float2) + (uint32_t)q * es;
    const int64_t t0 = (int64_t)blockIdx.x * tiles;
    const int64_t t1 = min(t0 + tiles, ntile);
    float2 nx[R1];
    auto load = [&](int64_t t) {
        const float2 *tin = in + tile_base(t);
        const bool ok = t * P + p < npencil;
#pragma unroll
        for (int r = 0; r < R1; ++r)   // element q + R2 r
            nx[r] = ok ? ld_stream(at_bytes(at_bytes(tin, (uint32_t)(R2 * r) * es), lane_off)) : make_float2(0.f, 0.f);
    };
    if (t0 < t1) load(t0);
    for (int64_t t = t0; t < t1; ++t) {
        float2 v[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r) v[r] = nx[r];
        if (t + 1 < t1) load(t + 1);   // in flight during the transform
        Dft<R1, SIGN>::run(v);
        __syncthreads();                 // the previous tile's exchange has been read
#pragma unroll
        for (int r = 0; r < R1; ++r) ex[(R1 * q + r) * PITCH + p] = v[r];
        __syncthreads();
        const bool ok = t * P + p < npencil;
        float2 *tout = out + tile_base(t);
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
            float2 u[R2];
#pragma unroll
            for (int r = 0; r < R2; ++r) {
                const float2 x = ex[(q + R2 * tt + R1 * r) * PITCH + p];
                const float2 tv = twl[(tt * R2 + r) * R2 + q];   // the inverse takes the conjugate
                const float2 w = SIGN < 0 ? tv : make_float2(tv.x, -tv.y);
                u[r] = r == 0 ? x : cmul(x, w);
            }
            Dft<R2, SIGN>::run(u);
            if (ok)
#pragma unroll
                for (int r = 0; r < R2; ++r)   // element q + R2 (tt + T r)
                    st_stream(at_bytes(at_bytes(tout, (uint32_t)(R2 * (tt + T * r)) * es), lane_off), u[r]);
        }
    }
}

// The same for the three-stage radix lists (reg_stages): thread q < T = n / R0 of a pencil owns
// elements q + T s, the stages exchange through one LDS buffer (two barriers per exchange), so
// that two 512-thread workgroups share a CU.  P divides
// the stride, so a tile's pencils share one uniform base and a lane addresses its elements by
// 32-bit byte offsets from it (the launcher checks that n * stride elements span less than 4 GiB).
template <int N, int P, int SIGN, bool PF, int R0, int... REST>
__global__ __launch_bounds__(P * (N / R0), 4) void mid_rs_kernel(FftPass a, int tiles) {
    constexpr int T = N / R0;
    constexpr int PITCH = P + 1;
    __shared__ float2 ex[N * PITCH];
    __shared__ float2 tw[N];
    const int tid = threadIdx.x;
    const int p = tid % P, q = tid / P;
    for (int i = tid; i < N; i += P * T) tw[i] = a.tw[i];
    const int64_t npencil = a.ng / N;
    const int64_t ntile = (npencil + P - 1) / P;
    const float2 *in = reinterpret_cast<const float2 *>(a.in) + blockIdx.y * a.in_bs;
    float2 *out = a.out + blockIdx.y * a.out_bs;
    // first element of tile t (pencils t P .. t P + P - 1, adjacent along the faster axes)
    auto tile_base = [&](int64_t t) -> int64_t {
        const int64_t g0 = t * P;
        return (g0 / a.stride) * (int64_t)N * a.stride + (g0 % a.stride);
    };
    const uint32_t es = (uint32_t)a.stride * (uint32_t)sizeof(float2);        // bytes between elements
    const uint32_t lane_off = (uint32_t)p * (uint32_t)sizeof(float2) + (uint32_t)q * es;
    const int64_t t0 = (int64_t)blockIdx.x * tiles;
    const int64_t t1 = min(t0 + tiles, ntile);
    // element q + T r of a tile: the uniform row pointer of r plus the lane's offset
    auto load = [&](int64_t t, float2 *dst) {
        const float2 *tin = in + tile_base(t);
        const bool ok = t * P + p < npencil;
#pragma unroll
        for (int r = 0; r < R0; ++r)
            dst[r] = ok ? ld_stream(at_bytes(at_bytes(tin, (uint32_t)(T * r) * es), lane_off)) : make_float2(0.f, 0.f);
    };
    // PF: the next tile's loads are in flight during the transform; otherwise the other
    // workgroup's waves cover the load latency
    float2 nx[PF ? R0 : 1];
    if (PF && t0 < t1) load(t0, nx);
    for (int64_t t = t0; t < t1; ++t) {
        const bool ok = t * P + p < npencil;
        float2 v[R0];
        if constexpr (PF) {
#pragma unroll
            for (int r = 0; r < R0; ++r) v[r] = nx[r];
            if (t + 1 < t1) load(t + 1, nx);
        } else {
            load(t, v);
        }
        __syncthreads();                 // the previous tile's last stage has read the buffer
        reg_stages<N, SIGN, R0, REST...>(v, ex, ex, tw, q, p, PITCH);
        if (ok) {
            float2 *tout = out + tile_base(t);
#pragma unroll
            for (int r = 0; r < R0; ++r) st_stream(at_bytes(at_bytes(tout, (uint32_t)(T * r) * es), lane_off), v[r]);
        }
    }
}

template <int R1, int R2, int P>
hipError_t launch_mid_reg(const FftPass &a, hipStream_t s, int tiles) {
    constexpr int N = R1 * R2;
    const int64_t ntile = (a.ng / N + P - 1) / P;
    dim3 grid((unsigned)((ntile + tiles - 1) / tiles), (unsigned)a.batch);
    if (a.sign < 0) hipLaunchKernelGGL((mid_reg_kernel<R1, R2, P, -1>), grid, dim3(P * R2), 0, s, a, tiles);
    else hipLaunchKernelGGL((mid_reg_kernel<R1, R2, P, 1>), grid, dim3(P * R2), 0, s, a, tiles);
    return hipGetLastError();
}

template <int N, int TPP, int NT, int... RAD>
hipError_t launch_pf(const FftPass &a, hipStream_t s, int tiles) {
    constexpr int P = NT / TPP;
    const int64_t ntile = (a.ng / N + P - 1) / P;
    dim3 grid((unsigned)((ntile + tiles - 1) / tiles), (unsigned)a.batch);
    if (a.sign < 0)
        hipLaunchKernelGGL((fft_pass_pf_kernel<N, TPP, NT, -1, RAD...>), grid, dim3(NT), 0, s, a, tiles);
    else
        hipLaunchKernelGGL((fft_pass_pf_kernel<N, TPP, NT, 1, RAD...>), grid, dim3(NT), 0, s, a, tiles);
    return hipGetLastError();
}

template <int N, int TPP, int NT, int... RAD>
hipError_t launch(const FftPass &a, hipStream_t s) {
    constexpr int P = NT / TPP;
    const int64_t npencil = a.ng / N;
    dim3 grid((unsigned)((npencil + P - 1) / P), (unsigned)a.batch);
    if (a.sign < 0)
        hipLaunchKernelGGL((fft_pass_kernel<N, TPP, NT, -1, RAD...>), grid, dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL((fft_pass_kernel<N, TPP, NT, 1, RAD...>), grid, dim3(NT), 0, s, a);
    return hipGetLastError();
}

}  // namespace

// Per-length launch shapes: (threads per pencil, workgroup threads, radices).
// The variants are the autotuner's candidates.
hipError_t launch_fft_pass(const FftPass &a, hipStream_t s) {
    const int v = a.variant;
    // variants 6 to 9 (lengths 64, 128, 256 along a strided axis whose stride is a multiple of
    // 16): register-resident; 6: tiles of 32 pencils (16 if the stride is not a multiple of 32),
    // 8 per workgroup, 7: 16 pencils, 16 per workgroup; 8 and 9: 64 pencils (rows of 512
    // contiguous bytes; 32 or 16 where the stride allows no more), 8 and 4 tiles per workgroup.
    // Elsewhere they run as variants 4 and 5.
    // (the register-resident kernels address a tile's n * stride elements by 32-bit byte offsets,
    // so those must span less than 4 GiB)
    const bool off32 = (int64_t)a.n * a.stride * (int64_t)sizeof(float2) <= (int64_t)UINT32_MAX;
    if (v >= 6 && a.load == LOAD_C && a.store == STORE_C && a.stride > 1 && a.stride % 16 == 0 && off32) {
        const bool x64 = v >= 8 && a.stride % 64 == 0;
        const bool wide = v != 7 && a.stride % 32 == 0;
        const int tiles = v == 7 ? 16 : (v == 9 ? 4 : 8);
        if (a.n == 256)
            return x64 ? launch_mid_reg<16, 16, 64>(a, s, tiles)
                       : wide ? launch_mid_reg<16, 16, 32>(a, s, tiles) : launch_mid_reg<16, 16, 16>(a, s, tiles);
        if (a.n == 128)
            return x64 ? launch_mid_reg<16, 8, 64>(a, s, tiles)
                       : wide ? launch_mid_reg<16, 8, 32>(a, s, tiles) : launch_mid_reg<16, 8, 16>(a, s, tiles);
        if (a.n == 64)
            return x64 ? launch_mid_reg<8, 8, 64>(a, s, tiles)
                       : wide ? launch_mid_reg<8, 8, 32>(a, s, tiles) : launch_mid_reg<8, 8, 16>(a, s, tiles);
        if (a.n == 512) {
            constexpr int P = 16;
            const int64_t ntile = (a.ng / 512 + P - 1) / P;
            dim3 grid((unsigned)((ntile + tiles - 1) / tiles), (unsigned)a.batch);
            // variant 7 keeps the next tile's loads in flight
            if (v == 6) {
                if (a.sign < 0) hipLaunchKernelGGL((mid_rs_kernel<512, P, -1, false, 16, 8, 4>), grid, dim3(32 * P), 0, s, a, tiles);
                else hipLaunchKernelGGL((mid_rs_kernel<512, P, 1, false, 16, 8, 4>), grid, dim3(32 * P), 0, s, a, tiles);
            } else {
                if (a.sign < 0) hipLaunchKernelGGL((mid_rs_kernel<512, P, -1, true, 16, 8, 4>), grid, dim3(32 * P), 0, s, a, tiles);
                else hipLaunchKernelGGL((mid_rs_kernel<512, P, 1, true, 16, 8, 4>), grid, dim3(32 * P), 0, s, a, tiles);
            }
            return hipGetLastError();
        }
        if (a.n == 96 || a.n == 160 || a.n == 192) {
            // three-stage forms (96 = 12 x 4 x 2, 160 = 20 x 4 x 2, 192 = 12 x 4 x 4): 32 pencils
            // (16 where the stride allows no more) for 6, 16 for 7, 64 (or fewer) for 8 and 9;
            // variant 9 keeps the next tile's loads in flight
            const int pw = v == 7 ? 16 : (v >= 8 && a.stride % 64 == 0) ? 64 : a.stride % 32 == 0 ? 32 : 16;
            auto go = [&](auto p_c, auto pf_c) {
                constexpr int P = decltype(p_c)::value;
                constexpr bool PF = decltype(pf_c)::value;
                const int64_t ntile = (a.ng / a.n + P - 1) / P;
                dim3 grid((unsigned)((ntile + tiles - 1) / tiles), (unsigned)a.batch);
                auto l3 = [&](auto kern, int t) { hipLaunchKernelGGL(kern, grid, dim3(P * t), 0, s, a, tiles); };
                if (a.n == 96) {
                    if (a.sign < 0) l3(mid_rs_kernel<96, P, -1, PF, 12, 4, 2>, 8);
                    else l3(mid_rs_kernel<96, P, 1, PF, 12, 4, 2>, 8);
                } else if (a.n == 160) {
                    constexpr bool PF160 = PF && P > 16;   // 16 pencils with the prefetch would spill
                    if (a.sign < 0) l3(mid_rs_kernel<160, P, -1, PF160, 20, 4, 2>, 8);
                    else l3(mid_rs_kernel<160, P, 1, PF160, 20, 4, 2>, 8);
                } else {
                    if (a.sign < 0) l3(mid_rs_kernel<192, P, -1, PF, 12, 4, 4>, 16);
                    else l3(mid_rs_kernel<192, P, 1, PF, 12, 4, 4>, 16);
                }
            };
            using T_ = std::true_type;
            using F_ = std::false_type;
            if (pw == 64) {
                if (v == 9) go(std::integral_constant<int, 64>{}, T_{});
                else go(std::integral_constant<int, 64>{}, F_{});
            } else if (pw == 32) {
                if (v == 9) go(std::integral_constant<int, 32>{}, T_{});
                else go(std::integral_constant<int, 32>{}, F_{});
            } else {
                if (v == 9) go(std::integral_constant<int, 16>{}, T_{});
                else go(std::integral_constant<int, 16>{}, F_{});
            }
            return hipGetLastError();
        }
        if (a.n == 1024) {
            // 16 x 16 x 4 in registers, 64 threads per pencil: 16 pencils (1024 threads, 139 KB of LDS)
            // for variant 6, 8 pencils (512 threads) for variant 7
            auto go = [&](auto p_c) {
                constexpr int P = decltype(p_c)::value;
                const int64_t ntile = (a.ng / 1024 + P - 1) / P;
                dim3 grid((unsigned)((ntile + tiles - 1) / tiles), (unsigned)a.batch);
                if (a.sign < 0) hipLaunchKernelGGL((mid_rs_kernel<1024, P, -1, false, 16, 16, 4>), grid, dim3(64 * P), 0, s, a, tiles);
                else hipLaunchKernelGGL((mid_rs_kernel<1024, P, 1, false, 16, 16, 4>), grid, dim3(64 * P), 0, s, a, tiles);
            };
            if (v == 6) go(std::integral_constant<int, 16>{});
            else go(std::integral_constant<int, 8>{});
            return hipGetLastError();
        }
    }
    // variants 4 and 5: persistent with few, wide radix stages (64: 8 x 8, 96: 12 x 4 x 2,
    // 128: 16 x 8, 160: 20 x 4 x 2, 192: 12 x 4 x 4, 256: 16 x 16), 4 / 16 tiles
    if (v >= 4 && a.load == LOAD_C && a.store == STORE_C) {
        const int tiles = v % 2 == 0 ? 4 : 16;
        if (a.n == 256) return launch_pf<256, 16, 256, 16, 16>(a, s, tiles);
        if (a.n == 128) return launch_pf<128, 8, 256, 16, 8>(a, s, tiles);
        if (a.n == 64) return launch_pf<64, 8, 256, 8, 8>(a, s, tiles);
        if (a.n == 192) return launch_pf<192, 16, 256, 12, 4, 4>(a, s, tiles);
        if (a.n == 160) return launch_pf<160, 8, 256, 20, 4, 2>(a, s, tiles);
        if (a.n == 96) return launch_pf<96, 8, 256, 12, 4, 2>(a, s, tiles);
    }
    // variants 2 and 3: persistent passes with register prefetch (plain loads and stores only)
    if (v >= 2 && a.load == LOAD_C && a.store == STORE_C) {
        const int tiles = v == 2 ? 4 : 16;
        switch (a.n) {
#define SB_X(N, TPP, NT, ...) case N: return launch_pf<N, TPP, NT, __VA_ARGS__>(a, s, tiles);
            SB_FFT_CONFIGS(SB_X)
#undef SB_X
            default: return hipErrorInvalidValue;
        }
    }
    switch (a.n) {
        case 8: return launch<8, 1, 64, 8>(a, s);
        case 12: return launch<12, 1, 64, 4, 3>(a, s);
        case 16: return launch<16, 4, 64, 4, 4>(a, s);
        case 24: return launch<24, 2, 128, 4, 2, 3>(a, s);
        case 32: return v == 1 ? launch<32, 4, 128, 4, 8>(a, s) : launch<32, 4, 64, 4, 8>(a, s);
        case 48: return launch<48, 4, 64, 4, 4, 3>(a, s);
        case 64: return v == 1 ? launch<64, 4, 64, 8, 8>(a, s) : launch<64, 8, 128, 8, 8>(a, s);
        case 96: return v == 1 ? launch<96, 4, 128, 4, 8, 3>(a, s) : launch<96, 4, 64, 4, 8, 3>(a, s);
        case 128: return v == 1 ? launch<128, 8, 128, 8, 8, 2>(a, s) : launch<128, 16, 256, 8, 8, 2>(a, s);
        case 160: return v == 1 ? launch<160, 4, 128, 4, 8, 5>(a, s) : launch<160, 4, 64, 4, 8, 5>(a, s);
        case 192: return launch<192, 8, 128, 8, 8, 3>(a, s);
        case 256: return v == 1 ? launch<256, 32, 256, 8, 8, 4>(a, s) : launch<256, 16, 256, 8, 8, 4>(a, s);
        case 512: return v == 1 ? launch<512, 64, 256, 8, 8, 8>(a, s) : launch<512, 32, 256, 8, 8, 8>(a, s);
        case 1024: return v == 1 ? launch<1024, 128, 512, 8, 8, 4, 4>(a, s) : launch<1024, 64, 256, 16, 16, 4>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_axis0(const Axis0Args &a, hipStream_t s) {
    if (a.n == 1024 && a.mode == 0) {
        // 8 x 8 x 4 x 4 in registers, 128 threads per pencil (8 elements each, which leaves room
        // for the density spectrum), 8 pencils (rows of 64 contiguous bytes) per 1024-thread
        // workgroup, one exchange buffer (74 KB of LDS)
        constexpr int P = 8;
        dim3 grid((unsigned)((a.plane + P - 1) / P), (unsigned)a.groups, (unsigned)(a.fields > 1 ? a.fields : 1));
        const int kr = support_rows(a, 8, 128);
        if (kr <= 1) hipLaunchKernelGGL((axis0_rs_kernel<1024, P, 0, 1, true, 8, 8, 4, 4>), grid, dim3(128 * P), 0, s, a);
        else if (kr <= 2) hipLaunchKernelGGL((axis0_rs_kernel<1024, P, 0, 2, true, 8, 8, 4, 4>), grid, dim3(128 * P), 0, s, a);
        else hipLaunchKernelGGL((axis0_rs_kernel<1024, P, 0, 8, true, 8, 8, 4, 4>), grid, dim3(128 * P), 0, s, a);
        return hipGetLastError();
    }
    if ((a.n == 512 && a.mode == 0) || a.n == 192 || a.n == 160 || a.n == 96) {
        // register-resident stages: 512 = 16 x 8 x 4, 192 = 12 x 4 x 4, 160 = 20 x 4 x 2, 96 = 12 x 4 x 2
        // (the adjoint accumulation at 512 keeps the LDS-staged kernel: its registers would spill)
        constexpr int P = 16;
        dim3 grid((unsigned)((a.plane + P - 1) / P), (unsigned)a.groups, (unsigned)(a.fields > 1 ? a.fields : 1));
        auto go = [&](auto mode_c) {
            constexpr int M = decltype(mode_c)::value;
            if constexpr (M == 0) {
                if (a.n == 512) {
                    const int kr = support_rows(a, 16, 32);
                    if (kr <= 1) hipLaunchKernelGGL((axis0_rs_kernel<512, P, 0, 1, false, 16, 8, 4>), grid, dim3(32 * P), 0, s, a);
                    else if (kr <= 2) hipLaunchKernelGGL((axis0_rs_kernel<512, P, 0, 2, false, 16, 8, 4>), grid, dim3(32 * P), 0, s, a);
                    else hipLaunchKernelGGL((axis0_rs_kernel<512, P, 0, 16, false, 16, 8, 4>), grid, dim3(32 * P), 0, s, a);
                    return;
                }
            }
            // rows of a thread that the compact support can reach: KR = 2 where it allows (r0 below
            // about a tenth of the axis), all rows otherwise.  One exchange buffer (one more barrier
            // per exchange): with two, the LDS (27-54 KB per workgroup) held these lengths to 2-5
            // workgroups per CU, below what their registers allow
            if (a.n == 192) {
                if (support_rows(a, 12, 16) <= 2) hipLaunchKernelGGL((axis0_rs_kernel<192, P, M, 2, true, 12, 4, 4>), grid, dim3(16 * P), 0, s, a);
                else hipLaunchKernelGGL((axis0_rs_kernel<192, P, M, 12, true, 12, 4, 4>), grid, dim3(16 * P), 0, s, a);
            } else if (a.n == 160) {
                if (support_rows(a, 20, 8) <= 2) hipLaunchKernelGGL((axis0_rs_kernel<160, P, M, 2, true, 20, 4, 2>), grid, dim3(8 * P), 0, s, a);
                else hipLaunchKernelGGL((axis0_rs_kernel<160, P, M, 20, true, 20, 4, 2>), grid, dim3(8 * P), 0, s, a);
            } else {
                if (support_rows(a, 12, 8) <= 2) hipLaunchKernelGGL((axis0_rs_kernel<96, P, M, 2, true, 12, 4, 2>), grid, dim3(8 * P), 0, s, a);
                else hipLaunchKernelGGL((axis0_rs_kernel<96, P, M, 12, true, 12, 4, 2>), grid, dim3(8 * P), 0, s, a);
            }
        };
        if (a.mode == 1) go(std::integral_constant<int, 1>{});
        else go(std::integral_constant<int, 0>{});
        return hipGetLastError();
    }
    // the register-resident kernels of 64-256 address an array by 32-bit byte offsets
    if ((a.n == 256 || a.n == 128 || a.n == 64) && a.ng * (int64_t)sizeof(float2) <= (int64_t)UINT32_MAX) {
        constexpr int P = 16;
        dim3 grid((unsigned)((a.plane + P - 1) / P), (unsigned)a.groups, (unsigned)(a.fields > 1 ? a.fields : 1));
        auto go = [&](auto mode_c) {
            constexpr int M = decltype(mode_c)::value;
            if (a.n == 256) {
                const int kr = support_rows(a, 16, 16);
                if (kr <= 2) hipLaunchKernelGGL((axis0_reg_kernel<16, 16, P, M, 2>), grid, dim3(16 * P), 0, s, a);
                else if (kr <= 3) hipLaunchKernelGGL((axis0_reg_kernel<16, 16, P, M, 3>), grid, dim3(16 * P), 0, s, a);
                else hipLaunchKernelGGL((axis0_reg_kernel<16, 16, P, M, 16>), grid, dim3(16 * P), 0, s, a);
            } else if (a.n == 128) {
                const int kr = support_rows(a, 16, 8);
                if (kr <= 3) hipLaunchKernelGGL((axis0_reg_kernel<16, 8, P, M, 3>), grid, dim3(8 * P), 0, s, a);
                else if (kr <= 4) hipLaunchKernelGGL((axis0_reg_kernel<16, 8, P, M, 4>), grid, dim3(8 * P), 0, s, a);
                else hipLaunchKernelGGL((axis0_reg_kernel<16, 8, P, M, 16>), grid, dim3(8 * P), 0, s, a);
            } else {
                hipLaunchKernelGGL((axis0_reg_kernel<8, 8, P, M, 8>), grid, dim3(8 * P), 0, s, a);
            }
        };
        if (a.mode == 1) go(std::integral_constant<int, 1>{});
        else go(std::integral_constant<int, 0>{});
        return hipGetLastError();
    }
    switch (a.n) {
#define SB_X(N, TPP, NT, ...) case N: return launch_axis0_t<N, TPP, NT, __VA_ARGS__>(a, s);
        SB_FUSED_CONFIGS(SB_X)
#undef SB_X
        default: return hipErrorInvalidValue;
    }
}

int fused_last_rows(int n, int nb) {
    switch (n) {
#define SB_X(N, TPP, ...) case N: return last_rows<N>(nb);
        SB_LAST_CONFIGS(SB_X)
#undef SB_X
        default: return 0;
    }
}

hipError_t launch_last_contract(const LastArgs &a, hipStream_t s) {
    switch (a.n) {
#define SB_X(N, TPP, ...) case N: return launch_last_for<N>(a, s);
        SB_LAST_CONFIGS(SB_X)
#undef SB_X
        default: return hipErrorInvalidValue;
    }
}

bool fft_supported(int n) {
    switch (n) {
        case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 96:
        case 128: case 160: case 192: case 256: case 512: case 1024: return true;
        default: return false;
    }
}

int fft_num_variants(int n) {
    // 0, 1: one tile per workgroup (two shapes where defined); 2, 3: persistent, 4 / 16 tiles;
    // 4, 5 (lengths 64-256): persistent with few, wide radix stages; 6 to 9 (64 - 256; 6, 7 at
    // 512 and 1024): register-resident along a strided axis
    if (n == 256 || n == 128 || n == 64 || n == 192 || n == 160 || n == 96) return 10;
    if (n == 512 || n == 1024) return 8;
    return 4;
}

}  // namespace sb
