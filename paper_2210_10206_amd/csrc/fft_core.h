// Mixed-radix Stockham FFT building blocks for gfx950 (shared by the FFT translation units).
//
// A launch transforms every pencil of one axis of a batch of C-ordered complex
// arrays.  A workgroup owns P pencils: it stages them in LDS (coalesced: P
// adjacent pencils along the fastest axis for a strided axis, P whole rows for
// the contiguous axis), runs the radix stages in LDS with TPP threads per
// pencil, and writes the tile back.  Loads can fuse the spectral product
// (delta_hat * kernel_hat) or read a real field; stores can fuse a spectral
// multiply-accumulate.  Twiddles come from a float64-computed table of the n-th
// roots of unity, so every twiddle is correctly rounded to float32.
//
// Stockham autosort (decimation in time): with the radices R_0..R_{S-1} and
// Ns = R_0 * .. * R_{s-1}, stage s takes butterfly k in [0, n/R) from
// x[k + r n/R], multiplies input r by w^{(k mod Ns) r} with w = e^{sign 2 pi i/(Ns R)},
// applies the R-point DFT and writes output r to (k div Ns) Ns R + (k mod Ns) + r Ns.
// The result is in natural order.
#pragma once
#include "sb_common.h"

namespace sb {
namespace fftcore {

template <int SIGN>
__device__ __forceinline__ float2 mul_i(float2 a) {  // a * (SIGN * i)
    return SIGN < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

template <int R, int SIGN> struct Dft;

template <int SIGN> struct Dft<2, SIGN> {
    __device__ __forceinline__ static void run(float2 *v) {
        float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <int SIGN> struct Dft<3, SIGN> {
    __device__ __forceinline__ static void run(float2 *v) {
        const float s3 = 0.86602540378443864676f;  // sin(2 pi / 3)
        float2 t1 = cadd(v[1], v[2]);
        float2 t2 = csub(v[1], v[2]);
        float2 y0 = cadd(v[0], t1);
        float2 t = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
        float2 u = mul_i<SIGN>(cscale(t2, s3));
        v[0] = y0;
        v[1] = cadd(t, u);
        v[2] = csub(t, u);
    }
};

template <int SIGN> struct Dft<4, SIGN> {
    __device__ __forceinline__ static void run(float2 *v) {
        float2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
        float2 c = cadd(v[1], v[3]), d = mul_i<SIGN>(csub(v[1], v[3]));
        v[0] = cadd(a, c);
        v[2] = csub(a, c);
        v[1] = cadd(b, d);
        v[3] = csub(b, d);
    }
};

template <int SIGN> struct Dft<5, SIGN> {
    __device__ __forceinline__ static void run(float2 *v) {
        const float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
        const float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
        const float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
        const float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
        float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
        float2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
        float2 y0 = cadd(v[0], cadd(t1, t2));
        float2 a1 = make_float2(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
        float2 a2 = make_float2(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
        float2 b1 = mul_i<SIGN>(make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y));
        float2 b2 = mul_i<SIGN>(make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y));
        v[0] = y0;
        v[1] = cadd(a1, b1);
        v[4] = csub(a1, b1);
        v[2] = cadd(a2, b2);
        v[3] = csub(a2, b2);
    }
};

template <int SIGN> struct Dft<8, SIGN> {
    // Radix-2 split into two 4-point DFTs of the even and odd inputs.
    __device__ __forceinline__ static void run(float2 *v) {
        const float r = 0.70710678118654752440f;
        float2 e[4] = {v[0], v[2], v[4], v[6]};
        float2 o[4] = {v[1], v[3], v[5], v[7]};
        Dft<4, SIGN>::run(e);
        Dft<4, SIGN>::run(o);
        // w8^k = e^{SIGN 2 pi i k / 8}
        float2 o1 = cmul(o[1], make_float2(r, SIGN * r));
        float2 o2 = mul_i<SIGN>(o[2]);
        float2 o3 = cmul(o[3], make_float2(-r, SIGN * r));
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);
        v[7] = csub(e[3], o3);
    }
};

template <int SIGN> struct Dft<16, SIGN> {
    // 4 x 4 split (decimation in time): n = 4 n1 + n2, k = k1 + 4 k2; 4-point DFTs over n1,
    // twiddles w16^{n2 k1}, 4-point DFTs over n2.
    __device__ __forceinline__ static void run(float2 *v) {
        const float c1 = 0.92387953251128675613f;   // cos(pi / 8)
        const float s1 = 0.38268343236508977173f;   // sin(pi / 8)
        const float r = 0.70710678118654752440f;
        float2 a[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < 4; ++n1) a[n2][n1] = v[4 * n1 + n2];
            Dft<4, SIGN>::run(a[n2]);
        }
        const float2 w1 = make_float2(c1, SIGN * s1), w2 = make_float2(r, SIGN * r);
        const float2 w3 = make_float2(s1, SIGN * c1), w6 = make_float2(-r, SIGN * r);
        a[1][1] = cmul(a[1][1], w1);
        a[1][2] = cmul(a[1][2], w2);
        a[1][3] = cmul(a[1][3], w3);
        a[2][1] = cmul(a[2][1], w2);
        a[2][2] = mul_i<SIGN>(a[2][2]);
        a[2][3] = cmul(a[2][3], w6);
        a[3][1] = cmul(a[3][1], w3);
        a[3][2] = cmul(a[3][2], w6);
        a[3][3] = cmul(a[3][3], make_float2(-c1, -SIGN * s1));   // w16^9 = -w16
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            float2 b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
            Dft<4, SIGN>::run(b);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = b[k2];
        }
    }
};

// e^{SIGN 2 pi i j / N} for the composite radices below (angles in steps of 30 and 18 degrees)
template <int N, int SIGN>
__device__ __forceinline__ float2 root_of_unity(int j) {
    static_assert(N == 12 || N == 20, "tabulated for 12 and 20");
    float c = 1.f, s = 0.f;
    if constexpr (N == 12) {
        const float c30 = 0.86602540378443864676f;
        switch (j % 12) {
            case 1: c = c30; s = 0.5f; break;
            case 2: c = 0.5f; s = c30; break;
            case 3: c = 0.f; s = 1.f; break;
            case 4: c = -0.5f; s = c30; break;
            case 5: c = -c30; s = 0.5f; break;
            case 6: c = -1.f; s = 0.f; break;
            default: break;   // the 4 x 3 split uses j <= 6
        }
    } else {
        const float c18 = 0.95105651629515357212f, s18 = 0.30901699437494742410f;
        const float c36 = 0.80901699437494742410f, s36 = 0.58778525229247312917f;
        switch (j % 20) {
            case 1: c = c18; s = s18; break;
            case 2: c = c36; s = s36; break;
            case 3: c = s36; s = c36; break;
            case 4: c = s18; s = c18; break;
            case 5: c = 0.f; s = 1.f; break;
            case 6: c = -s18; s = c18; break;
            case 7: c = -s36; s = c36; break;
            case 8: c = -c36; s = s36; break;
            case 9: c = -c18; s = s18; break;
            case 10: c = -1.f; s = 0.f; break;
            case 11: c = -c18; s = -s18; break;
            case 12: c = -c36; s = -s36; break;
            default: break;   // the 4 x 5 split uses j <= 12
        }
    }
    return make_float2(c, SIGN * s);
}

// 4 x N2 split (decimation in time), as for 16: n = N2 n1 + n2, k = k1 + 4 k2; 4-point DFTs
// over n1, twiddles w_N^{n2 k1}, N2-point DFTs over n2.
template <int N2, int SIGN>
struct Dft4xN {
    __device__ __forceinline__ static void run(float2 *v) {
        constexpr int N = 4 * N2;
        float2 a[N2][4];
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < 4; ++n1) a[n2][n1] = v[N2 * n1 + n2];
            Dft<4, SIGN>::run(a[n2]);
        }
#pragma unroll
        for (int n2 = 1; n2 < N2; ++n2)
#pragma unroll
            for (int k1 = 1; k1 < 4; ++k1) a[n2][k1] = cmul(a[n2][k1], root_of_unity<N, SIGN>(n2 * k1));
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            float2 b[N2];
#pragma unroll
            for (int n2 = 0; n2 < N2; ++n2) b[n2] = a[n2][k1];
            Dft<N2, SIGN>::run(b);
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) v[k1 + 4 * k2] = b[k2];
        }
    }
};
template <int SIGN> struct Dft<12, SIGN> : Dft4xN<3, SIGN> {};
template <int SIGN> struct Dft<20, SIGN> : Dft4xN<5, SIGN> {};

// One Stockham stage on pencils stored in LDS as sm[j * pitch + p] (p = pencil in the
// tile, j = element), TPP threads per pencil, thread (p, q).
template <int N, int TPP, int SIGN, int NS, int R>
__device__ __forceinline__ void stage(float2 *sm, const float2 *tw, int p, int q, int pitch) {
    constexpr int NB = N / R;
    static_assert(N % R == 0, "radix must divide n");
    static_assert(NB % TPP == 0, "threads per pencil must divide n / R");
    constexpr int PER = NB / TPP;
    float2 v[PER][R];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int k = q + t * TPP;
#pragma unroll
        for (int r = 0; r < R; ++r) v[t][r] = sm[(k + r * NB) * pitch + p];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int k = q + t * TPP;
        const int kk = k % NS;
        if (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w = tw[kk * r * (N / (NS * R))];
                if (SIGN > 0) w.y = -w.y;
                v[t][r] = cmul(v[t][r], w);
            }
        }
        Dft<R, SIGN>::run(v[t]);
        const int base = (k / NS) * NS * R + kk;
#pragma unroll
        for (int r = 0; r < R; ++r) sm[(base + r * NS) * pitch + p] = v[t][r];
    }
    __syncthreads();
}

template <int N, int TPP, int SIGN, int NS, int R, int... REST>
__device__ __forceinline__ void stages(float2 *sm, const float2 *tw, int p, int q, int pitch) {
    stage<N, TPP, SIGN, NS, R>(sm, tw, p, q, pitch);
    if constexpr (sizeof...(REST) > 0) stages<N, TPP, SIGN, NS * R, REST...>(sm, tw, p, q, pitch);
}

// Stockham stages with the first stage's inputs and the last stage's outputs in registers.
// With radices R0, ..., RL (RL divides R0) thread q < T = n / R0 of a pencil owns elements
// q + T s (s < R0): the inputs of first-stage butterfly q and the outputs of last-stage
// butterflies q + T t (t < R0 / RL), which write positions q + T t + (n / RL) r.  The stages in
// between exchange through two LDS buffers stored as buf[j * pitch + p + (j >> gsh) * skew]
// (pencil p; the skew, one extra slot every 2^gsh positions, is 0 unless a caller lays its
// buffers out that way), used alternately, so each exchange needs one barrier (passing the
// same buffer twice costs a second barrier per exchange).  v[s] holds element q + T s on entry
// and on exit.
template <int N, int T, int SIGN, int NS, int R, int... REST>
__device__ __forceinline__ void reg_stage_rest(float2 *v, float2 *b0, float2 *b1, const float2 *tw, int q, int p,
                                               int pitch, int skew = 0, int gsh = 0) {
    auto at = [&](int j) { return j * pitch + p + (j >> gsh) * skew; };
    constexpr int NBF = N / R;        // butterflies of this stage
    constexpr int PER = NBF / T;      // per thread
    static_assert(NBF % T == 0, "butterflies must split evenly over the threads");
    constexpr bool LAST = sizeof...(REST) == 0;
    float2 u[PER][R];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int k = q + T * t;
        const int kk = k % NS;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            float2 x = b0[at(k + r * NBF)];
            if (r > 0) {
                float2 w = tw[kk * r * (N / (NS * R))];
                if (SIGN > 0) w.y = -w.y;
                x = cmul(x, w);
            }
            u[t][r] = x;
        }
        Dft<R, SIGN>::run(u[t]);
    }
    if constexpr (LAST) {
        static_assert(NS % T == 0, "the last radix must divide the first");
#pragma unroll
        for (int t = 0; t < PER; ++t)
#pragma unroll
            for (int r = 0; r < R; ++r) v[t + (NS / T) * r] = u[t][r];
    } else {
        if (b1 == b0) __syncthreads();   // one buffer: every thread has read this stage's inputs
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int k = q + T * t;
            const int base = (k / NS) * NS * R + k % NS;
#pragma unroll
            for (int r = 0; r < R; ++r) b1[at(base + r * NS)] = u[t][r];
        }
        __syncthreads();
        reg_stage_rest<N, T, SIGN, NS * R, REST...>(v, b1, b0, tw, q, p, pitch, skew, gsh);
    }
}

template <int N, int SIGN, int R0, int... REST>
__device__ __forceinline__ void reg_stages(float2 *v, float2 *b0, float2 *b1, const float2 *tw, int q, int p,
                                           int pitch, int skew = 0, int gsh = 0) {
    Dft<R0, SIGN>::run(v);   // first stage: butterfly q on the own elements, no twiddles
#pragma unroll
    for (int r = 0; r < R0; ++r) {
        const int j = q * R0 + r;
        b0[j * pitch + p + (j >> gsh) * skew] = v[r];
    }
    __syncthreads();
    reg_stage_rest<N, N / R0, SIGN, R0, REST...>(v, b0, b1, tw, q, p, pitch, skew, gsh);
}

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace fftcore

// Default shape (threads per pencil, workgroup threads, radices) of each length.
#define SB_FFT_CONFIGS(X)                                                                   \
    X(8, 1, 64, 8) X(12, 1, 64, 4, 3) X(16, 4, 64, 4, 4) X(24, 2, 128, 4, 2, 3)             \
    X(32, 4, 64, 4, 8) X(48, 4, 64, 4, 4, 3) X(64, 8, 128, 8, 8) X(96, 4, 64, 4, 8, 3)      \
    X(128, 16, 256, 8, 8, 2) X(160, 4, 64, 4, 8, 5) X(192, 8, 128, 8, 8, 3)                  \
    X(256, 16, 256, 8, 8, 4) X(512, 32, 256, 8, 8, 8) X(1024, 64, 256, 16, 16, 4)

// Shape of the fused passes (axis-0 correlation, last pass + contraction): more threads
// per pencil than the plain passes, so that each thread holds at most ~12 elements and
// the extra live state of the fusion (prefetch buffer, density spectrum, pair totals)
// fits the register file: (length, threads per pencil, axis-0 workgroup threads, radices).
#define SB_FUSED_CONFIGS(X)                                                                  \
    X(8, 1, 64, 8) X(12, 1, 64, 4, 3) X(16, 4, 64, 4, 4) X(24, 2, 128, 4, 2, 3)              \
    X(32, 4, 64, 4, 8) X(48, 4, 64, 4, 4, 3) X(64, 8, 128, 8, 8) X(96, 8, 128, 4, 4, 2, 3)   \
    X(128, 16, 256, 8, 8, 2) X(160, 8, 128, 4, 4, 2, 5) X(192, 16, 256, 4, 4, 4, 3)          \
    X(256, 16, 256, 16, 16) X(512, 64, 512, 8, 8, 8) X(1024, 128, 512, 8, 8, 4, 4)

// Threads per pencil of the fused last pass (the axis-0 pass uses SB_FUSED_CONFIGS):
// at most 512 threads per workgroup for up to 16 bins, except 1024 (64 threads per pencil, up
// to 1024 per workgroup, register-resident 16 x 16 x 4 stages with one exchange buffer).
#define SB_LAST_CONFIGS(X)                                                                   \
    X(8, 1, 8) X(12, 1, 4, 3) X(16, 4, 4, 4) X(24, 2, 4, 2, 3) X(32, 4, 4, 8) X(48, 4, 4, 4, 3) \
    X(64, 8, 8, 8) X(96, 8, 4, 4, 2, 3) X(128, 16, 8, 8, 2) X(160, 8, 4, 4, 2, 5)              \
    X(192, 16, 4, 4, 4, 3) X(256, 32, 8, 8, 4) X(512, 32, 8, 8, 8) X(1024, 64, 16, 16, 4)

// Fused last pass + contraction for one length (defined in fft_last_*.hip), and the
// rows per tile it needs for nb bins.
template <int N> hipError_t launch_last_for(const LastArgs &a, hipStream_t s);
template <int N> int last_rows(int nb);

}  // namespace sb
