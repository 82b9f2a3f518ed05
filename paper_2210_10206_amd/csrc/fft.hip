// Mixed-radix Stockham FFT passes for gfx950, LDS-staged.
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
#include "sb_common.h"

namespace sb {
namespace {

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

template <int N, int TPP, int P, int SIGN, int NS, int R>
__device__ __forceinline__ void stage(float2 *sm, const float2 *tw, int p, int q) {
    constexpr int PITCH = P + 1;
    constexpr int NB = N / R;
    static_assert(N % R == 0, "radix must divide n");
    static_assert(NB % TPP == 0, "threads per pencil must divide n / R");
    constexpr int PER = NB / TPP;
    float2 v[PER][R];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int k = q + t * TPP;
#pragma unroll
        for (int r = 0; r < R; ++r) v[t][r] = sm[(k + r * NB) * PITCH + p];
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
        for (int r = 0; r < R; ++r) sm[(base + r * NS) * PITCH + p] = v[t][r];
    }
    __syncthreads();
}

template <int N, int TPP, int P, int SIGN, int NS, int R, int... REST>
__device__ __forceinline__ void stages(float2 *sm, const float2 *tw, int p, int q) {
    stage<N, TPP, P, SIGN, NS, R>(sm, tw, p, q);
    if constexpr (sizeof...(REST) > 0) stages<N, TPP, P, SIGN, NS * R, REST...>(sm, tw, p, q);
}

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
    stages<N, TPP, P, SIGN, 1, RAD...>(sm, tw, tid % P, tid / P);
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
        default: return hipErrorInvalidValue;
    }
}

bool fft_supported(int n) {
    switch (n) {
        case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 96:
        case 128: case 160: case 192: case 256: case 512: return true;
        default: return false;
    }
}

int fft_num_variants(int n) {
    switch (n) {
        case 32: case 64: case 96: case 128: case 160: case 256: case 512: return 2;
        default: return 1;
    }
}

}  // namespace sb
