// Last inverse pass (contiguous axis) fused with the two-coefficient contraction,
// instantiated for the lengths listed at the end of the including file.
#pragma once
#include "fft_core.h"

namespace sb {
namespace fftlast {
using namespace fftcore;

// ------------------------------------------------------------------------------
// Last inverse pass (contiguous axis) fused with the two-coefficient contraction:
// a workgroup transforms `rows` rows of each of the nb kernel arrays of one group
// (P = nb * rows pencils, TPP threads each) and, per cell of those rows, adds
// w(x) A^b1 conj(A^b2) for b1 <= b2 to float32 per-thread totals; the coefficient
// arrays are never written.  Block totals are combined in float64.
template <int N, int TPP, int NBT, bool IMAG, int... RAD>
__global__ __launch_bounds__(512) void last_contract_kernel(LastArgs a) {
    constexpr int NPT = NBT * (NBT + 1) / 2;
    constexpr int NACC = NPT * (IMAG ? 2 : 1);
    constexpr int EPT = N / TPP;      // tile elements loaded per thread (P N / (P TPP))
    extern __shared__ float2 smem[];
    const int nb = a.nb, R = a.rows;
    const int P = nb * R, pitch = P + 1;
    const int NT = blockDim.x;
    float2 *sm = smem;
    float2 *tw = smem + N * pitch;
    const int tid = threadIdx.x;
    for (int i = tid; i < N; i += NT) tw[i] = a.tw[i];
    float acc[NACC];
#pragma unroll
    for (int v = 0; v < NACC; ++v) acc[v] = 0.f;
    const int64_t nrows = a.ng / N;
    const int64_t r_begin = (int64_t)blockIdx.x * a.rows_per_block;
    const int64_t r_end = min(r_begin + a.rows_per_block, nrows);
    const float2 *in = a.in + (int64_t)blockIdx.y * nb * a.ng;
    // element e of the load pattern: f = tid + e NT, pencil pp = f / N (bin pp / R, row pp % R), column f % N
    auto load_tile = [&](int64_t row0, float2 *dst) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int f = tid + e * NT;
            const int pp = f / N, j = f % N;
            const int64_t row = row0 + pp % R;
            dst[e] = row < r_end ? in[(int64_t)(pp / R) * a.ng + row * N + j] : make_float2(0.f, 0.f);
        }
    };
    float2 nx[EPT];
    if (r_begin < r_end) load_tile(r_begin, nx);
    for (int64_t row0 = r_begin; row0 < r_end; row0 += R) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int f = tid + e * NT;
            sm[(f % N) * pitch + f / N] = nx[e];
        }
        if (row0 + R < r_end) load_tile(row0 + R, nx);     // next tile in flight during this one
        __syncthreads();
        stages<N, TPP, 1, 1, RAD...>(sm, tw, tid % P, tid / P, pitch);
        for (int c = tid; c < R * N; c += NT) {
            const int r = c / N, j = c % N;
            const int64_t row = row0 + r;
            if (row >= r_end) continue;
            const float wv = a.w[row * N + j];
            float2 v[NBT];
#pragma unroll
            for (int b = 0; b < NBT; ++b) v[b] = b < nb ? sm[j * pitch + b * R + r] : make_float2(0.f, 0.f);
            int q = 0;
#pragma unroll
            for (int b1 = 0; b1 < NBT; ++b1) {
                const float2 u = make_float2(wv * v[b1].x, wv * v[b1].y);
#pragma unroll
                for (int b2 = b1; b2 < NBT; ++b2, ++q) {
                    acc[q] += u.x * v[b2].x + u.y * v[b2].y;
                    if (IMAG) acc[NPT + q] += u.y * v[b2].x - u.x * v[b2].y;
                }
            }
        }
    }
    // float64 combine over the block's waves; partial[(g * nv + v) * nblocks + blk]
    __syncthreads();
    const int nwave = NT >> 6, lane = tid & 63, wave = tid >> 6;
    const int npn = nb * (nb + 1) / 2;
    const int nv = npn * (IMAG ? 2 : 1);
    double *red = reinterpret_cast<double *>(smem);
    int q = 0;
#pragma unroll
    for (int b1 = 0; b1 < NBT; ++b1)
#pragma unroll
        for (int b2 = b1; b2 < NBT; ++b2, ++q) {
            if (b2 < nb) {
                const int vq = b1 * nb - b1 * (b1 - 1) / 2 + (b2 - b1);
                const double s0 = wave_sum64((double)acc[q]);
                if (lane == 0) red[wave * nv + vq] = s0;
                if (IMAG) {
                    const double s1 = wave_sum64((double)acc[NPT + q]);
                    if (lane == 0) red[wave * nv + npn + vq] = s1;
                }
            }
        }
    __syncthreads();
    for (int v = tid; v < nv; v += NT) {
        double s = 0.0;
        for (int wv = 0; wv < nwave; ++wv) s += red[wv * nv + v];
        a.partial[((int64_t)blockIdx.y * nv + v) * a.nblocks + blockIdx.x] = s;
    }
}

template <int N, int TPP, int NBT, bool IMAG, int... RAD>
hipError_t launch_last_t(const LastArgs &a, hipStream_t s) {
    const int P = a.nb * a.rows;
    const int nt = P * TPP;
    const size_t tile = (size_t)(N * (P + 1) + N) * sizeof(float2);
    const int nv = a.nb * (a.nb + 1) / 2 * (IMAG ? 2 : 1);
    const size_t red = (size_t)(nt / 64) * nv * sizeof(double);
    const size_t shm = tile > red ? tile : red;
    dim3 grid((unsigned)a.nblocks, (unsigned)a.groups);
    hipLaunchKernelGGL((last_contract_kernel<N, TPP, NBT, IMAG, RAD...>), grid, dim3(nt), shm, s, a);
    return hipGetLastError();
}

template <int N, int TPP, int... RAD>
hipError_t launch_last_nb(const LastArgs &a, hipStream_t s) {
    const bool im = a.want_imag != 0;
    if (a.nb <= 4) return im ? launch_last_t<N, TPP, 4, true, RAD...>(a, s) : launch_last_t<N, TPP, 4, false, RAD...>(a, s);
    if (a.nb <= 8) return im ? launch_last_t<N, TPP, 8, true, RAD...>(a, s) : launch_last_t<N, TPP, 8, false, RAD...>(a, s);
    if (a.nb <= 10) return im ? launch_last_t<N, TPP, 10, true, RAD...>(a, s) : launch_last_t<N, TPP, 10, false, RAD...>(a, s);
    if (a.nb <= 12) return im ? launch_last_t<N, TPP, 12, true, RAD...>(a, s) : launch_last_t<N, TPP, 12, false, RAD...>(a, s);
    return im ? launch_last_t<N, TPP, 16, true, RAD...>(a, s) : launch_last_t<N, TPP, 16, false, RAD...>(a, s);
}

}  // namespace fftlast
}  // namespace sb
