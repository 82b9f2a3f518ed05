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
// Rows per tile of the fused pass for a length n handled by tpp threads per pencil and
// nbt (padded) bins: the smallest count that makes nbt * rows * tpp a whole number of
// waves, then doubled up to 128 threads when the tile stays small.
constexpr int fused_rows(int n, int tpp, int nbt) {
    int r = 1;
    while ((nbt * r * tpp) % 64 != 0) ++r;
    while (nbt * r * tpp < 128 && nbt * 2 * r * tpp <= 512 && (n * (nbt * 2 * r + 1) + n) * 8 <= 65536) r *= 2;
    return r;
}

// Each thread owns whole cells: it reads the nb coefficients of a cell once from LDS and
// adds every pair b1 <= b2 to its float32 totals (nb (nb + 1) / 2 of them).  The tile
// shape (NBT bins x R rows, TPP threads per pencil) is fixed at compile time so that every
// LDS address folds into an immediate offset.
template <int N, int TPP, int NBT, int R, bool IMAG, int... RAD>
__global__ __launch_bounds__(NBT * R * TPP) void last_contract_kernel(LastArgs a) {
    constexpr int P = NBT * R, PITCH = P + 1, NT = P * TPP;
    constexpr int NPT = NBT * (NBT + 1) / 2;
    constexpr int NACC = NPT * (IMAG ? 2 : 1);
    constexpr int EPT = N / TPP;      // tile elements loaded per thread
    extern __shared__ float2 smem[];
    const int nb = a.nb;
    float2 *sm = smem;
    float2 *tw = smem + N * PITCH;
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
            const int b = pp / R;
            const int64_t row = row0 + pp % R;
            dst[e] = (row < r_end && b < nb) ? in[(int64_t)b * a.ng + row * N + j] : make_float2(0.f, 0.f);
        }
    };
    float2 nx[EPT];
    if (r_begin < r_end) load_tile(r_begin, nx);
    for (int64_t row0 = r_begin; row0 < r_end; row0 += R) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int f = tid + e * NT;
            sm[(f % N) * PITCH + f / N] = nx[e];
        }
        if (row0 + R < r_end) load_tile(row0 + R, nx);     // next tile in flight during this one
        __syncthreads();
        stages<N, TPP, 1, 1, RAD...>(sm, tw, tid % P, tid / P, PITCH);
        for (int c = tid; c < R * N; c += NT) {
            const int r = c / N, j = c % N;
            const int64_t row = row0 + r;
            if (row >= r_end) continue;
            const float wv = a.w[row * N + j];
            float2 v[NBT];
#pragma unroll
            for (int b = 0; b < NBT; ++b) v[b] = sm[j * PITCH + b * R + r];   // zero beyond nb
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
    // float64 combine: every thread stores its float32 totals, then pair v sums them over
    // the block's threads in thread order; partial[(g * nv + v) * nblocks + blk]
    __syncthreads();
    float *red = reinterpret_cast<float *>(smem);   // [tid][NACC]
#pragma unroll
    for (int u = 0; u < NACC; ++u) red[tid * NACC + u] = acc[u];
    __syncthreads();
    const int npn = nb * (nb + 1) / 2;
    const int nv = npn * (IMAG ? 2 : 1);
    const int ncontrib = min(NT, R * N);           // threads that own cells
    for (int v = tid; v < nv; v += NT) {
        const int vp = v % npn, part = v / npn;
        int b1 = 0, rem = vp;                      // pair index (nb layout) -> (b1, b2)
        while (rem >= nb - b1) { rem -= nb - b1; ++b1; }
        const int b2 = b1 + rem;
        const int q = b1 * NBT - b1 * (b1 - 1) / 2 + (b2 - b1) + part * NPT;   // NBT layout
        double sum = 0.0;
        for (int t = 0; t < ncontrib; ++t) sum += (double)red[t * NACC + q];
        a.partial[((int64_t)blockIdx.y * nv + v) * a.nblocks + blockIdx.x] = sum;
    }
}

template <int N, int TPP, int NBT, bool IMAG, int... RAD>
hipError_t launch_last_t(const LastArgs &a, hipStream_t s) {
    constexpr int R = fused_rows(N, TPP, NBT);
    constexpr int P = NBT * R, NT = P * TPP;
    if (a.rows != R) return hipErrorInvalidValue;
    const size_t tile = (size_t)(N * (P + 1) + N) * sizeof(float2);
    const size_t red = (size_t)NT * (NBT * (NBT + 1) / 2) * (IMAG ? 2 : 1) * sizeof(float);
    const size_t shm = tile > red ? tile : red;
    dim3 grid((unsigned)a.nblocks, (unsigned)a.groups);
    hipLaunchKernelGGL((last_contract_kernel<N, TPP, NBT, R, IMAG, RAD...>), grid, dim3(NT), shm, s, a);
    return hipGetLastError();
}

constexpr int padded_bins(int nb) { return nb <= 4 ? 4 : nb <= 8 ? 8 : nb <= 10 ? 10 : nb <= 12 ? 12 : 16; }

template <int N, int TPP, int... RAD>
hipError_t launch_last_nb(const LastArgs &a, hipStream_t s) {
    const bool im = a.want_imag != 0;
    switch (padded_bins(a.nb)) {
        case 4: return im ? launch_last_t<N, TPP, 4, true, RAD...>(a, s) : launch_last_t<N, TPP, 4, false, RAD...>(a, s);
        case 8: return im ? launch_last_t<N, TPP, 8, true, RAD...>(a, s) : launch_last_t<N, TPP, 8, false, RAD...>(a, s);
        case 10: return im ? launch_last_t<N, TPP, 10, true, RAD...>(a, s) : launch_last_t<N, TPP, 10, false, RAD...>(a, s);
        case 12: return im ? launch_last_t<N, TPP, 12, true, RAD...>(a, s) : launch_last_t<N, TPP, 12, false, RAD...>(a, s);
        default: return im ? launch_last_t<N, TPP, 16, true, RAD...>(a, s) : launch_last_t<N, TPP, 16, false, RAD...>(a, s);
    }
}

// Rows per tile the fused pass uses for length n (tpp threads per pencil) and nb bins.
template <int N, int TPP>
int last_rows_for(int nb) {
    switch (padded_bins(nb)) {
        case 4: return fused_rows(N, TPP, 4);
        case 8: return fused_rows(N, TPP, 8);
        case 10: return fused_rows(N, TPP, 10);
        case 12: return fused_rows(N, TPP, 12);
        default: return fused_rows(N, TPP, 16);
    }
}

}  // namespace fftlast
}  // namespace sb
