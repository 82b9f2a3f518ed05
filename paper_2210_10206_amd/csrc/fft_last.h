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
    while (nbt * r * tpp < 128 && nbt * 2 * r * tpp <= 512 && (n * (nbt * 2 * r + 1) + n) * 8 + 2 * r * n * 4 <= 65536) r *= 2;
    return r;
}

typedef float f4v __attribute__((ext_vector_type(4)));

// The pair sums run on the matrix cores: for a quad of cells, Z[b1][b2] += w A^b1 conj(A^b2)
// is a 16 x 16 x 4 float32 MFMA whose row and column index is the bin (padded to 16) and
// whose K index is the cell, once with the real and once with the imaginary parts (twice
// more for the imaginary part of projected sums).  Lane l = i + 16 g holds bin i of cell g of
// the quad, which is both its A value (row i) and its B value (column i); the 16 x 16 result
// has b1 = 4 g + r and b2 = i in register r of lane l.  Each tile's float32 result is added
// to float64 totals, so float32 sums never span more than one tile.  The tile shape (NBT bins
// x R rows, TPP threads per pencil) is fixed at compile time so that every LDS address folds
// into an immediate offset.
template <int N, int TPP, int NBT, int R, bool IMAG, int... RAD>
__global__ __launch_bounds__(NBT * R * TPP) void last_contract_kernel(LastArgs a) {
    constexpr int P = NBT * R, PITCH = P + 1, NT = P * TPP;
    constexpr int NW = NT / 64;       // waves
    constexpr int NQ = R * N / 4;     // cell quads per tile
    constexpr int NPART = IMAG ? 2 : 1;
    constexpr int EPT = N / TPP;      // tile elements loaded per thread
    static_assert(NT % 64 == 0, "whole waves");
    extern __shared__ float2 smem[];
    const int nb = a.nb;
    float2 *sm = smem;
    float2 *tw = smem + N * PITCH;
    float *wsm = reinterpret_cast<float *>(tw + N);   // the tile's weights w(x), R N values
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    for (int i = tid; i < N; i += NT) tw[i] = a.tw[i];
    double tot[NPART][4];
#pragma unroll
    for (int q = 0; q < NPART; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) tot[q][r] = 0.0;
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
    constexpr int WPT = (R * N + NT - 1) / NT;          // weights loaded per thread
    auto load_w = [&](int64_t row0, float *dst) {
#pragma unroll
        for (int e = 0; e < WPT; ++e) {
            const int c = tid + e * NT;
            const int64_t row = row0 + c / N;
            dst[e] = (c < R * N && row < r_end) ? a.w[row * N + c % N] : 0.f;
        }
    };
    float2 nx[EPT];
    float nw[WPT];
    if (r_begin < r_end) { load_tile(r_begin, nx); load_w(r_begin, nw); }
    for (int64_t row0 = r_begin; row0 < r_end; row0 += R) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int f = tid + e * NT;
            sm[(f % N) * PITCH + f / N] = nx[e];
        }
#pragma unroll
        for (int e = 0; e < WPT; ++e)
            if (tid + e * NT < R * N) wsm[tid + e * NT] = nw[e];
        if (row0 + R < r_end) { load_tile(row0 + R, nx); load_w(row0 + R, nw); }   // next tile in flight
        __syncthreads();
        stages<N, TPP, 1, 1, RAD...>(sm, tw, tid % P, tid / P, PITCH);
        // two independent accumulator chains per part (real and imaginary operand halves)
        f4v acc[2 * NPART];
#pragma unroll
        for (int q = 0; q < 2 * NPART; ++q) acc[q] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < (NQ + NW - 1) / NW; ++k) {
            const int qd = wave + k * NW;
            if (qd < NQ) {
                const int c = 4 * qd + lg;                 // this lane's cell of the quad
                const int r = c / N, j = c % N;
                const float wv = wsm[c];                   // zero beyond the last row
                const float2 v = li < NBT ? sm[j * PITCH + li * R + r] : make_float2(0.f, 0.f);   // zero beyond nb
                const float wx = wv * v.x, wy = wv * v.y;
                acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(wx, v.x, acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(wy, v.y, acc[1], 0, 0, 0);
                if constexpr (IMAG) {
                    acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(wy, v.x, acc[2], 0, 0, 0);
                    acc[3] = __builtin_amdgcn_mfma_f32_16x16x4f32(-wx, v.y, acc[3], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NPART; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) tot[q][r] += (double)acc[2 * q][r] + (double)acc[2 * q + 1][r];
    }
    // float64 combine over the waves in wave order; partial[(g * nv + v) * nblocks + blk] with
    // v = part * npairs + pair (b1 <= b2, b1 outer)
    __syncthreads();
    double *red = reinterpret_cast<double *>(smem);   // [wave][part][b1 * 16 + b2]
#pragma unroll
    for (int q = 0; q < NPART; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[(wave * NPART + q) * 256 + (4 * lg + r) * 16 + li] = tot[q][r];
    __syncthreads();
    const int npn = nb * (nb + 1) / 2;
    const int nv = npn * NPART;
    for (int v = tid; v < nv; v += NT) {
        const int vp = v % npn, part = v / npn;
        int b1 = 0, rem = vp;                      // pair index (nb layout) -> (b1, b2)
        while (rem >= nb - b1) { rem -= nb - b1; ++b1; }
        const int b2 = b1 + rem;
        double sum = 0.0;
        for (int w = 0; w < NW; ++w) sum += red[(w * NPART + part) * 256 + b1 * 16 + b2];
        a.partial[((int64_t)blockIdx.y * nv + v) * a.nblocks + blockIdx.x] = sum;
    }
}

// Register-resident form for n = RX * RX (RX threads per row): a tile is one row of the
// NBT (padded) bins of one (l, m).  Thread q of a pencil loads elements q + RX r (coalesced:
// the RX threads of a pencil are adjacent lanes), runs the first radix-RX stage in
// registers, exchanges through LDS (positions RX q + r written, q + RX r read), runs the
// second stage and holds elements q + RX r of the transformed row, which it writes once to
// the [cell][bin] tile read by the MFMA pair sums.  The exchange and the contraction tile
// are separate LDS buffers, so a tile needs two barriers.
template <int R1, int R2, int NBT, bool IMAG>
__global__ __launch_bounds__(NBT * R2, 3) void last_reg_kernel(LastArgs a) {
    constexpr int N = R1 * R2;
    constexpr int T = R1 / R2;             // second-stage butterflies per thread
    static_assert(R1 % R2 == 0, "R2 must divide R1");
    constexpr int P = NBT;                 // pencils (bins) per tile
    constexpr int NT = P * R2;
    constexpr int NW = NT / 64;
    constexpr int NQ = N / 4;              // cell quads per tile
    constexpr int NPART = IMAG ? 2 : 1;
    constexpr int EXP = R2 * (R1 + 1);     // exchange float2 per pencil: R2 rows of R1, padded by one
    constexpr int PITCH = P + 1;
    constexpr int WPT = (N + NT - 1) / NT;
    static_assert(NT % 64 == 0, "whole waves");
    __shared__ float2 ex[P * EXP];
    __shared__ float2 cs[N * PITCH];
    __shared__ float wsm[N];
    const int nb = a.nb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int q = tid % R2, pp = tid / R2;  // element column, pencil (= bin)
    float2 tw[T][R2];                       // w^{(q + R2 t) r}, w = e^{-2 pi i / N}; the inverse takes the conjugate
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int r = 0; r < R2; ++r) tw[t][r] = a.tw[((q + R2 * t) * r) % N];
    double tot[NPART][4];
#pragma unroll
    for (int u = 0; u < NPART; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) tot[u][r] = 0.0;
    const int64_t nrows = a.ng / N;
    const int64_t r_begin = (int64_t)blockIdx.x * a.rows_per_block;
    const int64_t r_end = min(r_begin + a.rows_per_block, nrows);
    const float2 *in = a.in + ((int64_t)blockIdx.y * nb + pp) * a.ng;
    const bool live = pp < nb;
    auto load_row = [&](int64_t row, float2 *dst, float *wdst) {
#pragma unroll
        for (int r = 0; r < R1; ++r) dst[r] = live ? in[row * N + q + R2 * r] : make_float2(0.f, 0.f);
#pragma unroll
        for (int e = 0; e < WPT; ++e) {
            const int c = tid + e * NT;
            wdst[e] = c < N ? a.w[row * N + c] : 0.f;
        }
    };
    float2 nx[R1];
    float nw[WPT];
    if (r_begin < r_end) load_row(r_begin, nx, nw);
    for (int64_t row = r_begin; row < r_end; ++row) {
        float2 v[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r) v[r] = nx[r];
        float wv[WPT];
#pragma unroll
        for (int e = 0; e < WPT; ++e) wv[e] = nw[e];
        if (row + 1 < r_end) load_row(row + 1, nx, nw);    // next row in flight
        // first stage: radix-R1 butterfly q (elements q + R2 s) -> positions R1 q + r
        Dft<R1, 1>::run(v);
#pragma unroll
        for (int r = 0; r < R1; ++r) ex[pp * EXP + q * (R1 + 1) + r] = v[r];
        __syncthreads();
        // second stage: radix-R2 butterflies q + R2 t, positions q + R2 t + R1 r
#pragma unroll
        for (int t = 0; t < T; ++t) {
            float2 u[R2];
#pragma unroll
            for (int r = 0; r < R2; ++r) {
                const float2 x = ex[pp * EXP + r * (R1 + 1) + q + R2 * t];
                u[r] = r == 0 ? x : cmul(x, make_float2(tw[t][r].x, -tw[t][r].y));
            }
            Dft<R2, 1>::run(u);
#pragma unroll
            for (int r = 0; r < R2; ++r) cs[(q + R2 * t + R1 * r) * PITCH + pp] = u[r];
        }
#pragma unroll
        for (int e = 0; e < WPT; ++e)
            if (tid + e * NT < N) wsm[tid + e * NT] = wv[e];
        __syncthreads();
        f4v acc[2 * NPART];
#pragma unroll
        for (int u = 0; u < 2 * NPART; ++u) acc[u] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
        for (int k = 0; k < (NQ + NW - 1) / NW; ++k) {
            const int qd = wave + k * NW;
            if (qd < NQ) {
                const int c = 4 * qd + lg;
                const float w = wsm[c];
                const float2 x = li < NBT ? cs[c * PITCH + li] : make_float2(0.f, 0.f);   // zero beyond nb
                const float wx = w * x.x, wy = w * x.y;
                acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(wx, x.x, acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(wy, x.y, acc[1], 0, 0, 0);
                if constexpr (IMAG) {
                    acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(wy, x.x, acc[2], 0, 0, 0);
                    acc[3] = __builtin_amdgcn_mfma_f32_16x16x4f32(-wx, x.y, acc[3], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < NPART; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) tot[u][r] += (double)acc[2 * u][r] + (double)acc[2 * u + 1][r];
    }
    // float64 combine over the waves in wave order (as in last_contract_kernel)
    __syncthreads();
    double *red = reinterpret_cast<double *>(cs);
#pragma unroll
    for (int u = 0; u < NPART; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[(wave * NPART + u) * 256 + (4 * lg + r) * 16 + li] = tot[u][r];
    __syncthreads();
    const int npn = nb * (nb + 1) / 2;
    const int nv = npn * NPART;
    for (int vv = tid; vv < nv; vv += NT) {
        const int vp = vv % npn, part = vv / npn;
        int b1 = 0, rem = vp;
        while (rem >= nb - b1) { rem -= nb - b1; ++b1; }
        const int b2 = b1 + rem;
        double sum = 0.0;
        for (int w = 0; w < NW; ++w) sum += red[(w * NPART + part) * 256 + b1 * 16 + b2];
        a.partial[((int64_t)blockIdx.y * nv + vv) * a.nblocks + blockIdx.x] = sum;
    }
}

// bins padded to the instantiated tile widths 4, 8, 12, 16 so that NBT * t threads make whole
// waves (0: none fits)
constexpr int reg_padded_bins(int nb, int t) {
    for (int c = 4; c <= 16; c += 4)
        if (c >= nb && (c * t) % 64 == 0) return c;
    return 0;
}

template <int R1, int R2>
hipError_t launch_last_reg(const LastArgs &a, hipStream_t s) {
    if (a.rows != 1) return hipErrorInvalidValue;
    dim3 grid((unsigned)a.nblocks, (unsigned)a.groups);
    const bool im = a.want_imag != 0;
    const int nbt = reg_padded_bins(a.nb, R2);
#define SB_LR(NBT)                                                                                          \
    case NBT:                                                                                                \
        if constexpr ((NBT * R2) % 64 == 0) {                                                                \
            if (im) hipLaunchKernelGGL((last_reg_kernel<R1, R2, NBT, true>), grid, dim3(NBT * R2), 0, s, a);   \
            else hipLaunchKernelGGL((last_reg_kernel<R1, R2, NBT, false>), grid, dim3(NBT * R2), 0, s, a);     \
            break;                                                                                           \
        } else {                                                                                             \
            return hipErrorInvalidValue;                                                                     \
        }
    switch (nbt) {
        SB_LR(4) SB_LR(8) SB_LR(12) SB_LR(16)
        default: return hipErrorInvalidValue;
    }
#undef SB_LR
    return hipGetLastError();
}

// Register-resident form for any radix list R0, ... (each radix divides R0; see reg_stages):
// a tile is one row of the NBT (padded) bins of one (l, m); thread q < T = n / R0 of a
// pencil loads elements q + T s.  The stages exchange through two LDS buffers laid out
// [position][bin]; the transformed row is written to the buffer the last stage did not read,
// which is then the [cell][bin] tile of the MFMA pair sums.
template <int N, int NBT, bool IMAG, int R0, int... REST>
__global__ __launch_bounds__(NBT * (N / R0)) void last_rs_kernel(LastArgs a) {
    constexpr int T = N / R0;
    constexpr int P = NBT;
    constexpr int NT = P * T;
    constexpr int NW = NT / 64;
    constexpr int NQ = N / 4;
    constexpr int NPART = IMAG ? 2 : 1;
    constexpr int PITCH = P + 1;
    constexpr int NSTAGE = 1 + sizeof...(REST);
    constexpr int CSB = (NSTAGE - 1) % 2;       // buffer the last stage does not read
    constexpr int WPT = (N + NT - 1) / NT;
    static_assert(NT % 64 == 0 && NSTAGE >= 2, "whole waves, two stages or more");
    __shared__ float2 ex[2][N * PITCH];
    __shared__ float2 tw[N];
    __shared__ float wsm[N];
    const int nb = a.nb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int q = tid % T, pp = tid / T;        // element column, pencil (= bin)
    for (int i = tid; i < N; i += NT) tw[i] = a.tw[i];
    double tot[NPART][4];
#pragma unroll
    for (int u = 0; u < NPART; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) tot[u][r] = 0.0;
    const int64_t nrows = a.ng / N;
    const int64_t r_begin = (int64_t)blockIdx.x * a.rows_per_block;
    const int64_t r_end = min(r_begin + a.rows_per_block, nrows);
    const float2 *in = a.in + ((int64_t)blockIdx.y * nb + pp) * a.ng;
    const bool live = pp < nb;
    auto load_row = [&](int64_t row, float2 *dst, float *wdst) {
#pragma unroll
        for (int r = 0; r < R0; ++r) dst[r] = live ? in[row * N + q + T * r] : make_float2(0.f, 0.f);
#pragma unroll
        for (int e = 0; e < WPT; ++e) {
            const int c = tid + e * NT;
            wdst[e] = c < N ? a.w[row * N + c] : 0.f;
        }
    };
    float2 nx[R0];
    float nw[WPT];
    if (r_begin < r_end) load_row(r_begin, nx, nw);
    for (int64_t row = r_begin; row < r_end; ++row) {
        float2 v[R0];
#pragma unroll
        for (int r = 0; r < R0; ++r) v[r] = nx[r];
        float wv[WPT];
#pragma unroll
        for (int e = 0; e < WPT; ++e) wv[e] = nw[e];
        if (row + 1 < r_end) load_row(row + 1, nx, nw);    // next row in flight
        __syncthreads();                                    // the previous row's pair sums are done
        reg_stages<N, 1, R0, REST...>(v, ex[0], ex[1], tw, q, pp, PITCH);
        float2 *cs = ex[CSB];
#pragma unroll
        for (int r = 0; r < R0; ++r) cs[(q + T * r) * PITCH + pp] = v[r];
#pragma unroll
        for (int e = 0; e < WPT; ++e)
            if (tid + e * NT < N) wsm[tid + e * NT] = wv[e];
        __syncthreads();
        f4v acc[2 * NPART];
#pragma unroll
        for (int u = 0; u < 2 * NPART; ++u) acc[u] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
        for (int k = 0; k < (NQ + NW - 1) / NW; ++k) {
            const int qd = wave + k * NW;
            if (qd < NQ) {
                const int c = 4 * qd + lg;
                const float w = wsm[c];
                const float2 x = li < NBT ? cs[c * PITCH + li] : make_float2(0.f, 0.f);   // zero beyond nb
                const float wx = w * x.x, wy = w * x.y;
                acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(wx, x.x, acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(wy, x.y, acc[1], 0, 0, 0);
                if constexpr (IMAG) {
                    acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(wy, x.x, acc[2], 0, 0, 0);
                    acc[3] = __builtin_amdgcn_mfma_f32_16x16x4f32(-wx, x.y, acc[3], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < NPART; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) tot[u][r] += (double)acc[2 * u][r] + (double)acc[2 * u + 1][r];
    }
    // float64 combine over the waves in wave order (as in last_contract_kernel)
    __syncthreads();
    double *red = reinterpret_cast<double *>(&ex[0][0]);
#pragma unroll
    for (int u = 0; u < NPART; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[(wave * NPART + u) * 256 + (4 * lg + r) * 16 + li] = tot[u][r];
    __syncthreads();
    const int npn = nb * (nb + 1) / 2;
    const int nv = npn * NPART;
    for (int vv = tid; vv < nv; vv += NT) {
        const int vp = vv % npn, part = vv / npn;
        int b1 = 0, rem = vp;
        while (rem >= nb - b1) { rem -= nb - b1; ++b1; }
        const int b2 = b1 + rem;
        double sum = 0.0;
        for (int w = 0; w < NW; ++w) sum += red[(w * NPART + part) * 256 + b1 * 16 + b2];
        a.partial[((int64_t)blockIdx.y * nv + vv) * a.nblocks + blockIdx.x] = sum;
    }
}

template <int N, int R0, int... REST>
hipError_t launch_last_rs(const LastArgs &a, hipStream_t s) {
    constexpr int T = N / R0;
    if (a.rows != 1) return hipErrorInvalidValue;
    dim3 grid((unsigned)a.nblocks, (unsigned)a.groups);
    const bool im = a.want_imag != 0;
    const int nbt = reg_padded_bins(a.nb, T);
#define SB_LR(NBT)                                                                                               \
    case NBT:                                                                                                     \
        if constexpr ((NBT * T) % 64 == 0 && NBT * T <= 1024) {                                                   \
            if (im) hipLaunchKernelGGL((last_rs_kernel<N, NBT, true, R0, REST...>), grid, dim3(NBT * T), 0, s, a);  \
            else hipLaunchKernelGGL((last_rs_kernel<N, NBT, false, R0, REST...>), grid, dim3(NBT * T), 0, s, a);    \
            break;                                                                                                \
        } else {                                                                                                  \
            return hipErrorInvalidValue;                                                                          \
        }
    switch (nbt) {
        SB_LR(4) SB_LR(8) SB_LR(12) SB_LR(16)
        default: return hipErrorInvalidValue;
    }
#undef SB_LR
    return hipGetLastError();
}

template <int N, int TPP, int NBT, bool IMAG, int... RAD>
hipError_t launch_last_t(const LastArgs &a, hipStream_t s) {
    constexpr int R = fused_rows(N, TPP, NBT);
    constexpr int P = NBT * R, NT = P * TPP;
    if (a.rows != R) return hipErrorInvalidValue;
    const size_t tile = (size_t)(N * (P + 1) + N) * sizeof(float2) + (size_t)R * N * sizeof(float);
    const size_t red = (size_t)(NT / 64) * (IMAG ? 2 : 1) * 256 * sizeof(double);
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
