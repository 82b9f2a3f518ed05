// Adjoint of the full 3PCF: the last inverse pass of the coefficients fused with the
// per-cell adjoint weights and the forward transform of the reflected field along the same
// (contiguous) axis.
//
// For one (l, m) group and a tile of R rows x NBT (padded) bins:
//   a^b(x)   = inverse transform along the last axis of the group's arrays (axes 0, 1 done);
//   h^b(x)   = sum_b' G_l[b][b'] conj(a^b'(x)),  G_l = (g_l + g_l^T) / 2;
//   D(x)    += w_m sum_b Re(a^b(x) h^b(x))                     (direct term, float32 per cell);
//   v^b(x)   = w_m delta(x) h^b(x);
//   out^b    = forward transform along the last axis of v^b(-x): the row of -x is the row of
//              x reflected in the other axes and, with k -> -k, the transform of v^b's row:
//              out^b(flip(row), k) = V^b(row, (n - k) mod n).
// This replaces a write and a read of the coefficient arrays, of v and of the first forward
// pass of v, per (l, m) group.
//
// A packed group carries two real m = 0 fields as a^b = a^b_{l_a 0} + i a^b_{l_b 0}.  Its h takes
// G_{l_a} on the real parts and G_{l_b} on the imaginary parts (PACK: a second matrix, gz2):
// h = G_{l_a} Re a - i G_{l_b} Im a.  D and v keep their form (w_m = 1), and since the packed
// kernel is K_{l_a 0} + i K_{l_b 0}, 2 Re of its accumulation adds both fields' terms.
#pragma once
#include "fft_core.h"

namespace sb {

struct AdjLastArgs {
    int n;                  // last-axis length
    int ndim;
    int64_t shape[3];
    int64_t ng;
    const float2 *in;       // NB arrays of the group, transformed along every axis but the last
    const float *w;         // density
    const double *gz;       // g_l (NB x NB)
    const double *gz2;      // packed groups: g_{l_b} for the imaginary parts (null: gz for both)
    const float *gt;        // G_l as float, 16 x 16, zero beyond nb (register-resident form)
    const float *gt2;       // packed groups: G_{l_b} likewise (null when gz2 is)
    float wm;               // 1 for m = 0, 2 for m > 0
    int nb;
    int64_t rows_per_block; // rows walked by one workgroup
    int first;              // 1: D is written, 0: accumulated
    float *dsum;            // D, one float per cell
    float2 *out;            // NB arrays: the reflected v, transformed along the last axis
    const float2 *tw;
};
hipError_t launch_adj_last(const AdjLastArgs &a, hipStream_t s);

namespace adjlast {
using namespace fftcore;

// G (and, for PACK, the second matrix at G + NBT * NBT) into LDS: NBT x NBT, zero beyond nb.
template <int NBT, bool PACK>
__device__ __forceinline__ void load_weights(float *G, const AdjLastArgs &a, int tid, int nt) {
    const int nb = a.nb;
    for (int i = tid; i < (PACK ? 2 : 1) * NBT * NBT; i += nt) {
        const int k = i / (NBT * NBT), b1 = i % (NBT * NBT) / NBT, b2 = i % NBT;
        const double *g = k ? a.gz2 : a.gz;
        G[i] = (b1 < nb && b2 < nb) ? (float)(0.5 * (g[b1 * nb + b2] + g[b2 * nb + b1])) : 0.f;
    }
}

template <int N, int TPP, int NBT, int R, bool PACK, int... RAD>
__global__ __launch_bounds__(NBT * R * TPP) void adj_last_kernel(AdjLastArgs a) {
    constexpr int P = NBT * R, PITCH = P + 1, NT = P * TPP;
    constexpr int EPT = N / TPP;
    extern __shared__ float2 smem[];
    float2 *sm = smem;
    float2 *tw = smem + N * PITCH;
    float *G = reinterpret_cast<float *>(tw + N);   // (PACK ? 2 : 1) x NBT x NBT
    const int nb = a.nb;
    const int tid = threadIdx.x;
    for (int i = tid; i < N; i += NT) tw[i] = a.tw[i];
    load_weights<NBT, PACK>(G, a, tid, NT);
    const int64_t nrows = a.ng / N;
    const int64_t r_begin = (int64_t)blockIdx.x * a.rows_per_block;
    const int64_t r_end = min(r_begin + a.rows_per_block, nrows);
    // row index -> row index of the reflected cell (every axis but the last reflected)
    auto flip_row = [&](int64_t row) -> int64_t {
        if (a.ndim == 3) {
            const int64_t n1 = a.shape[1];
            const int64_t i0 = row / n1, i1 = row % n1;
            return ((a.shape[0] - i0) % a.shape[0]) * n1 + (n1 - i1) % n1;
        }
        return (a.shape[0] - row) % a.shape[0];
    };
    // per thread: elements e of the load pattern (f = tid + e NT: pencil f / N, column f % N) and
    // cells c = tid + k NT of the per-cell phase; the next tile's values are loaded into
    // registers while the current one is processed
    constexpr int CPT = (R * N + NT - 1) / NT;
    auto load_tile = [&](int64_t row0, float2 *x, float *wv, float *dv) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int f = tid + e * NT;
            const int pp = f / N, j = f % N;
            const int b = pp / R;
            const int64_t row = row0 + pp % R;
            x[e] = (row < r_end && b < nb) ? a.in[(int64_t)b * a.ng + row * N + j] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = tid + k * NT;
            const int64_t row = row0 + c / N;
            const bool in = c < R * N && row < r_end;
            wv[k] = in ? a.w[row * N + c % N] : 0.f;
            dv[k] = (in && !a.first) ? a.dsum[row * N + c % N] : 0.f;
        }
    };
    float2 nx[EPT];
    float nw[CPT], nd[CPT];
    if (r_begin < r_end) load_tile(r_begin, nx, nw, nd);
    for (int64_t row0 = r_begin; row0 < r_end; row0 += R) {
        float cw[CPT], cd[CPT];
#pragma unroll
        for (int k = 0; k < CPT; ++k) { cw[k] = nw[k]; cd[k] = nd[k]; }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int f = tid + e * NT;
            sm[(f % N) * PITCH + f / N] = nx[e];
        }
        if (row0 + R < r_end) load_tile(row0 + R, nx, nw, nd);   // next tile in flight
        __syncthreads();
        stages<N, TPP, 1, 1, RAD...>(sm, tw, tid % P, tid / P, PITCH);
        // per cell: h, the direct term and v (each thread owns whole cells: all bins of a cell)
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = tid + k * NT;
            const int r = c / N, j = c % N;
            const int64_t row = row0 + r;
            if (c >= R * N || row >= r_end) continue;
            const int64_t cell = row * N + j;
            float2 av[NBT];
#pragma unroll
            for (int b = 0; b < NBT; ++b) av[b] = sm[j * PITCH + b * R + r];
            const float dw = a.wm * cw[k];
            float d = 0.f;
#pragma unroll
            for (int b1 = 0; b1 < NBT; ++b1) {
                float hx = 0.f, hy = 0.f;
#pragma unroll
                for (int b2 = 0; b2 < NBT; ++b2) {
                    const float g = G[b1 * NBT + b2];
                    const float g2 = PACK ? G[NBT * NBT + b1 * NBT + b2] : g;
                    hx = __builtin_fmaf(g, av[b2].x, hx);
                    hy = __builtin_fmaf(-g2, av[b2].y, hy);   // conj(a)
                }
                d = __builtin_fmaf(av[b1].x, hx, d);
                d = __builtin_fmaf(-av[b1].y, hy, d);
                sm[j * PITCH + b1 * R + r] = make_float2(dw * hx, dw * hy);
            }
            a.dsum[cell] = cd[k] + a.wm * d;   // cd = 0 on the first group
        }
        __syncthreads();
        stages<N, TPP, -1, 1, RAD...>(sm, tw, tid % P, tid / P, PITCH);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int f = tid + e * NT;
            const int pp = f / N, k = f % N;
            const int b = pp / R;
            const int64_t row = row0 + pp % R;
            if (row < r_end && b < nb)
                a.out[(int64_t)b * a.ng + flip_row(row) * N + (N - k) % N] = sm[k * PITCH + pp];
        }
    }
}

// Register-resident form for the lengths with a radix list R0, REST... whose last radix
// divides the first (reg_stages): a tile is one row of the NBT (padded) bins; thread q < T =
// N / R0 of pencil pp (= bin) holds elements q + T s of it, so the loads, both transforms and
// the stores stay in registers and LDS is used for the stage exchanges and for the [cell][bin]
// view of the per-cell phase.  The weights are read from the float table gt through the
// constant address space: the addresses are uniform, so they become scalar loads and the
// products take them from SGPRs instead of broadcast LDS reads (up to 2 x 144 per cell).
//
// With two stages the transforms exchange through one buffer, which the [cell][bin] view then
// reuses (one more barrier per row); that and at most 168 VGPRs (3 waves per SIMD) let four
// 3-wave workgroups share a CU instead of two at 256 points and 12 padded bins.
//
// LDS layout: position j of pencil p at j * (P + 1) + p, and at 256 points, in the transform's
// stages, with one skew slot every 16 positions (+ j >> 4); the [cell][bin] view of the per-cell
// phase keeps the plain layout (a pencil's threads an odd pitch apart: no conflicts).  The first stage writes positions q R0 + r: in the plain layout
// the threads of a pencil sit R0 (P + 1) float2 apart, a multiple of the 16 float2 that span the
// 32 banks, so they all meet in one bank; the skew spreads them.  A bank model of every exchange,
// transpose and per-cell access (32 banks, 16 lanes per float2 phase; it reproduces the measured
// conflict share of the plain layout, 67 % of the LDS cycles at 128 points) puts the skewed
// layout at 0.21 of the plain one's LDS cycles at 256 points, and the pass there runs 25 %
// faster (8 bins: 9.8 -> 7.4 ms per 13 launches).  At 128 points (0.31 in the model) the time did
// not move, and 64 and 160 points were slower with it, so the other lengths keep the plain layout.
constexpr int adj_rs_min_waves(int nstage, int nt) { return nstage == 2 && nt >= 192 ? 3 : 1; }

template <int N, int NBT, bool PACK, int R0, int... REST>
__global__ __launch_bounds__(NBT * (N / R0), adj_rs_min_waves(1 + sizeof...(REST), NBT * (N / R0))) void adj_rs_kernel(
    AdjLastArgs a) {
    constexpr int T = N / R0;
    constexpr int P = NBT, PITCH = P + 1, NT = P * T;
    constexpr int SKEW = N == 256 ? 1 : 0, GSH = 4;   // layout above
    constexpr int NSTAGE = 1 + sizeof...(REST);
    constexpr bool ONE = NSTAGE == 2;           // one exchange buffer
    constexpr int CSB = ONE ? 0 : (NSTAGE - 1) % 2;   // buffer of the [cell][bin] view
    constexpr int CPT = (N + NT - 1) / NT;      // cells per thread in the per-cell phase
    static_assert(NSTAGE >= 2, "two stages or more");
    static_assert(NBT <= 16, "the weight table is 16 x 16");
    __shared__ float2 ex[ONE ? 1 : 2][N * PITCH + (N >> GSH) * SKEW];
    auto at = [](int j, int b) { return j * PITCH + b; };   // the [cell][bin] view: plain layout
    float2 *ex1 = ex[ONE ? 0 : 1];
    __shared__ float2 tw[N];
    typedef const __attribute__((address_space(4))) float cfloat;
    cfloat *G = (cfloat *)a.gt;                   // 16 x 16, zero beyond nb
    cfloat *G2 = PACK ? (cfloat *)a.gt2 : G;
    const int nb = a.nb;
    const int tid = threadIdx.x;
    const int q = tid % T, pp = tid / T;         // element column, pencil (= bin)
    for (int i = tid; i < N; i += NT) tw[i] = a.tw[i];
    const int64_t nrows = a.ng / N;
    const int64_t r_begin = (int64_t)blockIdx.x * a.rows_per_block;
    const int64_t r_end = min(r_begin + a.rows_per_block, nrows);
    const bool live = pp < nb;
    const float2 *in = a.in + (int64_t)(live ? pp : 0) * a.ng;
    auto flip_row = [&](int64_t row) -> int64_t {
        if (a.ndim == 3) {
            const int64_t n1 = a.shape[1];
            const int64_t i0 = row / n1, i1 = row % n1;
            return ((a.shape[0] - i0) % a.shape[0]) * n1 + (n1 - i1) % n1;
        }
        return (a.shape[0] - row) % a.shape[0];
    };
    auto load_row = [&](int64_t row, float2 *x, float *wv, float *dv) {
#pragma unroll
        for (int r = 0; r < R0; ++r) x[r] = live ? ld_stream(&in[row * N + q + T * r]) : make_float2(0.f, 0.f);
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = tid + k * NT;
            wv[k] = c < N ? a.w[row * N + c] : 0.f;
            dv[k] = (c < N && !a.first) ? a.dsum[row * N + c] : 0.f;
        }
    };
    float2 nx[R0];
    float nw[CPT], nd[CPT];
    if (r_begin < r_end) load_row(r_begin, nx, nw, nd);
    for (int64_t row = r_begin; row < r_end; ++row) {
        float2 v[R0];
        float cw[CPT], cd[CPT];
#pragma unroll
        for (int r = 0; r < R0; ++r) v[r] = nx[r];
#pragma unroll
        for (int k = 0; k < CPT; ++k) { cw[k] = nw[k]; cd[k] = nd[k]; }
        if (row + 1 < r_end) load_row(row + 1, nx, nw, nd);   // next row in flight
        __syncthreads();                                       // the previous row's buffers are free
        reg_stages<N, 1, R0, REST...>(v, ex[0], ex1, tw, q, pp, PITCH, SKEW, GSH);   // inverse
        float2 *cs = ex[CSB];
        if constexpr (ONE) __syncthreads();   // the last stage has read the exchange buffer
#pragma unroll
        for (int r = 0; r < R0; ++r) cs[at(q + T * r, pp)] = v[r];
        __syncthreads();
        // per cell: h = G conj(a), the direct term and v = w_m delta h (whole cells per thread)
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = tid + k * NT;
            if (c >= N) continue;
            float2 av[NBT];
#pragma unroll
            for (int b = 0; b < NBT; ++b) av[b] = cs[at(c, b)];
            const float dw = a.wm * cw[k];
            float d = 0.f;
#pragma unroll
            for (int b1 = 0; b1 < NBT; ++b1) {
                float hx = 0.f, hy = 0.f;
#pragma unroll
                for (int b2 = 0; b2 < NBT; ++b2) {
                    const float g = G[b1 * 16 + b2];
                    const float g2 = PACK ? G2[b1 * 16 + b2] : g;
                    hx = __builtin_fmaf(g, av[b2].x, hx);
                    hy = __builtin_fmaf(-g2, av[b2].y, hy);   // conj(a)
                }
                d = __builtin_fmaf(av[b1].x, hx, d);
                d = __builtin_fmaf(-av[b1].y, hy, d);
                cs[at(c, b1)] = make_float2(dw * hx, dw * hy);
            }
            a.dsum[row * N + c] = cd[k] + a.wm * d;   // cd = 0 on the first group
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R0; ++r) v[r] = cs[at(q + T * r, pp)];
        __syncthreads();                                       // cs may be the first exchange buffer
        reg_stages<N, -1, R0, REST...>(v, ex[0], ex1, tw, q, pp, PITCH, SKEW, GSH);  // forward
        if (live) {
            float2 *out = a.out + (int64_t)pp * a.ng + flip_row(row) * N;
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const int k = q + T * r;
                st_stream(&out[(N - k) % N], v[r]);
            }
        }
    }
}

// bins padded to 4, 8, 12 or 16 so that NBT * t threads make whole waves (0: none fits)
constexpr int rs_padded_bins(int nb, int t) {
    for (int c = 4; c <= 16; c += 4)
        if (c >= nb && (c * t) % 64 == 0 && c * t <= 1024) return c;
    return 0;
}

template <int N, int R0, int... REST>
hipError_t launch_rs(const AdjLastArgs &a, hipStream_t s) {
    constexpr int T = N / R0;
    const int64_t nrows = a.ng / N;
    dim3 grid((unsigned)((nrows + a.rows_per_block - 1) / a.rows_per_block));
    switch (rs_padded_bins(a.nb, T)) {
#define SB_AR(NBT)                                                                               \
    case NBT:                                                                                    \
        if constexpr ((NBT * T) % 64 == 0 && NBT * T <= 1024) {                                  \
            if (a.gz2) hipLaunchKernelGGL((adj_rs_kernel<N, NBT, true, R0, REST...>), grid, dim3(NBT * T), 0, s, a);  \
            else hipLaunchKernelGGL((adj_rs_kernel<N, NBT, false, R0, REST...>), grid, dim3(NBT * T), 0, s, a); \
            return hipGetLastError();                                                            \
        } else {                                                                                 \
            return hipErrorInvalidValue;                                                         \
        }
        SB_AR(4) SB_AR(8) SB_AR(12) SB_AR(16)
#undef SB_AR
        default: return hipErrorInvalidValue;
    }
}

// rows per tile: the fewest that make whole waves
constexpr int tile_rows(int tpp, int nbt) {
    int r = 1;
    while ((nbt * r * tpp) % 64 != 0) ++r;
    return r;
}

template <int N, int TPP, int NBT, bool PACK, int... RAD>
hipError_t launch_tp(const AdjLastArgs &a, hipStream_t s) {
    constexpr int R = tile_rows(TPP, NBT);
    constexpr int P = NBT * R, NT = P * TPP;
    static_assert(NT <= 1024, "workgroup size");
    const size_t shm = (size_t)(N * (P + 1) + N) * sizeof(float2) + (size_t)(PACK ? 2 : 1) * NBT * NBT * sizeof(float);
    if (shm > 160 * 1024) return hipErrorInvalidValue;
    if (shm > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&adj_last_kernel<N, TPP, NBT, R, PACK, RAD...>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
    }
    const int64_t nrows = a.ng / N;
    dim3 grid((unsigned)((nrows + a.rows_per_block - 1) / a.rows_per_block));
    hipLaunchKernelGGL((adj_last_kernel<N, TPP, NBT, R, PACK, RAD...>), grid, dim3(NT), shm, s, a);
    return hipGetLastError();
}

template <int N, int TPP, int NBT, int... RAD>
hipError_t launch_t(const AdjLastArgs &a, hipStream_t s) {
    return a.gz2 ? launch_tp<N, TPP, NBT, true, RAD...>(a, s) : launch_tp<N, TPP, NBT, false, RAD...>(a, s);
}

template <int N, int TPP, int... RAD>
hipError_t launch_n(const AdjLastArgs &a, hipStream_t s) {
    const int nb = a.nb;
    if (nb <= 4) return launch_t<N, TPP, 4, RAD...>(a, s);
    if (nb <= 8) return launch_t<N, TPP, 8, RAD...>(a, s);
    if (nb <= 12) return launch_t<N, TPP, 12, RAD...>(a, s);
    if (nb <= 16) return launch_t<N, TPP, 16, RAD...>(a, s);
    return hipErrorInvalidValue;
}

}  // namespace adjlast
}  // namespace sb
