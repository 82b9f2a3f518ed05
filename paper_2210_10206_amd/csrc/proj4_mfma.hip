// Projected 4PCF contraction (Alg. 8) on the matrix cores: one launch over every (cell block,
// canonical m triple), in an XCD-aware order (xcd_work).
//
// For the triple (m1, m2, m3 = -(m1 + m2)) and every cell x:
//   L[b1 b2](x)    = (w c^b1_m1)(x) c^b2_m2(x)           (vector ALU, one complex product)
//   Z[b1 b2][b3]  += L[b1 b2](x) c^b3_m3(x)               (complex, on MFMA)
// with c_{-m} = conj(c_m).  The second line is a GEMM with M = the NB^2 bin pairs (tiles of 16
// rows: row i of tile mt is pair p = 16 mt + i = b1 NB + b2), N = b3 (padded to 16) and K = the
// cells, taken as v_mfma_f32_16x16x4f32 with the four lane groups' cells as K.  The complex
// product takes three real products instead of four (Gauss): with
//   P1 = sum (Lr + Li) Br,   P2 = sum Lr (Bi - Br),   P3 = sum Li (Br + Bi)
// the real part is P1 - P3 and the imaginary part P1 + P2, three MFMAs per four cells.  The
// rounding error grows by at most about a factor of two (each product's operand is a sum of
// two).  Lane l = i + 16 g supplies row i of the A tile and column i (b3 = i) of B for cell g
// of the four.
//
// The float32 kernel has one wave per M tile: every wave contracts all cells of a staged tile
// against its own 16 pairs, so it holds one tile's three accumulators (12 registers), the waves
// need no combine at the end, and the small register count leaves room for two workgroups per CU.
// The float32 sums of each staged tile are combined into the real and imaginary parts in
// float64 (exactly) and added to float64 totals.
//
// Staging as in the full-4PCF matrix-core kernels: a tile of 64 cells in LDS, cell-major, one
// row per cell padded to a stride = 2 (mod 8) float2 (bank-conflict free stores and reads) that
// holds per bin w c_m1, c_m2, (Br, Bi - Br) and (Br + Bi, 0); the next tile's global loads are
// issued before the current one is contracted and staged into a second buffer after it.  Block
// partials: partial[(pair * NB^3 * 2 + (p NB + b3) 2 + part) * nblocks + block], as for the
// vector kernel.
#include "sb_kgen.h"

namespace sb {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

template <int NB>
constexpr int proj4_tiles() { return (NB * NB + 15) / 16; }

// Work of block b: the chip deals the workgroups of a launch to its eight XCDs in turn (b to
// XCD b mod 8), and each XCD has an L2 of its own.  Work item w = c T + t (cell block c, triple
// t of T) goes to block b with w = (b mod 8) per + b / 8, so an XCD runs a contiguous range of
// w: all triples of a cell block one after the other, while that block's coefficient columns
// (every m of the cell range) stay in its L2.  Blocks past the last item return false.
__device__ __forceinline__ bool xcd_work(int b, int nblocks, int ntriples, int *cb, int *tr) {
    const int total = nblocks * ntriples;
    const int per = (total + 7) / 8;
    const int w = (b % 8) * per + b / 8;
    if (w >= total) return false;
    *cb = w / ntriples;
    *tr = w % ntriples;
    return true;
}

template <int NB>
__global__ __launch_bounds__(64 * proj4_tiles<NB>()) void proj4_mfma_kernel(Proj4Args a) {
    a.coef += (int64_t)blockIdx.z * a.coef_fs;   // field of the launch (grid.z)
    a.w += (int64_t)blockIdx.z * a.w_fs;
    a.partial += (int64_t)blockIdx.z * a.part_fs;
    int cb = 0, pr_ = 0;
    if (!xcd_work(blockIdx.x, a.nblocks, a.npairs, &cb, &pr_)) return;
    constexpr int NP = NB * NB;
    constexpr int NMT = proj4_tiles<NB>();     // M tiles of 16 pairs = waves
    constexpr int NT = 64 * NMT;
    constexpr int TC = 64;                     // cells per staged tile
    constexpr int WL = 3 * NB;                 // loaded float2 per cell (m1, m2, m3 columns)
    constexpr int W = 4 * NB;                  // staged float2 per cell (see stage)
    constexpr int S = (W + 7) / 8 * 8 + 2;     // padded row stride, = 2 (mod 8)
    constexpr int NLD = (TC * WL + NT - 1) / NT;   // loaded float2 per thread and tile
    constexpr int NV = NB * NB * NB * 2;
    static_assert(NT % TC == 0, "every load of a thread is of the cell of its lane");
    __shared__ float2 tiles[2][TC * S];        // double-buffered: one barrier per staged tile
    const int tid = threadIdx.x, lane = tid & 63;
    const int mt = __builtin_amdgcn_readfirstlane(tid >> 6);   // this wave's M tile
    const int i = lane & 15, g = lane >> 4;
    const int m1 = a.pairs[2 * pr_], m2 = a.pairs[2 * pr_ + 1];
    const int ms[3] = {m1, m2, -(m1 + m2)};
    const int p = 16 * mt + i;                 // pair of this lane's row
    // rows past the last pair and columns past the last bin read bin 0 / bin NB - 1 (valid LDS
    // addresses, no branch in the cell loop); their sums are never written
    const int b1 = p < NP ? p / NB : 0, b2 = p < NP ? p % NB : 0;
    const int ib = i < NB ? i : NB - 1;
    f4v acc1 = f4v{0.f, 0.f, 0.f, 0.f}, acc2 = acc1, acc3 = acc1;
    double totr[4] = {0.0, 0.0, 0.0, 0.0}, toti[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t c0 = (int64_t)cb * a.cells_per_block;
    const int64_t c1 = min(c0 + a.cells_per_block, a.ng);
    // load k of this thread: f = tid + NT k -> cell f % 64 (= lane), loaded column (slot, bin) f / 64
    float2 pf[NLD];
    float pw = 0.f;
    auto gload = [&](int64_t tc) {
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int f = tid + NT * k;
            const int c = f % TC, kb = f / TC;
            float2 v = make_float2(0.f, 0.f);
            if (kb < WL && tc + c < c1) {
                const int slot = kb / NB, b = kb % NB;
                const int m = ms[slot];
                v = a.coef[((int64_t)(m < 0 ? -m : m) * NB + b) * a.ng + tc + c];
                if (m < 0) v.y = -v.y;   // c_{-m} = conj(c_m)
            }
            pf[k] = v;
        }
        pw = tc + lane < c1 ? a.w[tc + lane] : 0.f;
    };
    // a staged row holds, per bin, w c_m1 (the weight folded in once here instead of in every
    // wave), c_m2, (Br, Bi - Br) and (Br + Bi, 0) of B = c_m3: every operand of the three
    // products, formed once per cell rather than once per wave
    auto stage = [&](int buf) {
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int f = tid + NT * k;
            const int c = f % TC, kb = f / TC;
            float2 *row = tiles[buf] + c * S;
            const float2 v = pf[k];
            if (kb < NB) {
                row[kb] = make_float2(pw * v.x, pw * v.y);
            } else if (kb < 2 * NB) {
                row[kb] = v;
            } else if (kb < WL) {
                row[kb] = make_float2(v.x, v.y - v.x);
                row[kb + NB] = make_float2(v.x + v.y, 0.f);
            }
        }
    };
    // tile t is contracted from buffer t % 2 while tile t + 1 is loaded into registers, then
    // staged into the other buffer; the barrier after it makes that buffer readable and frees
    // this one for tile t + 2
    gload(c0);
    stage(0);
    __syncthreads();
    int buf = 0;
    for (int64_t tc = c0; tc < c1; tc += TC, buf ^= 1) {
        const bool more = tc + TC < c1;
        if (more) gload(tc + TC);
        const float2 *tile = tiles[buf];
#pragma unroll 2
        for (int cc = 0; cc < TC / 4; ++cc) {
            const int c = 4 * cc + g;
            const float2 *row = tile + c * S;
            const float2 bv = row[2 * NB + ib];       // (Br, Bi - Br)
            const float bs = row[3 * NB + ib].x;      // Br + Bi
            const float2 u = row[b1], x2 = row[NB + b2];   // u = w c_m1
            float2 L;
            L.x = __builtin_fmaf(u.x, x2.x, -u.y * x2.y);
            L.y = __builtin_fmaf(u.x, x2.y, u.y * x2.x);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(L.x + L.y, bv.x, acc1, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(L.x, bv.y, acc2, 0, 0, 0);
            acc3 = __builtin_amdgcn_mfma_f32_16x16x4f32(L.y, bs, acc3, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {   // P1 - P3 and P1 + P2, exact in float64
            const double p1 = (double)acc1[r];
            totr[r] += p1 - (double)acc3[r];
            toti[r] += p1 + (double)acc2[r];
        }
        acc1 = f4v{0.f, 0.f, 0.f, 0.f};
        acc2 = acc1;
        acc3 = acc1;
        if (more) stage(buf ^ 1);
        __syncthreads();
    }
    // accumulator: lane l holds rows 4 g + r (pair 16 mt + 4 g + r), column i (bin b3); each
    // (pair, b3, part) of the block is held by exactly one lane
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int pp = 16 * mt + 4 * g + r;
        if (pp < NP && i < NB) {
            const int64_t v = (int64_t)pr_ * NV + (pp * NB + i) * 2;
            a.partial[v * a.nblocks + cb] = totr[r];
            a.partial[(v + 1) * a.nblocks + cb] = toti[r];
        }
    }
}

// Split-BF16 form on v_mfma_f32_16x16x32_bf16.  Each lane group g takes one cell per
// instruction in K slots 8 g .. 8 g + 7; the N columns carry (b3, part) = (8 t + i / 2, i % 2)
// for lane i of N tile t, so one row operand serves both parts:
//   row    (pair p):            (Lr_h, Lr_h, Lr_l, nLi_h, nLi_h, nLi_l, 0, 0),   nLi = -Li
//   column (b3, real part):     (Br_h, Br_l, Br_h,  Bi_h,  Bi_l,  Bi_h, 0, 0)  -> Lr Br - Li Bi
//   column (b3, imaginary part):(Bi_h, Bi_l, Bi_h, nBr_h, nBr_l, nBr_h, 0, 0)  -> Lr Bi + Li Br
// with v = v_h + v_l split as hi = bf16(v), lo = bf16(v - hi) (the lo * lo terms dropped).
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split2(float v, __bf16 &h, __bf16 &l) {
    h = (__bf16)v;
    l = (__bf16)(v - (float)h);
}

template <int NB>
__global__ __launch_bounds__(256, 2) void proj4_split_kernel(Proj4Args a) {
    a.coef += (int64_t)blockIdx.z * a.coef_fs;   // field of the launch (grid.z)
    a.w += (int64_t)blockIdx.z * a.w_fs;
    a.partial += (int64_t)blockIdx.z * a.part_fs;
    int cb = 0, pr_ = 0;
    if (!xcd_work(blockIdx.x, a.nblocks, a.npairs, &cb, &pr_)) return;
    constexpr int NP = NB * NB;
    constexpr int NMT = (NP + 15) / 16;        // M tiles of 16 pairs
    constexpr int NNT = (2 * NB + 15) / 16;    // N tiles of 8 (b3, part) column pairs
    constexpr int TC = 64;
    constexpr int W = 3 * NB;
    constexpr int S = (W + 7) / 8 * 8 + 2;
    constexpr int NLD = (TC * W + 255) / 256;
    constexpr int NV = NB * NB * NB * 2;
    constexpr int NTILE = TC * S > 2 * NV ? TC * S : 2 * NV;
    __shared__ float2 tile[NTILE];
    __shared__ float wt[TC];
    float *red = reinterpret_cast<float *>(tile);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int i = lane & 15, g = lane >> 4;
    const int m1 = a.pairs[2 * pr_], m2 = a.pairs[2 * pr_ + 1];
    const int ms[3] = {m1, m2, -(m1 + m2)};
    int b1s[NMT], b2s[NMT];
#pragma unroll
    for (int mt = 0; mt < NMT; ++mt) {
        const int p = 16 * mt + i;
        b1s[mt] = p < NP ? p / NB : -1;
        b2s[mt] = p < NP ? p % NB : 0;
    }
    f4v acc[NMT][NNT];
#pragma unroll
    for (int mt = 0; mt < NMT; ++mt)
#pragma unroll
        for (int t = 0; t < NNT; ++t) acc[mt][t] = f4v{0.f, 0.f, 0.f, 0.f};
    const int64_t c0 = (int64_t)cb * a.cells_per_block;
    const int64_t c1 = min(c0 + a.cells_per_block, a.ng);
    float2 pf[NLD];
    float pw = 0.f;
    auto gload = [&](int64_t tc) {
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int f = tid + 256 * k;
            const int c = f % TC, kb = f / TC;
            float2 v = make_float2(0.f, 0.f);
            if (kb < W && tc + c < c1) {
                const int slot = kb / NB, b = kb % NB;
                const int m = ms[slot];
                v = a.coef[((int64_t)(m < 0 ? -m : m) * NB + b) * a.ng + tc + c];
                if (m < 0) v.y = -v.y;   // c_{-m} = conj(c_m)
            }
            pf[k] = v;
        }
        if (wave == 0) pw = tc + lane < c1 ? a.w[tc + lane] : 0.f;
    };
    const bool imag_col = (i & 1) != 0;
    gload(c0);
    for (int64_t tc = c0; tc < c1; tc += TC) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int f = tid + 256 * k;
            const int c = f % TC, kb = f / TC;
            if (kb < W) tile[c * S + kb] = pf[k];
        }
        if (wave == 0) wt[lane] = pw;
        __syncthreads();
        if (tc + TC < c1) gload(tc + TC);
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            const int c = 16 * wave + 4 * g + cc;
            const float2 *row = tile + c * S;
            const float wv = wt[c];
            bf8v bop[NNT];
#pragma unroll
            for (int t = 0; t < NNT; ++t) {
                const int b3 = 8 * t + (i >> 1);
                const float2 bv = b3 < NB ? row[2 * NB + b3] : make_float2(0.f, 0.f);
                // real column: (Br, Bi); imaginary column: (Bi, -Br)
                const float u0 = imag_col ? bv.y : bv.x, u1 = imag_col ? -bv.x : bv.y;
                __bf16 h0, l0, h1, l1;
                split2(u0, h0, l0);
                split2(u1, h1, l1);
                bop[t] = bf8v{h0, l0, h0, h1, l1, h1, (__bf16)0.f, (__bf16)0.f};
            }
#pragma unroll
            for (int mt = 0; mt < NMT; ++mt) {
                float lr = 0.f, nli = 0.f;
                if (b1s[mt] >= 0) {
                    const float2 x1 = row[b1s[mt]], x2 = row[NB + b2s[mt]];
                    const float2 u = make_float2(wv * x1.x, wv * x1.y);
                    lr = __builtin_fmaf(u.x, x2.x, -u.y * x2.y);
                    nli = -__builtin_fmaf(u.x, x2.y, u.y * x2.x);
                }
                __bf16 h0, l0, h1, l1;
                split2(lr, h0, l0);
                split2(nli, h1, l1);
                const bf8v aop = {h0, h0, l0, h1, h1, l1, (__bf16)0.f, (__bf16)0.f};
#pragma unroll
                for (int t = 0; t < NNT; ++t)
                    acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop[t], acc[mt][t], 0, 0, 0);
            }
        }
    }
    // accumulator (mt, t): lane l holds rows 4 g + r (pair 16 mt + 4 g + r), column (b3, part)
    __syncthreads();
    for (int v = tid; v < 4 * NV; v += 256) red[v] = 0.f;
    __syncthreads();
#pragma unroll
    for (int mt = 0; mt < NMT; ++mt)
#pragma unroll
        for (int t = 0; t < NNT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = 16 * mt + 4 * g + r;
                const int b3 = 8 * t + (i >> 1);
                if (p < NP && b3 < NB) red[wave * NV + (p * NB + b3) * 2 + (i & 1)] = acc[mt][t][r];
            }
    __syncthreads();
    for (int v = tid; v < NV; v += 256) {
        const double s = ((double)red[v] + (double)red[NV + v]) + ((double)red[2 * NV + v] + (double)red[3 * NV + v]);
        a.partial[((int64_t)pr_ * NV + v) * a.nblocks + cb] = s;
    }
}

template <int NB>
hipError_t launch_nb(const Proj4Args &a, hipStream_t s) {
    const int64_t total = (int64_t)a.nblocks * a.npairs;   // one block per item, 8 | grid.x (xcd_work)
    dim3 grid((unsigned)((total + 7) / 8 * 8), 1, (unsigned)(a.fields > 1 ? a.fields : 1));
    if (a.precision == 1)
        hipLaunchKernelGGL((proj4_split_kernel<NB>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((proj4_mfma_kernel<NB>), grid, dim3(64 * proj4_tiles<NB>()), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_proj4_mfma(const Proj4Args &a, hipStream_t s) {
    switch (a.nbins) {
#define SB_CASE(N) case N: return launch_nb<N>(a, s);
        SB_CASE(1) SB_CASE(2) SB_CASE(3) SB_CASE(4) SB_CASE(5) SB_CASE(6) SB_CASE(7) SB_CASE(8)
        SB_CASE(9) SB_CASE(10)
#undef SB_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace sb
