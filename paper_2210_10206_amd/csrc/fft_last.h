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

// The pair sums run on the matrix cores as 16-block 4 x 4 x 1 float32 MFMAs: block b of an
// instruction is slot b, one (cell, part) of a group of 8 cells (slot b = cell b / 2, real part
// for even b, imaginary for odd), and holds the 4 x 4 outer product of bins 4 qa .. 4 qa + 3
// (weighted, rows) and 4 qb .. 4 qb + 3 (columns) of that slot.  The instructions of a group
// walk the bin-quad pairs qa <= qb, so only the upper-triangle blocks of the NBT x NBT result
// are computed (6 instructions per 8 cells for 12 padded bins), and each lane reads the values
// of its slot once per group.  Lane 4 b + j supplies row j and column j of block b and holds
// row r, column j of it in register r.  Each tile's float32 result is added to float64 totals
// per lane; at the end the 16 slots are summed by a fixed butterfly over lanes and the waves
// in wave order.  Three modes:
//   PS_REAL    Re(A^b1 conj A^b2): the real- and imaginary-part slots of a cell are summed.
//   PS_COMPLEX also Im(A^b1 conj A^b2) = Im A^b1 Re A^b2 - Re A^b1 Im A^b2 (projected sums): a
//              second set of instructions takes the other part of the column value with the
//              sign of the slot's part.
//   PS_PACKED  Re A^b1 Re A^b2 and Im A^b1 Im A^b2 kept apart, for arrays that carry two real
//              coefficient fields as real and imaginary part.
// The outputs are part-major: value v = part * npairs + pair.
enum PairMode : int { PS_REAL = 0, PS_COMPLEX = 1, PS_PACKED = 2 };

typedef short s4v __attribute__((ext_vector_type(4)));

// Split-BF16 operands of the 4 x 4 x 4 bf16 MFMA: v = hi + lo with hi = bf16(v) and
// lo = bf16(v - hi), both rounded to nearest.  The row operand carries (hi, hi, lo, 0) and the
// column operand (hi, lo, hi, 0) in the four K slots, so one instruction adds
// hi_a hi_b + hi_a lo_b + lo_a hi_b (the lo * lo term, below 2^-16 of the product, is dropped).
__device__ __forceinline__ void bf16_split(float v, short &h, short &l) {
    const __bf16 hb = (__bf16)v;
    const __bf16 lb = (__bf16)(v - (float)hb);
    h = __builtin_bit_cast(short, hb);
    l = __builtin_bit_cast(short, lb);
}
__device__ __forceinline__ s4v split_row(float v) {
    short h, l;
    bf16_split(v, h, l);
    return s4v{h, h, l, 0};
}
__device__ __forceinline__ s4v split_col(float v) {
    short h, l;
    bf16_split(v, h, l);
    return s4v{h, l, h, 0};
}

// PREC 0: float32 4 x 4 x 1 MFMA.  PREC 1: split-BF16 4 x 4 x 4 MFMA (split_row / split_col),
// float32 accumulation; the blocks, slots and lanes are the same.
template <int NBT, int MODE, int PREC = 0>
struct PairSums {
    static constexpr int Q = (NBT + 3) / 4;           // bin quads (bins >= NBT read as zero)
    static constexpr int NPB = Q * (Q + 1) / 2;       // quad pairs qa <= qb
    static constexpr int NACC = MODE == PS_COMPLEX ? 2 : 1;   // accumulator sets
    static constexpr int NOUT = MODE == PS_REAL ? 1 : 2;      // output parts
    static constexpr int CPG = 8;                     // cells per group
    static_assert(NBT >= 1 && NBT <= 16, "at most 16 bins");
    static constexpr int red_doubles(int nw) { return nw * NOUT * NPB * 16; }
    static constexpr int NV = NACC * NPB * 4;         // accumulator values per lane
    // The slots of lanes that differ only in the folded lane bits add into the same sums: all 16
    // slots (bits 2-5), or for PS_PACKED the 8 slots of one part (bits 3-5).  A flush folds those
    // lanes' values into float64 totals spread over them: NT2 totals per lane (see flush).
    static constexpr int FB0 = MODE == PS_PACKED ? 3 : 2;   // first folded lane bit
    static constexpr int NFB = 6 - FB0;                      // folded lane bits
    static constexpr int GS = 1 << NFB;                      // lanes sharing a sum
    static constexpr int NVP = (NV + GS - 1) / GS * GS;      // values per lane, padded to GS
    static constexpr int NT2 = NVP / GS;                     // float64 totals per lane
    double tot[NT2];
    f4v acc[NACC][NPB];                               // float32 sums since the last flush

    __device__ __forceinline__ void clear_acc() {
#pragma unroll
        for (int u = 0; u < NACC; ++u)
#pragma unroll
            for (int p = 0; p < NPB; ++p) acc[u][p] = f4v{0.f, 0.f, 0.f, 0.f};
    }

    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int m = 0; m < NT2; ++m) tot[m] = 0.0;
        clear_acc();
    }

    // Adds one tile of NCELL cells to the float32 sums: the value of bin b at cell c is
    // stage[off(c) + b * bstride] and its weight wsm[c].  The waves take groups of 8 cells in turn.
    // PLANE > 0 (not PS_COMPLEX): the stage holds separate real and imaginary planes, the part of
    // (c, b) at float offset off(c) + b * bstride + part * PLANE, so each lane reads its own part.
    template <int NCELL, int NW, int PLANE = 0, class Off>
    __device__ __forceinline__ void accumulate(const float2 *stage, int bstride, const float *wsm, Off off, int wave,
                                               int lane) {
        static_assert(PLANE == 0 || MODE != PS_COMPLEX, "the complex form reads both parts");
        constexpr int NG = (NCELL + CPG - 1) / CPG;
        const int slot = lane >> 2, j = lane & 3;
        const int cg = slot >> 1;
        const bool im_slot = (slot & 1) != 0;
        constexpr int UNROLL = MODE == PS_COMPLEX ? 1 : 2;   // the complex form has no registers to spare
#pragma unroll UNROLL
        for (int k = 0; k < (NG + NW - 1) / NW; ++k) {
            const int grp = wave + k * NW;
            if (grp < NG) {
                const int c = grp * CPG + cg;
                const bool ok = NCELL % CPG == 0 || c < NCELL;
                const float w = ok ? wsm[c] : 0.f;
                float x[Q], xo[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const bool in = ok && (NBT % 4 == 0 || 4 * q + j < NBT);
                    if constexpr (PLANE > 0) {
                        const float *sf = reinterpret_cast<const float *>(stage);
                        x[q] = in ? sf[off(c) + (4 * q + j) * bstride + (im_slot ? PLANE : 0)] : 0.f;
                        xo[q] = 0.f;
                    } else {
                        const float2 v = in ? stage[off(c) + (4 * q + j) * bstride] : make_float2(0.f, 0.f);
                        x[q] = im_slot ? v.y : v.x;
                        xo[q] = im_slot ? v.x : v.y;
                    }
                }
                int p = 0;
                if constexpr (PREC == 0) {
#pragma unroll
                    for (int qa = 0; qa < Q; ++qa) {
                        const float aw = w * x[qa];
#pragma unroll
                        for (int qb = qa; qb < Q; ++qb, ++p) {
                            acc[0][p] = __builtin_amdgcn_mfma_f32_4x4x1f32(aw, x[qb], acc[0][p], 0, 0, 0);
                            if constexpr (MODE == PS_COMPLEX)
                                acc[NACC - 1][p] = __builtin_amdgcn_mfma_f32_4x4x1f32(im_slot ? aw : -aw, xo[qb],
                                                                                      acc[NACC - 1][p], 0, 0, 0);
                        }
                    }
                } else {
                    s4v bx[Q], bxo[Q];
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        bx[q] = split_col(x[q]);
                        if constexpr (MODE == PS_COMPLEX) bxo[q] = split_col(xo[q]);
                    }
#pragma unroll
                    for (int qa = 0; qa < Q; ++qa) {
                        const s4v ar = split_row(w * x[qa]);
                        // -(hi + lo) = (-hi) + (-lo) exactly: flip the sign bits
                        const s4v an = ar ^ s4v{(short)0x8000, (short)0x8000, (short)0x8000, 0};
#pragma unroll
                        for (int qb = qa; qb < Q; ++qb, ++p) {
                            acc[0][p] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ar, bx[qb], acc[0][p], 0, 0, 0);
                            if constexpr (MODE == PS_COMPLEX)
                                acc[NACC - 1][p] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(im_slot ? ar : an, bxo[qb],
                                                                                          acc[NACC - 1][p], 0, 0, 0);
                        }
                    }
                }
            }
        }
    }

    // Adds the float32 sums to the float64 totals and clears them.  Recursive halving over the
    // folded lane bits: at bit FB0 + s a lane keeps the half of its values that the bit selects
    // and adds the partner lane's values of that half, so after NFB steps it holds NT2 sums, each
    // over all GS lanes of its group: value index k + sum_s bit_s NVP / 2^(s+1) (value_index).
    __device__ __forceinline__ void flush(int lane) {
        float flat[NVP];
#pragma unroll
        for (int u = 0; u < NACC; ++u)
#pragma unroll
            for (int p = 0; p < NPB; ++p)
#pragma unroll
                for (int r = 0; r < 4; ++r) flat[(u * NPB + p) * 4 + r] = acc[u][p][r];
#pragma unroll
        for (int v = NV; v < NVP; ++v) flat[v] = 0.f;
        halve<0>(flat, lane);
#pragma unroll
        for (int k = 0; k < NT2; ++k) tot[k] += (double)flat[k];
        clear_acc();
    }

    // one halving step of flush (compile-time lengths, so flat stays in registers)
    template <int ST>
    __device__ __forceinline__ static void halve(float *flat, int lane) {
        if constexpr (ST < NFB) {
            constexpr int HALF = NVP >> (ST + 1);
            const bool up = ((lane >> (FB0 + ST)) & 1) != 0;
#pragma unroll
            for (int k = 0; k < HALF; ++k) {
                const float keep = up ? flat[HALF + k] : flat[k];
                const float send = up ? flat[k] : flat[HALF + k];
                flat[k] = keep + __shfl_xor(send, 1 << (FB0 + ST));
            }
            halve<ST + 1>(flat, lane);
        }
    }

    // Value index (into the flattened (accumulator set, pair, r) values) of this lane's total 0.
    __device__ __forceinline__ static int value_index(int lane) {
        int v = 0;
#pragma unroll
        for (int st = 0; st < NFB; ++st)
            if ((lane >> (FB0 + st)) & 1) v += NVP >> (st + 1);
        return v;
    }

    // One tile added and flushed.
    template <int NCELL, int NW, class Off>
    __device__ __forceinline__ void tile(const float2 *stage, int bstride, const float *wsm, Off off, int wave,
                                         int lane) {
        accumulate<NCELL, NW>(stage, bstride, wsm, off, wave, lane);
        flush(lane);
    }

    // Writes this wave's totals to red[((wave * NOUT + part) * NPB + p) * 16 + r * 4 + j] (lane j
    // of a block holds column j; part: the accumulator set, or for PS_PACKED the lane's slot part).
    // Each (part, pair, r, j) is held by exactly one lane of the wave after the flushes.
    __device__ __forceinline__ void to_lds(double *red, int wave, int lane) {
        const int j = lane & 3;
        const int v0 = value_index(lane);
        const int lane_part = MODE == PS_PACKED ? (lane >> 2) & 1 : 0;
#pragma unroll
        for (int k = 0; k < NT2; ++k) {
            const int v = v0 + k;
            if (v < NV) {
                const int u = v / (NPB * 4), p = (v / 4) % NPB, r = v % 4;
                const int part = MODE == PS_PACKED ? lane_part : u;
                red[((wave * NOUT + part) * NPB + p) * 16 + r * 4 + j] = tot[k];
            }
        }
    }

    // Block partial of output v = part * npairs + pair (b1 <= b2, b1 outer): the waves in order.
    __device__ static double block_value(const double *red, int nw, int nb, int v) {
        const int npn = nb * (nb + 1) / 2;
        const int vp = v % npn, part = v / npn;
        int b1 = 0, rem = vp;
        while (rem >= nb - b1) { rem -= nb - b1; ++b1; }
        const int b2 = b1 + rem;
        const int qa = b1 >> 2, qb = b2 >> 2;
        const int p = qa * Q - qa * (qa - 1) / 2 + (qb - qa);
        double sum = 0.0;
        for (int w = 0; w < nw; ++w) sum += red[((w * NOUT + part) * NPB + p) * 16 + (b1 & 3) * 4 + (b2 & 3)];
        return sum;
    }
};

// Row of the block partials for output value v (part-major, npn pairs per part) of grid row y:
// the plan's row map gives the coefficient group of each (grid row, part) when present.
__device__ __forceinline__ int64_t partial_row(const LastArgs &a, int y, int nv, int npn, int v) {
    if (!a.rowmap) return (int64_t)y * nv + v;
    return (int64_t)a.rowmap[2 * y + v / npn] * npn + v % npn;
}

template <int N, int TPP, int NBT, int R, int MODE, int PREC, int... RAD>
__global__ __launch_bounds__(NBT * R * TPP) void last_contract_kernel(LastArgs a) {
    a.in += (int64_t)blockIdx.z * a.in_fs;   // field of the launch (grid.z)
    a.w += (int64_t)blockIdx.z * a.w_fs;
    a.partial += (int64_t)blockIdx.z * a.part_fs;
    using PS = PairSums<NBT, MODE, PREC>;
    constexpr int P = NBT * R, PITCH = P + 1, NT = P * TPP;
    constexpr int NW = NT / 64;       // waves
    constexpr int NOUT = PS::NOUT;
    constexpr int EPT = N / TPP;      // tile elements loaded per thread
    static_assert(NT % 64 == 0, "whole waves");
    extern __shared__ float2 smem[];
    const int nb = a.nb;
    float2 *sm = smem;
    float2 *tw = smem + N * PITCH;
    float *wsm = reinterpret_cast<float *>(tw + N);   // the tile's weights w(x), R N values
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < N; i += NT) tw[i] = a.tw[i];
    PS ps;
    ps.zero();
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
            dst[e] = (row < r_end && b < nb) ? ld_stream(&in[(int64_t)b * a.ng + row * N + j]) : make_float2(0.f, 0.f);
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
        ps.template tile<R * N, NW>(sm, R, wsm, [](int c) { return (c % N) * PITCH + c / N; }, wave, lane);
    }
    // float64 combine over the waves in wave order; partial[(g * nv + v) * nblocks + blk] with
    // v = part * npairs + pair (b1 <= b2, b1 outer), row from partial_row
    __syncthreads();
    double *red = reinterpret_cast<double *>(smem);   // [wave][part][quad pair][4 x 4]
    ps.to_lds(red, wave, lane);
    __syncthreads();
    const int nv = nb * (nb + 1) / 2 * NOUT;
    for (int v = tid; v < nv; v += NT)
        a.partial[partial_row(a, blockIdx.y, nv, nv / NOUT, v) * a.nblocks + blockIdx.x] =
            PS::block_value(red, NW, nb, v);
}

// LDS region of one pencil in the register-resident last pass: it holds the pencil's exchange
// rows and then its transformed row.  The size is 8 mod 16 float2, so the pair sums' reads of
// 4 bins (regions) at 8 adjacent cells fall into distinct banks.
constexpr int pencil_region(int exch, int n) {
    int s = exch > n ? exch : n;
    while (s % 16 != 8) ++s;
    return s;
}

// Orders the LDS accesses of one wave around the call; a pencil's threads are lanes of one wave,
// so its exchange needs no workgroup barrier.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Register-resident form for n = R1 * R2 (R2 threads per row): a tile is one row of the NBT
// (padded) bins of one array group.  Thread q of a pencil loads elements q + R2 s (coalesced: the
// R2 threads of a pencil are adjacent lanes), runs the first radix-R1 stage in registers,
// exchanges through its pencil's LDS region (row q of R1 values written, column q + R2 t read),
// runs the second stage and writes the transformed row into the same region, as separate real
// and imaginary float planes (interleaved complex values for the complex sums), which the MFMA
// pair sums read.  The exchange stays inside a wave; the workgroup meets at two barriers per tile
// (regions written, regions read).  The second-stage twiddles come from an LDS table ordered so
// that the threads of a pencil read adjacent entries, and the pair sums are flushed to float64
// every FLUSH (8) rows.
template <int R1, int R2, int NBT, int MODE, int PREC>
__global__ __launch_bounds__(NBT * R2, NBT <= 12 ? 4 : 3) void last_reg_kernel(LastArgs a) {
    a.in += (int64_t)blockIdx.z * a.in_fs;   // field of the launch (grid.z)
    a.w += (int64_t)blockIdx.z * a.w_fs;
    a.partial += (int64_t)blockIdx.z * a.part_fs;
    using PS = PairSums<NBT, MODE, PREC>;
    constexpr int N = R1 * R2;
    constexpr int T = R1 / R2;             // second-stage butterflies per thread
    static_assert(R1 % R2 == 0 && 64 % R2 == 0, "R2 divides R1 and the wave");
    constexpr int P = NBT;                 // pencils (bins) per tile
    constexpr int NT = P * R2;
    constexpr int NW = NT / 64;
    constexpr int NOUT = PS::NOUT;
    constexpr int EXR = R1 + 1;            // exchange row pitch (R2 rows)
    // the transformed row as separate real and imaginary planes (PLANE = 8 mod 64 floats apart,
    // so a group's reads of both parts fall into distinct banks), except for the complex sums
    constexpr bool SPLIT = MODE != PS_COMPLEX;
    constexpr int PLANE = N + 8;
    static_assert(N % 64 == 0, "plane offset 8 mod 64");
    constexpr int REG = pencil_region(R2 * EXR, SPLIT ? PLANE : N);
    constexpr int WPT = (N + NT - 1) / NT;
    static_assert(NT % 64 == 0, "whole waves");
    constexpr int FLUSH = NBT * PS::NACC <= 12 ? 8 : 1;   // larger accumulators would not stay in registers
    __shared__ float2 lds[P * REG];
    __shared__ float2 twl[N];              // [t][r][q]: w^{(q + R2 t) r}, w = e^{-2 pi i / N}
    __shared__ float wsm[N];
    const int nb = a.nb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = tid % R2, pp = tid / R2;  // element column, pencil (= bin)
    float2 *own = lds + pp * REG;
    for (int i = tid; i < N; i += NT) {
        const int t = i / (R2 * R2), r = i / R2 % R2, qq = i % R2;
        twl[i] = a.tw[((qq + R2 * t) * r) % N];
    }
    PS ps;
    ps.zero();
    const int64_t nrows = a.ng / N;
    const int64_t r_begin = (int64_t)blockIdx.x * a.rows_per_block;
    const int64_t r_end = min(r_begin + a.rows_per_block, nrows);
    const float2 *in = a.in + ((int64_t)blockIdx.y * nb + pp) * a.ng;
    const bool live = pp < nb;
    auto load_row = [&](int64_t row, float2 *dst, float *wdst) {
#pragma unroll
        for (int r = 0; r < R1; ++r) dst[r] = live ? ld_stream(&in[row * N + q + R2 * r]) : make_float2(0.f, 0.f);
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
        // first stage: radix-R1 butterfly q (elements q + R2 s) -> row q of the exchange
        Dft<R1, 1>::run(v);
        __syncthreads();                                    // the previous tile's pair sums are done
#pragma unroll
        for (int r = 0; r < R1; ++r) own[q * EXR + r] = v[r];
        wave_lds_sync();
        // second stage: radix-R2 butterflies q + R2 t over the rows, positions q + R2 t + R1 r
#pragma unroll
        for (int t = 0; t < T; ++t) {
            float2 *u = v + t * R2;
#pragma unroll
            for (int r = 0; r < R2; ++r) {
                const float2 x = own[r * EXR + q + R2 * t];
                if (r == 0) {
                    u[r] = x;
                } else {
                    const float2 w = twl[(t * R2 + r) * R2 + q];   // the inverse takes the conjugate
                    u[r] = cmul(x, make_float2(w.x, -w.y));
                }
            }
            Dft<R2, 1>::run(u);
        }
        wave_lds_sync();                                    // the pencil's exchange rows are read
        if constexpr (SPLIT) {
            float *ownf = reinterpret_cast<float *>(own);
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int r = 0; r < R2; ++r) {
                    ownf[q + R2 * t + R1 * r] = v[t * R2 + r].x;
                    ownf[PLANE + q + R2 * t + R1 * r] = v[t * R2 + r].y;
                }
        } else {
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int r = 0; r < R2; ++r) own[q + R2 * t + R1 * r] = v[t * R2 + r];
        }
#pragma unroll
        for (int e = 0; e < WPT; ++e)
            if (tid + e * NT < N) wsm[tid + e * NT] = wv[e];
        __syncthreads();
        if constexpr (SPLIT)
            ps.template accumulate<N, NW, PLANE>(lds, 2 * REG, wsm, [](int c) { return c; }, wave, lane);
        else
            ps.template accumulate<N, NW>(lds, REG, wsm, [](int c) { return c; }, wave, lane);
        if ((row - r_begin) % FLUSH == FLUSH - 1 || row + 1 == r_end) ps.flush(lane);
    }
    // float64 combine over the waves in wave order (as in last_contract_kernel)
    __syncthreads();
    static_assert(PS::red_doubles(NW) * sizeof(double) <= sizeof(lds), "block reduction fits");
    double *red = reinterpret_cast<double *>(lds);   // [wave][part][quad pair][4 x 4]
    ps.to_lds(red, wave, lane);
    __syncthreads();
    const int nv = nb * (nb + 1) / 2 * NOUT;
    for (int vv = tid; vv < nv; vv += NT)
        a.partial[partial_row(a, blockIdx.y, nv, nv / NOUT, vv) * a.nblocks + blockIdx.x] =
            PS::block_value(red, NW, nb, vv);
}

// bins padded to the instantiated tile widths 4, 8, 12, 16 so that NBT * t threads make whole
// waves (0: none fits)
constexpr int reg_padded_bins(int nb, int t) {
    for (int c = 4; c <= 16; c += 4)
        if (c >= nb && (c * t) % 64 == 0) return c;
    return 0;
}

// Pair-sum mode of a launch.
inline int pair_mode(const LastArgs &a) { return a.want_imag ? PS_COMPLEX : (a.packed ? PS_PACKED : PS_REAL); }

template <int R1, int R2, int PREC>
hipError_t launch_last_reg_p(const LastArgs &a, hipStream_t s) {
    dim3 grid((unsigned)a.nblocks, (unsigned)a.groups, (unsigned)(a.fields > 1 ? a.fields : 1));
    const int mode = pair_mode(a);
    const int nbt = reg_padded_bins(a.nb, R2);
#define SB_LR(NBT)                                                                                                  \
    case NBT:                                                                                                        \
        if constexpr ((NBT * R2) % 64 == 0) {                                                                        \
            if (mode == PS_COMPLEX)                                                                                  \
                hipLaunchKernelGGL((last_reg_kernel<R1, R2, NBT, PS_COMPLEX, PREC>), grid, dim3(NBT * R2), 0, s, a); \
            else if (mode == PS_PACKED)                                                                              \
                hipLaunchKernelGGL((last_reg_kernel<R1, R2, NBT, PS_PACKED, PREC>), grid, dim3(NBT * R2), 0, s, a);  \
            else                                                                                                     \
                hipLaunchKernelGGL((last_reg_kernel<R1, R2, NBT, PS_REAL, PREC>), grid, dim3(NBT * R2), 0, s, a);    \
            break;                                                                                                   \
        } else {                                                                                                     \
            return hipErrorInvalidValue;                                                                             \
        }
    switch (nbt) {
        SB_LR(4) SB_LR(8) SB_LR(12) SB_LR(16)
        default: return hipErrorInvalidValue;
    }
#undef SB_LR
    return hipGetLastError();
}

template <int R1, int R2>
hipError_t launch_last_reg(const LastArgs &a, hipStream_t s) {
    if (a.rows != 1) return hipErrorInvalidValue;
    return a.prec ? launch_last_reg_p<R1, R2, 1>(a, s) : launch_last_reg_p<R1, R2, 0>(a, s);
}

// Register-resident form for any radix list R0, ... (each radix divides R0; see reg_stages):
// a tile is one row of the NBT (padded) bins of one (l, m); thread q < T = n / R0 of a
// pencil loads elements q + T s.  The stages exchange through one LDS buffer laid out
// [position][bin], which, once the last stage has read it, takes the transformed row as the
// [cell][bin] tile of the MFMA pair sums (one more barrier per row).  Two buffers (one barrier
// fewer) would not fit the LDS at 1024 points, and below that they held the workgroups per CU
// under what the registers allow (one buffer: uneven 64-192^3 forward 401 -> 412 fields/s).
template <int N, int NBT, int MODE, int PREC, int R0, int... REST>
__global__ __launch_bounds__(NBT * (N / R0)) void last_rs_kernel(LastArgs a) {
    a.in += (int64_t)blockIdx.z * a.in_fs;   // field of the launch (grid.z)
    a.w += (int64_t)blockIdx.z * a.w_fs;
    a.partial += (int64_t)blockIdx.z * a.part_fs;
    using PS = PairSums<NBT, MODE, PREC>;
    constexpr int T = N / R0;
    constexpr int P = NBT;
    constexpr int NT = P * T;
    constexpr int NW = NT / 64;
    constexpr int NOUT = PS::NOUT;
    constexpr int PITCH = P + 1;
    // the transform's stages at 512 and 1024 points (first radix 16) keep position j of pencil p
    // at j PITCH + p + j / 16: the first stage writes positions q R0 + r, which without the skew
    // put a pencil's threads a multiple of 16 float2 (the width of the 32 banks) apart, all in one
    // bank.  The [cell][bin] view written after the last stage keeps the plain layout.
    constexpr int SKEW = N >= 512 ? 1 : 0, GSH = 4;
    constexpr int NSTAGE = 1 + sizeof...(REST);
    constexpr int WPT = (N + NT - 1) / NT;
    static_assert(NT % 64 == 0 && NSTAGE >= 2, "whole waves, two stages or more");
    __shared__ float2 ex[N * PITCH + (N >> GSH) * SKEW];
    __shared__ float2 tw[N];
    __shared__ float wsm[N];
    const int nb = a.nb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = tid % T, pp = tid / T;        // element column, pencil (= bin)
    for (int i = tid; i < N; i += NT) tw[i] = a.tw[i];
    PS ps;
    ps.zero();
    const int64_t nrows = a.ng / N;
    const int64_t r_begin = (int64_t)blockIdx.x * a.rows_per_block;
    const int64_t r_end = min(r_begin + a.rows_per_block, nrows);
    const float2 *in = a.in + ((int64_t)blockIdx.y * nb + pp) * a.ng;
    const bool live = pp < nb;
    auto load_row = [&](int64_t row, float2 *dst, float *wdst) {
#pragma unroll
        for (int r = 0; r < R0; ++r) dst[r] = live ? ld_stream(&in[row * N + q + T * r]) : make_float2(0.f, 0.f);
#pragma unroll
        for (int e = 0; e < WPT; ++e) {
            const int c = tid + e * NT;
            wdst[e] = c < N ? a.w[row * N + c] : 0.f;
        }
    };
    // PF: the next row's loads are in flight during this row.  The registers allow it except for
    // the 1024-point tiles of more than 8 bins; there the next row loads into the row's own
    // registers once they are stored to LDS, so its loads are in flight during the pair sums.
    constexpr bool PF = N < 1024 || NBT <= 8;
    float2 nx[PF ? R0 : 1];
    float nw[PF ? WPT : 1];
    float2 v[R0];
    float wv[WPT];
    if (r_begin < r_end) {
        if constexpr (PF) load_row(r_begin, nx, nw);
        else load_row(r_begin, v, wv);
    }
    for (int64_t row = r_begin; row < r_end; ++row) {
        if constexpr (PF) {
#pragma unroll
            for (int r = 0; r < R0; ++r) v[r] = nx[r];
#pragma unroll
            for (int e = 0; e < WPT; ++e) wv[e] = nw[e];
            if (row + 1 < r_end) load_row(row + 1, nx, nw);    // next row in flight
        }
        __syncthreads();                                    // the previous row's pair sums are done
        reg_stages<N, 1, R0, REST...>(v, ex, ex, tw, q, pp, PITCH, SKEW, GSH);
        float2 *cs = ex;
        __syncthreads();                                    // the last stage has read the buffer
#pragma unroll
        for (int r = 0; r < R0; ++r) cs[(q + T * r) * PITCH + pp] = v[r];
#pragma unroll
        for (int e = 0; e < WPT; ++e)
            if (tid + e * NT < N) wsm[tid + e * NT] = wv[e];
        __syncthreads();
        if constexpr (!PF)
            if (row + 1 < r_end) load_row(row + 1, v, wv);   // in flight during the pair sums
        ps.template tile<N, NW>(cs, 1, wsm, [](int c) { return c * PITCH; }, wave, lane);
    }
    // float64 combine over the waves in wave order (as in last_contract_kernel)
    __syncthreads();
    static_assert(PS::red_doubles(NW) * sizeof(double) <= sizeof(ex), "block reduction fits");
    double *red = reinterpret_cast<double *>(ex);
    ps.to_lds(red, wave, lane);
    __syncthreads();
    const int nv = nb * (nb + 1) / 2 * NOUT;
    for (int vv = tid; vv < nv; vv += NT)
        a.partial[partial_row(a, blockIdx.y, nv, nv / NOUT, vv) * a.nblocks + blockIdx.x] =
            PS::block_value(red, NW, nb, vv);
}

// (1024 points: at most 12 bins, as last_rows<1024> allows; wider tiles would spill)
template <int N, int PREC, int R0, int... REST>
hipError_t launch_last_rs_p(const LastArgs &a, hipStream_t s) {
    constexpr int T = N / R0;
    dim3 grid((unsigned)a.nblocks, (unsigned)a.groups, (unsigned)(a.fields > 1 ? a.fields : 1));
    const int mode = pair_mode(a);
    const int nbt = reg_padded_bins(a.nb, T);
#define SB_LR(NBT)                                                                                                   \
    case NBT:                                                                                                         \
        if constexpr ((NBT * T) % 64 == 0 && NBT * T <= 1024 && (N < 1024 || NBT <= 12)) {                           \
            if (mode == PS_COMPLEX)                                                                                   \
                hipLaunchKernelGGL((last_rs_kernel<N, NBT, PS_COMPLEX, PREC, R0, REST...>), grid, dim3(NBT * T), 0, s, \
                                   a);                                                                                \
            else if (mode == PS_PACKED)                                                                               \
                hipLaunchKernelGGL((last_rs_kernel<N, NBT, PS_PACKED, PREC, R0, REST...>), grid, dim3(NBT * T), 0, s,  \
                                   a);                                                                                \
            else                                                                                                      \
                hipLaunchKernelGGL((last_rs_kernel<N, NBT, PS_REAL, PREC, R0, REST...>), grid, dim3(NBT * T), 0, s, a); \
            break;                                                                                                    \
        } else {                                                                                                      \
            return hipErrorInvalidValue;                                                                              \
        }
    switch (nbt) {
        SB_LR(4) SB_LR(8) SB_LR(12) SB_LR(16)
        default: return hipErrorInvalidValue;
    }
#undef SB_LR
    return hipGetLastError();
}

template <int N, int R0, int... REST>
hipError_t launch_last_rs(const LastArgs &a, hipStream_t s) {
    if (a.rows != 1) return hipErrorInvalidValue;
    return a.prec ? launch_last_rs_p<N, 1, R0, REST...>(a, s) : launch_last_rs_p<N, 0, R0, REST...>(a, s);
}

template <int N, int TPP, int NBT, int MODE, int... RAD>
hipError_t launch_last_t(const LastArgs &a, hipStream_t s) {
    constexpr int R = fused_rows(N, TPP, NBT);
    constexpr int P = NBT * R, NT = P * TPP;
    if (a.rows != R) return hipErrorInvalidValue;
    const size_t tile = (size_t)(N * (P + 1) + N) * sizeof(float2) + (size_t)R * N * sizeof(float);
    const size_t red = (size_t)PairSums<NBT, MODE>::red_doubles(NT / 64) * sizeof(double);
    const size_t shm = tile > red ? tile : red;
    dim3 grid((unsigned)a.nblocks, (unsigned)a.groups, (unsigned)(a.fields > 1 ? a.fields : 1));
    if (a.prec)
        hipLaunchKernelGGL((last_contract_kernel<N, TPP, NBT, R, MODE, 1, RAD...>), grid, dim3(NT), shm, s, a);
    else
        hipLaunchKernelGGL((last_contract_kernel<N, TPP, NBT, R, MODE, 0, RAD...>), grid, dim3(NT), shm, s, a);
    return hipGetLastError();
}

constexpr int padded_bins(int nb) { return nb <= 4 ? 4 : nb <= 8 ? 8 : nb <= 10 ? 10 : nb <= 12 ? 12 : 16; }

template <int N, int TPP, int NBT, int... RAD>
hipError_t launch_last_m(const LastArgs &a, hipStream_t s) {
    switch (pair_mode(a)) {
        case PS_COMPLEX: return launch_last_t<N, TPP, NBT, PS_COMPLEX, RAD...>(a, s);
        case PS_PACKED: return launch_last_t<N, TPP, NBT, PS_PACKED, RAD...>(a, s);
        default: return launch_last_t<N, TPP, NBT, PS_REAL, RAD...>(a, s);
    }
}

template <int N, int TPP, int... RAD>
hipError_t launch_last_nb(const LastArgs &a, hipStream_t s) {
    switch (padded_bins(a.nb)) {
        case 4: return launch_last_m<N, TPP, 4, RAD...>(a, s);
        case 8: return launch_last_m<N, TPP, 8, RAD...>(a, s);
        case 10: return launch_last_m<N, TPP, 10, RAD...>(a, s);
        case 12: return launch_last_m<N, TPP, 12, RAD...>(a, s);
        default: return launch_last_m<N, TPP, 16, RAD...>(a, s);
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
