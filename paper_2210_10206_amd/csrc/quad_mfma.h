// Full-4PCF contraction on the matrix cores, one kernel per ordered Lambda = (LA, LB, LC).
// Even Lambda give the real part of the sums below, odd Lambda (LA + LB + LC odd) the
// imaginary part (the other part vanishes for a real density).
//
// For one Lambda, with mc >= 0 and the weighted 3j symbols C (factor 2 for mc > 0, Alg. 6):
//   L_mc[b1 b2](x) = w(x) sum_ma C(ma, mb, mc) a^b1_{LA,ma}(x) a^b2_{LB,mb}(x),  mb = -ma - mc
//   Z[b1 b2][b3]  += sum_x Re( L_mc[b1 b2](x) a^b3_{LC,mc}(x) )
// (the kernels multiply w(x) into a^b3 instead of L: the same sums for fewer products).
// The coupling (first line) runs on the vector ALUs with every coefficient index known at
// compile time, so the per-lane coefficients stay in registers; the contraction over the
// cells (second line) is a real GEMM with M = b1 b2 pairs (tiles of 16), N = b3 (padded to
// 16) and K = (cell, re/im) that runs on MFMA:
//   PREC 0: v_mfma_f32_16x16x4f32, K = the cells of the four lane groups, re and im in turn;
//   PREC 1: v_mfma_f32_16x16x32_bf16 with both operands split into bf16 hi + lo parts and
//           hi*hi + hi*lo + lo*hi accumulated in float32 (split-BF16); each lane group
//           fills six of its eight K slots (the three split products of re and im of its
//           cell), one instruction per product.
// Lane l of a wave is (i = l % 16, g = l / 16): row i of each A tile, column i of the B tile
// (bin b3 = i); the lane walks cells 4 g .. 4 g + 3 of the wave's 16-cell step in turn.
#pragma once
#include <utility>
#include "sb_kgen.h"

namespace sb {
namespace quadm {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int kTileCells = 64;   // cells staged per LDS tile (16 per wave)
constexpr int kMaxNB = 8;        // bins (pairs fill at most 4 tiles of 16)

// Pairs of the M tiles.  General Lambda: row i of tile mt is (b1, b2) = (2 mt + i / 8, i % 8),
// 4 tiles.  LA == LB: swapping the first two 3j columns multiplies the symbol by
// (-1)^(LA + LB + LC), so Z[b1][b2][b3] = +-Z[b2][b1][b3] and only the 36 pairs b1 <= b2 are
// computed, in 3 tiles: row i has one b2 (rows 0-2: 7, 3-5: 6, 6-7: 5, 8-9: 4, 10-11: 3, 12: 2,
// 13: 1, 14: 0, 15: none) and the b1 <= b2 of that b2 in turn over the tiles (-1: empty slot).
// In both layouts a lane keeps one b2 in all its tiles.
struct SymPairs {
    int b2[16];
    int b1[3][16];
};
constexpr SymPairs make_sym_pairs() {
    SymPairs t{};
    for (int i = 0; i < 16; ++i) {
        t.b2[i] = 0;
        for (int mt = 0; mt < 3; ++mt) t.b1[mt][i] = -1;
    }
    int row = 0;
    for (int b2 = kMaxNB - 1; b2 >= 0; --b2)
        for (int b1 = 0; b1 <= b2; ++row)
            for (int mt = 0; mt < 3 && b1 <= b2; ++mt, ++b1) {
                t.b2[row] = b2;
                t.b1[mt][row] = b1;
            }
    return t;
}
constexpr SymPairs kSym = make_sym_pairs();
static_assert(kSym.b2[14] == 0 && kSym.b1[0][14] == 0 && kSym.b1[0][15] == -1, "36 pairs in 15 rows");

// staged columns: distinct l values in the order LA, LB, LC; column = offset + m
template <int LA, int LB, int LC> struct Cols {
    static constexpr int offA = 0;
    static constexpr int offB = (LB == LA) ? 0 : LA + 1;
    static constexpr int offC = (LC == LA) ? 0 : (LC == LB ? offB : ((LB == LA) ? LA + 1 : LA + 1 + LB + 1));
    static constexpr int ncol = (LB == LA ? LA + 1 : LA + 1 + LB + 1) + ((LC == LA || LC == LB) ? 0 : LC + 1);
    static constexpr int lm_of(int col) {
        return col < LA + 1 ? LA * (LA + 1) / 2 + col
               : (LB != LA && col < LA + 1 + LB + 1) ? LB * (LB + 1) / 2 + (col - LA - 1)
                                                      : LC * (LC + 1) / 2 + (col - offC);
    }
};

// a_{l,m} for a signed m from the stored m >= 0 value: a_{l,-m} = (-1)^m conj(a_{l,m})
template <int M>
__device__ __forceinline__ float2 signed_m(float2 v) {
    if constexpr (M >= 0) return v;
    else if constexpr (((-M) & 1) == 0) return make_float2(v.x, -v.y);
    else return make_float2(-v.x, v.y);
}

template <int LA, int LB, int MC, int MA, int T, int NMT>
struct Couple {
    // add the terms ma = MA .. LA of one mc to L[mt] for every M tile; T = index of the term
    // in the table.  The 3j weight multiplies the b2 operand once (it is the same bin b2 in
    // every tile of a lane) and the product with the b1 operand of each tile is 4 FMAs.
    __device__ __forceinline__ static void run(const float *cw, const float2 (*A1)[LA + 1], const float2 *A2,
                                               float2 *L) {
        if constexpr (MA > LA) {
            return;
        } else {
            constexpr int MB = -MA - MC;
            if constexpr (MB >= -LB && MB <= LB) {
                const float c = cw[T];
                const float2 y = signed_m<MB>(A2[MB >= 0 ? MB : -MB]);
                // a_{l0} is real (real field, real Y_l0): m = 0 operands use their real part only
                const float2 u = MB == 0 ? make_float2(c * y.x, 0.f) : make_float2(c * y.x, c * y.y);
#pragma unroll
                for (int mt = 0; mt < NMT; ++mt) {
                    const float2 x = signed_m<MA>(A1[mt][MA >= 0 ? MA : -MA]);
                    if constexpr (MA == 0) {
                        L[mt].x = __builtin_fmaf(x.x, u.x, L[mt].x);
                        L[mt].y = __builtin_fmaf(x.x, u.y, L[mt].y);
                    } else if constexpr (MB == 0) {
                        L[mt].x = __builtin_fmaf(x.x, u.x, L[mt].x);
                        L[mt].y = __builtin_fmaf(x.y, u.x, L[mt].y);
                    } else {
                        L[mt].x = __builtin_fmaf(x.x, u.x, L[mt].x);
                        L[mt].x = __builtin_fmaf(-x.y, u.y, L[mt].x);
                        L[mt].y = __builtin_fmaf(x.x, u.y, L[mt].y);
                        L[mt].y = __builtin_fmaf(x.y, u.x, L[mt].y);
                    }
                }
                Couple<LA, LB, MC, MA + 1, T + 1, NMT>::run(cw, A1, A2, L);
            } else {
                Couple<LA, LB, MC, MA + 1, T, NMT>::run(cw, A1, A2, L);
            }
        }
    }
};

// mc = 0 of an even Lambda: the terms ma and -ma are complex conjugates of each other
// (a_{l,-m} = (-1)^m conj a_{lm} and the 3j symbol is even under m -> -m when l1 + l2 + l3 is
// even), so L_0 = C_0 a^b1_{LA,0} a^b2_{LB,0} + sum_{ma > 0} 2 (-1)^ma C_ma Re(a^b1_{LA,ma}
// conj a^b2_{LB,ma}) is real: 2 FMAs per ma > 0 instead of 8, and one MFMA instead of two.
// C_ma is the table entry of (ma, -ma, 0), at position ma + min(LA, LB) of the mc = 0 terms.
// mc = 0 of an odd Lambda: the pair (ma, -ma) gives 2 i (-1)^ma C_ma Im(a^b1_{LA,ma} conj
// a^b2_{LB,ma}) (the 3j symbol is odd under m -> -m, and the ma = 0 symbol vanishes), so L_0
// is imaginary: L_0.y = sum_{ma > 0} 2 (-1)^ma C_ma (x.y y.x - x.x y.y).
template <int LA, int LB, int MA, int NMT>
struct Couple0Odd {
    __device__ __forceinline__ static void run(const float *cw, const float2 (*A1)[LA + 1], const float2 *A2,
                                               float2 *L) {
        if constexpr (MA > LA || MA > LB) {
            return;
        } else {
            if constexpr (MA > 0) {
                constexpr int T = MA + (LA < LB ? LA : LB);
                const float c = ((MA & 1) ? -2.f : 2.f) * cw[T];
                const float2 u = make_float2(c * A2[MA].x, c * A2[MA].y);
#pragma unroll
                for (int mt = 0; mt < NMT; ++mt) {
                    L[mt].y = __builtin_fmaf(A1[mt][MA].y, u.x, L[mt].y);
                    L[mt].y = __builtin_fmaf(-A1[mt][MA].x, u.y, L[mt].y);
                }
            }
            Couple0Odd<LA, LB, MA + 1, NMT>::run(cw, A1, A2, L);
        }
    }
};

template <int LA, int LB, int MA, int NMT>
struct Couple0 {
    __device__ __forceinline__ static void run(const float *cw, const float2 (*A1)[LA + 1], const float2 *A2,
                                               float2 *L) {
        if constexpr (MA > LA || MA > LB) {
            return;
        } else {
            constexpr int T = MA + (LA < LB ? LA : LB);
            if constexpr (MA == 0) {
                const float u = cw[T] * A2[0].x;
#pragma unroll
                for (int mt = 0; mt < NMT; ++mt) L[mt].x = __builtin_fmaf(A1[mt][0].x, u, L[mt].x);
            } else {
                const float c = ((MA & 1) ? -2.f : 2.f) * cw[T];
                const float2 u = make_float2(c * A2[MA].x, c * A2[MA].y);
#pragma unroll
                for (int mt = 0; mt < NMT; ++mt) {
                    L[mt].x = __builtin_fmaf(A1[mt][MA].x, u.x, L[mt].x);
                    L[mt].x = __builtin_fmaf(A1[mt][MA].y, u.y, L[mt].x);
                }
            }
            Couple0<LA, LB, MA + 1, NMT>::run(cw, A1, A2, L);
        }
    }
};

// number of terms with mc < MC (offset of mc's first term in the table)
template <int LA, int LB> constexpr int terms_before(int MC) {
    int t = 0;
    for (int mc = 0; mc < MC; ++mc)
        for (int ma = -LA; ma <= LA; ++ma) {
            const int mb = -ma - mc;
            if (mb >= -LB && mb <= LB) ++t;
        }
    return t;
}

__device__ __forceinline__ void split_bf16(float v, __bf16 &hi, __bf16 &lo) {
    hi = (__bf16)v;
    lo = (__bf16)(v - (float)hi);
}

// Pair layout of the M tiles: lane row i of tile mt is (b1, b2) = (2 mt + i / 8, i % 8), so a
// lane keeps the same b2 in all four tiles; pairs with a bin >= nbins hold zeros.
//
// Staging: a tile of 64 cells sits in LDS cell-major, one row of NCOL x 8 float2 per cell padded
// to S = 8 NCOL + 2 float2.  S = 2 (mod 8) makes both LDS phases free of bank conflicts: the
// stores (64 consecutive cells of one (column, bin) per wave instruction, c S mod 32 distinct
// over 16 lanes) and the per-lane reads (cells 4 apart in the four lane groups land 8 float2
// apart, bins fill the slots between).  The next tile's global loads are issued into registers
// before the current tile is contracted, so their latency hides behind the coupling work.
// Workgroups per CU the kernel is compiled for: 4 (4 waves per SIMD, at most 128 VGPRs) for the
// float32 forms that fit that without spilling, else 1 (the compiler's own choice, 2-3 waves per
// SIMD).  The excluded Lambda spill at 128 VGPRs (resource usage of this compiler); the split-BF16
// forms, with their extra split registers, keep the compiler's choice.
constexpr bool quad_spills_at_128(int la, int lb, int lc) {
    constexpr int ex[][3] = {{3, 3, 4}, {3, 4, 3}, {3, 4, 4}, {4, 1, 4}, {4, 2, 2},
                             {4, 2, 4}, {4, 3, 3}, {4, 3, 4}, {4, 4, 2}, {4, 4, 3}};
    for (const auto &e : ex)
        if (e[0] == la && e[1] == lb && e[2] == lc) return true;
    return false;
}
constexpr int quad_blocks_per_cu(int la, int lb, int lc, int prec) {
    return prec == 0 && !quad_spills_at_128(la, lb, lc) ? 4 : 1;
}

template <int LA, int LB, int LC, int PREC>
__global__ __launch_bounds__(256, quad_blocks_per_cu(LA, LB, LC, PREC)) void quad_mfma_kernel(QuadMArgs a) {
    a.coef += (int64_t)blockIdx.z * a.coef_fs;   // field of the launch (grid.z)
    a.w += (int64_t)blockIdx.z * a.w_fs;
    a.partial += (int64_t)blockIdx.z * a.part_fs;
    constexpr bool ODD = ((LA + LB + LC) & 1) != 0;
    constexpr bool SYM = LA == LB;                // only the pairs b1 <= b2 (SymPairs)
    constexpr int NMT = SYM ? 3 : 4;              // M tiles of 16 pairs
    using CL = Cols<LA, LB, LC>;
    constexpr int NCOL = CL::ncol;
    constexpr int TC = kTileCells;
    constexpr int S = NCOL * kMaxNB + 2;          // float2 per staged cell row
    constexpr int NLD = NCOL * kMaxNB * TC / 256; // float2 loads per thread and tile
    constexpr int NRED = 4 * kMaxNB * kMaxNB * kMaxNB;
    constexpr int NTILE = TC * S > NRED / 2 ? TC * S : NRED / 2;
    __shared__ float2 tile[NTILE];
    __shared__ float wt[TC];
    float *red = reinterpret_cast<float *>(tile);   // reused for the block reduction at the end
    const int nb = a.nbins;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: row addresses stay scalar
    const int i = lane & 15, g = lane >> 4;
    const int b2 = SYM ? kSym.b2[i] : (i & 7);
    int b1s[NMT];   // b1 of this lane's row in each tile (-1: empty slot)
#pragma unroll
    for (int mt = 0; mt < NMT; ++mt) b1s[mt] = SYM ? kSym.b1[mt][i] : 2 * mt + (i >> 3);
    const float *cw = a.coefw;   // weighted 3j values of this Lambda, table order (mc outer, ma inner)
    f4v acc[NMT];
#pragma unroll
    for (int mt = 0; mt < NMT; ++mt) acc[mt] = f4v{0.f, 0.f, 0.f, 0.f};
    const int64_t c0 = (int64_t)blockIdx.x * a.cells_per_block;
    const int64_t c1 = min(c0 + a.cells_per_block, a.ng);
    // load k of this thread: cell = lane, (column, bin) row = wave + 4 k
    float2 pf[NLD];
    float pw = 0.f;
    // coefficient array and part of each load (packed m = 0 arrays hold two real columns)
    int karr[NLD], kpart[NLD];
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
        const int lm = CL::lm_of((wave + 4 * k) / kMaxNB);
        karr[k] = a.lm_src ? a.lm_src[2 * lm] : lm;
        kpart[k] = a.lm_src ? a.lm_src[2 * lm + 1] : 0;
    }
    auto gload = [&](int64_t tc) {
        const bool in = tc + lane < c1;
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int kb = wave + 4 * k;
            const int b = kb % kMaxNB;
            const float2 *src = a.coef + ((int64_t)karr[k] * nb + b) * a.ng + tc;
            pf[k] = (in && b < nb) ? src[lane] : make_float2(0.f, 0.f);   // part taken when staged
        }
        if (wave == 0) pw = in ? a.w[tc + lane] : 0.f;
    };
    gload(c0);
    for (int64_t tc = c0; tc < c1; tc += TC) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            const int kb = wave + 4 * k;
            float2 v = pf[k];
            if (kpart[k] == 1) v.y = 0.f;                       // packed m = 0 column: one real part
            else if (kpart[k] == 2) v = make_float2(v.y, 0.f);
            tile[lane * S + kb] = v;   // kb = column * 8 + bin
        }
        if (wave == 0) wt[lane] = pw;
        __syncthreads();
        if (tc + TC < c1) gload(tc + TC);
        // this lane's cells: 16 wave + 4 g + cc, one at a time (K of the MFMA = the lane groups)
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            const float2 *row = tile + (16 * wave + 4 * g + cc) * S;
            const float wv = wt[16 * wave + 4 * g + cc];
            float2 A1[NMT][LA + 1], A2[LB + 1], bv[LC + 1];
#pragma unroll
            for (int mt = 0; mt < NMT; ++mt)
#pragma unroll
                for (int m = 0; m <= LA; ++m)   // zero beyond nbins
                    A1[mt][m] = (!SYM || b1s[mt] >= 0) ? row[(CL::offA + m) * kMaxNB + b1s[mt]] : make_float2(0.f, 0.f);
#pragma unroll
            for (int m = 0; m <= LB; ++m) A2[m] = row[(CL::offB + m) * kMaxNB + b2];
            // the weight w(x) goes with the b3 operand: LC + 1 values per cell instead of NMT (LA + 1)
#pragma unroll
            for (int mc = 0; mc <= LC; ++mc) {
                const float2 v = i < kMaxNB ? row[(CL::offC + mc) * kMaxNB + i] : make_float2(0.f, 0.f);
                bv[mc] = make_float2(wv * v.x, wv * v.y);
            }
            // one mc: couple, then contract on the matrix cores (unrolled over mc below)
            auto step = [&](auto mc_c) {
                constexpr int MC = decltype(mc_c)::value;
                float2 L[NMT];
#pragma unroll
                for (int mt = 0; mt < NMT; ++mt) L[mt] = make_float2(0.f, 0.f);
                if constexpr (MC == 0 && !ODD)
                    Couple0<LA, LB, 0, NMT>::run(cw, A1, A2, L);
                else if constexpr (MC == 0)
                    Couple0Odd<LA, LB, 0, NMT>::run(cw, A1, A2, L);
                else
                    Couple<LA, LB, MC, -LA, terms_before<LA, LB>(MC), NMT>::run(cw, A1, A2, L);
                // even: Re(L a) = L.x a.x - L.y a.y;  odd: Im(L a) = L.y a.x + L.x a.y.  For mc = 0
                // a_{l0} is real and L_0 is real (even) or imaginary (odd): one product.
                if constexpr (PREC == 0) {
#pragma unroll
                    for (int mt = 0; mt < NMT; ++mt) {
                        if constexpr (!ODD) {
                            acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(L[mt].x, bv[MC].x, acc[mt], 0, 0, 0);
                            if constexpr (MC > 0)
                                acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(-L[mt].y, bv[MC].y, acc[mt], 0, 0, 0);
                        } else {
                            acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(L[mt].y, bv[MC].x, acc[mt], 0, 0, 0);
                            if constexpr (MC > 0)
                                acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(L[mt].x, bv[MC].y, acc[mt], 0, 0, 0);
                        }
                    }
                } else {
                    // K slots 8 g .. 8 g + 5 of lane group g carry the split products of its cell's two
                    // terms a0 b0 + a1 b1 (even: a = (Lr, -Li), b = (Br, Bi); odd: a = (Li, Lr)):
                    //   row (a0_h, a0_h, a0_l, a1_h, a1_h, a1_l, 0, 0), column (b0_h, b0_l, b0_h, b1_h, b1_l, b1_h, 0, 0)
                    // so one instruction adds hi*hi + hi*lo + lo*hi of both (the lo*lo terms dropped)
                    __bf16 h0, l0, h1, l1;
                    split_bf16(bv[MC].x, h0, l0);
                    split_bf16(bv[MC].y, h1, l1);
                    const bf8v bop = {h0, l0, h0, h1, l1, h1, (__bf16)0.f, (__bf16)0.f};
#pragma unroll
                    for (int mt = 0; mt < NMT; ++mt) {
                        split_bf16(ODD ? L[mt].y : L[mt].x, h0, l0);
                        split_bf16(ODD ? L[mt].x : -L[mt].y, h1, l1);
                        const bf8v aop = {h0, h0, l0, h1, h1, l1, (__bf16)0.f, (__bf16)0.f};
                        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop, acc[mt], 0, 0, 0);
                    }
                }
            };
            [&]<int... MCS>(std::integer_sequence<int, MCS...>) {
                (step(std::integral_constant<int, MCS>{}), ...);
            }(std::make_integer_sequence<int, LC + 1>{});
        }
    }
    // accumulator tile mt: lane l holds rows 4 g + r (their pairs as laid out above), column i
    // (bin b3)
    __syncthreads();
    const int nv = nb * nb * nb;
    for (int v = tid; v < 4 * nv; v += 256) red[v] = 0.f;
    __syncthreads();
#pragma unroll
    for (int mt = 0; mt < NMT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ro = 4 * g + r, pr = 16 * mt + ro;
            const int p1 = SYM ? kSym.b1[mt][ro] : pr >> 3;
            const int p2 = SYM ? kSym.b2[ro] : pr & 7;
            if (p1 >= 0 && p1 < nb && p2 < nb && i < nb) red[wave * nv + (p1 * nb + p2) * nb + i] = acc[mt][r];
        }
    __syncthreads();
    for (int v = tid; v < nv; v += 256) {
        int vs = v;
        double sg = 1.0;
        if constexpr (SYM) {   // b1 > b2: the mirrored pair (sign -1 for odd Lambda)
            const int p1 = v / (nb * nb), p2 = (v / nb) % nb, b3 = v % nb;
            if (p1 > p2) {
                vs = (p2 * nb + p1) * nb + b3;
                sg = ODD ? -1.0 : 1.0;
            }
        }
        const double s = ((double)red[vs] + (double)red[nv + vs]) + ((double)red[2 * nv + vs] + (double)red[3 * nv + vs]);
        a.partial[((int64_t)a.lam * nv + v) * a.nblocks + blockIdx.x] = sg * s;
    }
}

template <int LA, int LB, int LC>
hipError_t launch_lambda(const QuadMArgs &a, hipStream_t s) {
    dim3 grid((unsigned)a.nblocks, 1u, (unsigned)(a.fields > 1 ? a.fields : 1));
    if (a.precision == 1)
        hipLaunchKernelGGL((quad_mfma_kernel<LA, LB, LC, 1>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((quad_mfma_kernel<LA, LB, LC, 0>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace quadm
}  // namespace sb
