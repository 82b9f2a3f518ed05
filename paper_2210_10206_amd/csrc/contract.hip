// Grid-sum contractions of the expansion coefficients with the density.
//
// Every contraction writes float32-accumulated, float64-combined block partials:
// a thread sums its share of a block's cells in float32, the block combines its
// threads in float64 (wave shuffles, then LDS), and launch_block_sum adds the
// blocks in float64 in a fixed order.  Results are bit-reproducible run to run.
//
//  pair  : sum_x w(x) A^b1(x) conj(A^b2(x)), b1 <= b2, per coefficient group
//          (full 3PCF of Alg. 5 per (l, m >= 0); projected 3PCF of Alg. 7 per m)
//  quad  : Re sum_x w(x) sum_M 3j a a a for one canonical Lambda (full 4PCF, Alg. 6)
//  proj4 : sum_x w(x) c_m1 c_m2 c_m3 for one canonical (m1, m2) (projected 4PCF, Alg. 8)
#include "sb_kgen.h"

#include <algorithm>

namespace sb {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Combine NV float32 per-thread totals of a 256-thread block into float64 and write
// them to partial[(g * nv + v) * nblocks + blk].
template <int NV>
__device__ __forceinline__ void block_combine(const float *acc, double *red /* LDS 4*NV */, double *partial,
                                              int g, int blk, int nblocks) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double s = wave_sum((double)acc[v]);
        if (lane == 0) red[wave * NV + v] = s;
    }
    __syncthreads();
    for (int v = threadIdx.x; v < NV; v += blockDim.x) {
        const double s = ((red[v] + red[NV + v]) + (red[2 * NV + v] + red[3 * NV + v]));
        partial[((int64_t)g * NV + v) * nblocks + blk] = s;
    }
}

// ----------------------------------------------------------------- pair contraction
template <int NB, bool IMAG>
__global__ __launch_bounds__(256) void pair_kernel(PairArgs a) {
    a.coef += (int64_t)blockIdx.z * a.coef_fs;   // field of the launch (grid.z)
    a.w += (int64_t)blockIdx.z * a.w_fs;
    a.partial += (int64_t)blockIdx.z * a.part_fs;
    constexpr int NP = NB * (NB + 1) / 2;
    constexpr int NV = NP * (IMAG ? 2 : 1);
    __shared__ double red[4 * NV];
    float acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.f;
    const int g = blockIdx.y, blk = blockIdx.x;
    const float2 *A = a.coef + (int64_t)g * a.gstride;
    const int64_t c0 = (int64_t)blk * a.cells_per_block;
    const int64_t c1 = min(c0 + a.cells_per_block, a.ng);
    for (int64_t x = c0 + threadIdx.x; x < c1; x += 256) {
        const float wv = a.w[x];
        float2 v[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) v[b] = A[(int64_t)b * a.ng + x];
        int p = 0;
#pragma unroll
        for (int b1 = 0; b1 < NB; ++b1) {
            const float2 u = make_float2(wv * v[b1].x, wv * v[b1].y);
#pragma unroll
            for (int b2 = b1; b2 < NB; ++b2, ++p) {
                acc[p] += u.x * v[b2].x + u.y * v[b2].y;
                if (IMAG) acc[NP + p] += u.y * v[b2].x - u.x * v[b2].y;
            }
        }
    }
    block_combine<NV>(acc, red, a.partial, g, blk, a.nblocks);
}

template <int NB>
hipError_t launch_pair_nb(const PairArgs &a, hipStream_t s) {
    dim3 grid(a.nblocks, a.ngroups, (unsigned)(a.fields > 1 ? a.fields : 1));
    if (a.want_imag) hipLaunchKernelGGL((pair_kernel<NB, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((pair_kernel<NB, false>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// ----------------------------------------------------------------- quad contraction
// Lanes of a wave own (b1, b2) pair slots p = lane + 64 s; the four waves take
// interleaved cells of the LDS tile.  Per cell and per m3 group of terms:
//   L = w(x) sum_terms C a^{b1}_{la,ma} a^{b2}_{lb,mb};   acc[b3] += Re(L a^{b3}_{lc,mc})
// (Im for odd Lambda: the m3 < 0 half is minus the conjugate of the m3 > 0 half there).
template <int NB, bool ODD>
__global__ __launch_bounds__(256) void quad_kernel(QuadArgs a) {
    a.coef += (int64_t)blockIdx.z * a.coef_fs;   // field of the launch (grid.z)
    a.w += (int64_t)blockIdx.z * a.w_fs;
    a.partial += (int64_t)blockIdx.z * a.part_fs;
    constexpr int NPAIR = NB * NB;
    constexpr int SLOTS = (NPAIR + 63) / 64;
    constexpr int NV = NB * NB * NB;
    extern __shared__ float2 tile[];       // [cell][staged column][bin]
    __shared__ int sl[3];                  // LDS column of (l, m = 0) for la, lb, lc
    __shared__ int scol[3 * (kMaxL + 1)];  // global lm index of every staged column
    __shared__ int s_nst;
    const int lam = blockIdx.y, blk = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int *so = a.stage + kStageStride * lam;
    if (threadIdx.x == 0) { sl[0] = so[0]; sl[1] = so[1]; sl[2] = so[2]; s_nst = so[3]; }
    if (threadIdx.x < 3 * (kMaxL + 1)) scol[threadIdx.x] = so[4 + threadIdx.x];
    __syncthreads();
    const int nst = s_nst;
    const int width = nst * NB;
    float acc[SLOTS][NB];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[s][b] = 0.f;
    const int t0 = a.term_ptr[lam], t1 = a.term_ptr[lam + 1];
    const int64_t c0 = (int64_t)blk * a.cells_per_block;
    const int64_t c1 = min(c0 + a.cells_per_block, a.ng);
    for (int64_t tc = c0; tc < c1; tc += a.tile) {
        const int ncell = (int)min((int64_t)a.tile, c1 - tc);
        __syncthreads();
        // stage: tile[c][k * NB + b] = coefficient of staged column k, bin b, cell tc + c
        for (int f = threadIdx.x; f < width * a.tile; f += 256) {
            const int c = f % a.tile, kb = f / a.tile;
            const int k = kb / NB, b = kb % NB;
            float2 v = make_float2(0.f, 0.f);
            const int lm = scol[k];
            const int arr = a.lm_src ? a.lm_src[2 * lm] : lm, part = a.lm_src ? a.lm_src[2 * lm + 1] : 0;
            if (c < ncell) v = a.coef[((int64_t)arr * NB + b) * a.ng + tc + c];
            if (part == 1) v.y = 0.f;                          // packed m = 0 arrays: one real column each
            else if (part == 2) v = make_float2(v.y, 0.f);
            tile[c * width + kb] = v;
        }
        __syncthreads();
        for (int c = wave; c < ncell; c += 4) {
            const float wv = a.w[tc + c];
            const float2 *tc_ = tile + c * width;
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const int p = lane + 64 * s;
                if (p >= NPAIR) break;
                const int b1 = p / NB, b2 = p % NB;
                int t = t0;
                while (t < t1) {
                    const int mc = a.terms[t].mc;
                    float2 L = make_float2(0.f, 0.f);
                    for (; t < t1 && a.terms[t].mc == mc; ++t) {
                        const QuadTerm q = a.terms[t];
                        const int ma = q.ma, mb = q.mb;
                        float2 x1 = tc_[(sl[0] + abs(ma)) * NB + b1];
                        if (ma < 0) { x1.y = -x1.y; if (ma & 1) { x1.x = -x1.x; x1.y = -x1.y; } }
                        float2 x2 = tc_[(sl[1] + abs(mb)) * NB + b2];
                        if (mb < 0) { x2.y = -x2.y; if (mb & 1) { x2.x = -x2.x; x2.y = -x2.y; } }
                        const float2 pr = cmul(x1, x2);
                        L.x += q.c * pr.x;
                        L.y += q.c * pr.y;
                    }
                    L.x *= wv; L.y *= wv;
                    const float2 *r3 = tc_ + (sl[2] + mc) * NB;
#pragma unroll
                    for (int b3 = 0; b3 < NB; ++b3)
                        acc[s][b3] += ODD ? L.x * r3[b3].y + L.y * r3[b3].x : L.x * r3[b3].x - L.y * r3[b3].y;
                }
            }
        }
    }
    __syncthreads();
    // float64 combine: each wave sums its lanes' slots into LDS, then across waves
    double *red = reinterpret_cast<double *>(tile);   // reuse: 4 * NV doubles
    for (int v = threadIdx.x; v < 4 * NV; v += 256) red[v] = 0.0;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int p = lane + 64 * s;
        if (p < NPAIR)
#pragma unroll
            for (int b3 = 0; b3 < NB; ++b3) red[wave * NV + p * NB + b3] = (double)acc[s][b3];
    }
    __syncthreads();
    for (int v = threadIdx.x; v < NV; v += 256) {
        const double sum = (red[v] + red[NV + v]) + (red[2 * NV + v] + red[3 * NV + v]);
        a.partial[((int64_t)lam * NV + v) * a.nblocks + blk] = sum;
    }
}

// ----------------------------------------------------------------- projected 4PCF
template <int NB>
__global__ __launch_bounds__(256) void proj4_kernel(Proj4Args a) {
    a.coef += (int64_t)blockIdx.z * a.coef_fs;   // field of the launch (grid.z)
    a.w += (int64_t)blockIdx.z * a.w_fs;
    a.partial += (int64_t)blockIdx.z * a.part_fs;
    constexpr int NPAIR = NB * NB;
    constexpr int SLOTS = (NPAIR + 63) / 64;
    constexpr int NV = NB * NB * NB * 2;
    extern __shared__ float2 tile[];      // [cell][3][bin]: c_{|m1|}, c_{|m2|}, c_{|m3|}
    const int pr_ = blockIdx.y, blk = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m1 = a.pairs[2 * pr_], m2 = a.pairs[2 * pr_ + 1], m3 = -(m1 + m2);
    const int ms[3] = {m1, m2, m3};
    constexpr int width = 3 * NB;
    float acc[SLOTS][NB][2];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s)
#pragma unroll
        for (int b = 0; b < NB; ++b) { acc[s][b][0] = 0.f; acc[s][b][1] = 0.f; }
    const int64_t c0 = (int64_t)blk * a.cells_per_block;
    const int64_t c1 = min(c0 + a.cells_per_block, a.ng);
    for (int64_t tc = c0; tc < c1; tc += a.tile) {
        const int ncell = (int)min((int64_t)a.tile, c1 - tc);
        __syncthreads();
        for (int f = threadIdx.x; f < width * a.tile; f += 256) {
            const int c = f % a.tile, kb = f / a.tile;
            const int k = kb / NB, b = kb % NB;
            const int m = ms[k];
            float2 v = make_float2(0.f, 0.f);
            if (c < ncell) {
                v = a.coef[((int64_t)abs(m) * NB + b) * a.ng + tc + c];
                if (m < 0) v.y = -v.y;   // c_{-m} = conj(c_m)
            }
            tile[c * width + kb] = v;
        }
        __syncthreads();
        for (int c = wave; c < ncell; c += 4) {
            const float wv = a.w[tc + c];
            const float2 *t = tile + c * width;
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const int p = lane + 64 * s;
                if (p >= NPAIR) break;
                const int b1 = p / NB, b2 = p % NB;
                float2 L = cmul(t[b1], t[NB + b2]);
                L.x *= wv; L.y *= wv;
#pragma unroll
                for (int b3 = 0; b3 < NB; ++b3) {
                    const float2 r = t[2 * NB + b3];
                    acc[s][b3][0] += L.x * r.x - L.y * r.y;
                    acc[s][b3][1] += L.x * r.y + L.y * r.x;
                }
            }
        }
    }
    __syncthreads();
    double *red = reinterpret_cast<double *>(tile);
    for (int v = threadIdx.x; v < 4 * NV; v += 256) red[v] = 0.0;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int p = lane + 64 * s;
        if (p < NPAIR)
#pragma unroll
            for (int b3 = 0; b3 < NB; ++b3) {
                red[wave * NV + (p * NB + b3) * 2] = (double)acc[s][b3][0];
                red[wave * NV + (p * NB + b3) * 2 + 1] = (double)acc[s][b3][1];
            }
    }
    __syncthreads();
    for (int v = threadIdx.x; v < NV; v += 256) {
        const double sum = (red[v] + red[NV + v]) + (red[2 * NV + v] + red[3 * NV + v]);
        a.partial[((int64_t)pr_ * NV + v) * a.nblocks + blk] = sum;
    }
}

// ----------------------------------------------------------------- reductions
__global__ __launch_bounds__(64) void block_sum_kernel(const double *partial, int nblocks, double *tot) {
    const int64_t gv = blockIdx.x;   // (group, value) flattened
    const double *p = partial + gv * nblocks;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 64) s += p[b];
    s = wave_sum(s);
    if (threadIdx.x == 0) tot[gv] = s;
}

__global__ void gather_kernel(const double *src, const int *ptr, const int *idx, const double *coef,
                              int nout, double *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nout) return;
    double s = 0.0;
    for (int t = ptr[i]; t < ptr[i + 1]; ++t) s += coef[t] * src[idx[t]];
    out[i] = s;
}

__global__ void to_f32_kernel(const void *in, int dtype, int64_t n, float *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = dtype == 1 ? (float)reinterpret_cast<const double *>(in)[i] : reinterpret_cast<const float *>(in)[i];
}

// ----------------------------------------------------------------- input checks
// count[0] += number of NaN / Inf values among n float32 (dtype 0) or float64 (dtype 1) values
__global__ void nonfinite_kernel(const void *in, int dtype, int64_t n, unsigned int *count) {
    unsigned int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const bool ok = dtype == 1 ? isfinite(reinterpret_cast<const double *>(in)[i])
                                   : isfinite(reinterpret_cast<const float *>(in)[i]);
        bad += ok ? 0u : 1u;
    }
    for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o, 64);
    if ((threadIdx.x & 63) == 0 && bad) atomicAdd(count, bad);
}

__global__ void fill_u32_kernel(unsigned int *x, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0u;
}

// ----------------------------------------------------------------- normalization (Sec. 2.5)
// Block partials of sum_x delta(x) in float64: block b sums cells [b * chunk, (b + 1) * chunk).
__global__ __launch_bounds__(256) void density_sum_kernel(const void *in, int dtype, int64_t n, int64_t chunk,
                                                          double *partial) {
    __shared__ double red[4];
    const int64_t c0 = (int64_t)blockIdx.x * chunk;
    const int64_t c1 = min(c0 + chunk, n);
    double s = 0.0;
    for (int64_t i = c0 + threadIdx.x; i < c1; i += 256)
        s += dtype == 1 ? reinterpret_cast<const double *>(in)[i] : (double)reinterpret_cast<const float *>(in)[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// One block: N_gal = sum (delta + 1) from the partials (fixed order), nbar = N_gal / N_g and
// norm[t] = N_gal prod_i nbar V_{b_i} for every bin tuple t of (npcf - 1) bins; then every value
// of the field's result (rows x tuples x parts) is divided by the norm of its tuple.
__global__ __launch_bounds__(256) void normalize_kernel(const double *partial, int nparts, int64_t ng, NormArgs a,
                                                         double *zeta, int64_t nvals, double *norm_out) {
    __shared__ double s_ngal;
    __shared__ double s_norm[kMaxBins * kMaxBins * kMaxBins];
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < nparts; ++i) s += partial[i];
        s_ngal = s + (double)ng;
    }
    __syncthreads();
    const double ngal = s_ngal, nbar = ngal / (double)ng;
    int ntup = 1;
    for (int k = 0; k < a.order; ++k) ntup *= a.nbins;
    for (int t = threadIdx.x; t < ntup; t += blockDim.x) {
        double v = ngal;
        int rem = t;
        for (int k = 0; k < a.order; ++k) {
            v *= nbar * a.vbin[rem % a.nbins];
            rem /= a.nbins;
        }
        s_norm[t] = v;
        if (norm_out) norm_out[t] = v;
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < nvals; i += blockDim.x) zeta[i] /= s_norm[(i / a.parts) % ntup];
}

}  // namespace

hipError_t launch_pair_contract(const PairArgs &a, hipStream_t s) {
    switch (a.nbins) {
#define SB_CASE(N) case N: return launch_pair_nb<N>(a, s);
        SB_CASE(1) SB_CASE(2) SB_CASE(3) SB_CASE(4) SB_CASE(5) SB_CASE(6) SB_CASE(7) SB_CASE(8)
        SB_CASE(9) SB_CASE(10) SB_CASE(11) SB_CASE(12) SB_CASE(13) SB_CASE(14) SB_CASE(15) SB_CASE(16)
#undef SB_CASE
        default: return hipErrorInvalidValue;
    }
}

template <int NB>
static hipError_t launch_quad_nb(const QuadArgs &a, hipStream_t s) {
    constexpr int NV = NB * NB * NB;
    const size_t tile_bytes = (size_t)a.tile * a.max_cols * NB * sizeof(float2);
    const size_t red_bytes = (size_t)4 * NV * sizeof(double);
    const size_t shm = tile_bytes > red_bytes ? tile_bytes : red_bytes;
    dim3 grid(a.nblocks, a.nlam, (unsigned)(a.fields > 1 ? a.fields : 1));
    if (a.odd)
        hipLaunchKernelGGL((quad_kernel<NB, true>), grid, dim3(256), shm, s, a);
    else
        hipLaunchKernelGGL((quad_kernel<NB, false>), grid, dim3(256), shm, s, a);
    return hipGetLastError();
}

hipError_t launch_quad_contract(const QuadArgs &a, hipStream_t s) {
    switch (a.nbins) {
#define SB_CASE(N) case N: return launch_quad_nb<N>(a, s);
        SB_CASE(1) SB_CASE(2) SB_CASE(3) SB_CASE(4) SB_CASE(5) SB_CASE(6) SB_CASE(7) SB_CASE(8)
        SB_CASE(9) SB_CASE(10)
#undef SB_CASE
        default: return hipErrorInvalidValue;
    }
}

template <int NB>
static hipError_t launch_proj4_nb(const Proj4Args &a, hipStream_t s) {
    constexpr int NV = NB * NB * NB * 2;
    size_t tile_bytes = (size_t)a.tile * 3 * NB * sizeof(float2);
    size_t red_bytes = (size_t)4 * NV * sizeof(double);
    size_t shm = tile_bytes > red_bytes ? tile_bytes : red_bytes;
    dim3 grid(a.nblocks, a.npairs, (unsigned)(a.fields > 1 ? a.fields : 1));
    hipLaunchKernelGGL((proj4_kernel<NB>), grid, dim3(256), shm, s, a);
    return hipGetLastError();
}

hipError_t launch_proj4_contract(const Proj4Args &a, hipStream_t s) {
    if (a.mfma) return launch_proj4_mfma(a, s);
    switch (a.nbins) {
#define SB_CASE(N) case N: return launch_proj4_nb<N>(a, s);
        SB_CASE(1) SB_CASE(2) SB_CASE(3) SB_CASE(4) SB_CASE(5) SB_CASE(6) SB_CASE(7) SB_CASE(8)
        SB_CASE(9) SB_CASE(10)
#undef SB_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_block_sum(const double *partial, int ngroups, int nblocks, int nvals, double *tot,
                            hipStream_t s) {
    const int64_t n = (int64_t)ngroups * nvals;
    hipLaunchKernelGGL(block_sum_kernel, dim3((unsigned)n), dim3(64), 0, s, partial, nblocks, tot);
    return hipGetLastError();
}

hipError_t launch_gather(const double *src, const int *ptr, const int *idx, const double *coef, int nout,
                         double *out, hipStream_t s) {
    hipLaunchKernelGGL(gather_kernel, dim3((nout + 255) / 256), dim3(256), 0, s, src, ptr, idx, coef, nout, out);
    return hipGetLastError();
}

hipError_t launch_to_f32(const void *in, int dtype, int64_t n, float *out, hipStream_t s) {
    hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, dtype, n, out);
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(const void *in, int dtype, int64_t n, unsigned int *count, hipStream_t s) {
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    if (blocks > 0) hipLaunchKernelGGL(nonfinite_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, dtype, n, count);
    return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned int *x, int n, hipStream_t s) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, x, n);
    return hipGetLastError();
}

hipError_t launch_normalize(const void *delta, int dtype, int64_t ng, const NormArgs &a, double *partial,
                            double *zeta, int64_t nvals, double *norm_out, hipStream_t s) {
    const int nparts = kNormParts;
    const int64_t chunk = (ng + nparts - 1) / nparts;
    hipLaunchKernelGGL(density_sum_kernel, dim3(nparts), dim3(256), 0, s, delta, dtype, ng, chunk, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(normalize_kernel, dim3(1), dim3(256), 0, s, partial, nparts, ng, a, zeta, nvals, norm_out);
    return hipGetLastError();
}

hipError_t launch_quad_mfma_part0(int la, int lb, int lc, const QuadMArgs &a, hipStream_t s);
hipError_t launch_quad_mfma_part1(int la, int lb, int lc, const QuadMArgs &a, hipStream_t s);
hipError_t launch_quad_mfma_part2(int la, int lb, int lc, const QuadMArgs &a, hipStream_t s);

bool quad_mfma_available(int la, int lb, int lc, int nbins) {
    return nbins <= 8 && la <= 4 && lb <= 4 && lc <= 4;
}

hipError_t launch_quad_mfma(int la, int lb, int lc, const QuadMArgs &a, hipStream_t s) {
    if (!quad_mfma_available(la, lb, lc, a.nbins)) return hipErrorInvalidValue;
    if (la <= 1) return launch_quad_mfma_part0(la, lb, lc, a, s);
    if (la <= 3) return launch_quad_mfma_part1(la, lb, lc, a, s);
    return launch_quad_mfma_part2(la, lb, lc, a, s);
}

}  // namespace sb
