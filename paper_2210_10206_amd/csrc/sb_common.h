// Shared device helpers and launch descriptors of the SARABANDE HIP library.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace sb {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// Streaming accesses of the passes over the kernel arrays (each element read or written once
// per pass): non-temporal hints keep them from displacing reused data in the caches.
typedef float f2nt __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld_stream(const float2 *p) {
    const f2nt v = __builtin_nontemporal_load(reinterpret_cast<const f2nt *>(p));
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void st_stream(float2 *p, float2 v) {
    __builtin_nontemporal_store(f2nt{v.x, v.y}, reinterpret_cast<f2nt *>(p));
}

// Element at a 32-bit byte offset from an array base (arrays under 4 GiB): with a uniform base
// the loads and stores take one offset register instead of a 64-bit address.
__device__ __forceinline__ const float2 *at_bytes(const float2 *base, uint32_t bytes) {
    return reinterpret_cast<const float2 *>(reinterpret_cast<const char *>(base) + bytes);
}
__device__ __forceinline__ float2 *at_bytes(float2 *base, uint32_t bytes) {
    return reinterpret_cast<float2 *>(reinterpret_cast<char *>(base) + bytes);
}

// ---------------------------------------------------------------- FFT passes
// One pass = 1D transforms of length n along one axis of a C-ordered array of
// `ng` complex cells.  The axis has element stride `stride` (product of the later
// extents); the pencils are g = 0 .. ng/n - 1 with base (g / stride) * n * stride + g % stride.
enum FftLoad : int {
    LOAD_C = 0,        // complex float2 from in
    LOAD_MUL = 1,      // in[idx] * in2[idx]           (spectral product)
    LOAD_R32 = 2,      // real float  from in (imaginary part 0)
    LOAD_R64 = 3       // real double from in
};
enum FftStore : int {
    STORE_C = 0,       // out[idx] = value
    STORE_MACC = 1     // out[idx] += value * mul[idx]   (spectral multiply-accumulate)
};

struct FftPass {
    int n;             // transform length
    int64_t stride;    // element stride of the axis
    int64_t ng;        // cells per array
    int sign;          // -1 forward, +1 inverse (unnormalised)
    int load;          // FftLoad
    int store;         // FftStore
    const void *in;    // input (batch stride in_bs elements)
    const float2 *in2; // multiplier for LOAD_MUL (batch stride in2_bs)
    float2 *out;       // output (batch stride out_bs)
    const float2 *mul; // multiplier for STORE_MACC (batch stride mul_bs)
    int64_t in_bs, in2_bs, out_bs, mul_bs;
    int batch;         // arrays transformed in one launch (grid.y)
    const float2 *tw;  // n roots of unity exp(-2 pi i j / n), float32 from float64
    int variant;       // launch-shape variant (autotuned)
};

// Launch one FFT pass; returns hipSuccess or the launch error (hipErrorInvalidValue when
// no kernel exists for the length).
hipError_t launch_fft_pass(const FftPass &p, hipStream_t s);
bool fft_supported(int n);
int fft_num_variants(int n);

// First inverse pass along axis 0 with the kernel spectra regenerated from their
// compact storage (transformed along the other axes, np planes along axis 0: stored
// plane p holds axis-0 index p for p <= r0 and n - (np - p) above; all n when np == n).
struct Axis0Args {
    int n;                // axis-0 length
    int64_t plane;        // product of the other extents (= axis-0 stride)
    int64_t ng;           // n * plane
    int np, r0;
    int mode;             // 0: correlation (writes out[k]), 1: adjoint (accumulates into out)
    const float2 *dhat;   // mode 0: density spectrum
    const float2 *kc;     // compact kernels [k][np][plane]
    float2 *out;          // mode 0: [k][ng]; mode 1: accumulator [ng]
    const float2 *vin;    // mode 1: [b][ng] arrays already transformed along the other axes
    int nb;               // kernels per group (mode 0: per grid.y; mode 1: in this launch)
    int groups;           // grid.y (mode 0: kernel groups; mode 1: 1)
    int kfirst;           // mode 1: index of the first kernel of this launch
    int accgroups;        // mode 1: kernel groups accumulated in turn (0: one), nb arrays of vin
                          // each; group i reads kernels kmap[i] * nb + b (with kmap) or
                          // kfirst + i * nb + b, and out += its sum after every group
    const int *kmap;      // optional: kernel group of grid row y (mode 0) or of accumulated
                          // group i (mode 1); kc is then the whole kernel store (mode 0 without
                          // it: grid row y reads group y of kc)
    const float2 *tw;
    int fields;           // mode 0: fields of one shape in the launch (grid.z; 0 counts as 1)
    int64_t dhat_fs, out_fs;   // mode 0: element strides between the fields' dhat and out
    // Half store (half = 1): only the planes c_0 = 0 .. r0 are kept (np = r0 + 1).  A kernel with
    // definite parity under r -> -r gives the planes c_0 < 0 from them: K(-c_0, k) = s K(c_0, -k)
    // for global kernel groups g below nflip (s = -1 where bit g of odd_lo, or bit g - 64 of
    // odd_hi, is set: odd l), and K(-c_0, k) = conj K(c_0, k) for the packed m = 0 pairs from
    // nflip on.  (Scalars, not an array: an array member keeps the kernel's argument copy in
    // scratch memory.)
    int half;
    int nflip;
    int kgroup0;          // global kernel group of group 0 of kc
    uint64_t odd_lo, odd_hi;
    int64_t n1, n2;       // in-plane extents (n2 = 1 on 2D grids): the cell of -k
};
hipError_t launch_axis0(const Axis0Args &a, hipStream_t s);

// Last inverse pass (contiguous axis) fused with the two-coefficient contraction.
struct LastArgs {
    int n;                // last-axis length
    int64_t ng;
    const float2 *in;     // [group][b][ng] arrays transformed along every other axis
    const float *w;       // density (float32)
    int nb;               // bins
    int groups;           // coefficient groups (grid.y)
    int rows;             // rows per tile (P = nb * rows pencils)
    int64_t rows_per_block;
    int nblocks;
    int want_imag;
    int packed;           // each array carries two real coefficient fields (real and imaginary
                          // part): their pair sums are kept apart (value = part * npairs + pair)
    double *partial;      // [row][block]; row = group * nvalues + value, value = b1 <= b2 pair
                          // (then imaginary parts or the second packed field)
    const int *rowmap;    // optional: 2 per grid row, the group row of part 0 and part 1
                          // (row = rowmap[2 y + part] * npairs + pair)
    int prec;             // 0: float32 MFMA pair sums, 1: split-BF16 MFMA pair sums
    const float2 *tw;
    int fields;           // fields of one shape in the launch (grid.z; 0 counts as 1)
    int64_t in_fs, w_fs, part_fs;   // strides between the fields' in, w and partial
};
hipError_t launch_last_contract(const LastArgs &a, hipStream_t s);
int fused_last_rows(int n, int nb);   // rows per tile the fused last pass uses (0: no kernel)

}  // namespace sb
