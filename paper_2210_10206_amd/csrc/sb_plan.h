// Plan object behind the C ABI.
#pragma once

#include "sarabande_hip.h"
#include "sb_kgen.h"
#include "sb_tables.h"

#include <array>
#include <map>
#include <string>
#include <utility>
#include <vector>

namespace sb {

constexpr double kKernelCacheCap = 64.0 * 1024 * 1024 * 1024;   // bytes of kernel spectra kept at most
constexpr double kBatchBytes = 32.0 * 1024 * 1024 * 1024;       // kernel arrays of a field batch by default

enum Stage : int { STAGE_FFT = 0, STAGE_CONTRACT = 1, STAGE_OTHER = 2, STAGE_COUNT = 3 };

struct ShapeGroup {
    int64_t n[3] = {1, 1, 1};
    int64_t ng = 0;
    int64_t plane = 0;            // cells per axis-0 plane
    int np = 0, r0 = 0;           // stored axis-0 planes of the kernels, support radius along axis 0
    bool half = false;            // only the planes c_0 = 0 .. r0 stored (the others by parity)
    int rows = 0;                 // rows per tile of the fused last pass (0: not available)
    int64_t rows_per_block = 0;
    std::vector<int> fields;
    size_t khat_off = 0;          // byte offset of this shape's kernel spectra in the persistent buffer
    int64_t counts[kMaxBins] = {};
};

enum KernelId : int { K_FFT = 0, K_AXIS0 = 1, K_LAST = 2, K_PAIR = 3, K_QUAD = 4, K_PROJ4 = 5, K_ADJPREP = 6, K_QUAD_MFMA = 7 };

struct TimedLaunch {
    int stage, kernel;
    int fft_n, fft_sign, batch;
    double bytes, flops;
    hipEvent_t a, b;
};

}  // namespace sb

struct sb_plan {
    sb_problem prob{};
    std::vector<double> edges;
    int64_t thr[sb::kMaxBins + 1] = {};
    int batch = 0;
    std::vector<std::array<int64_t, 3>> shapes;
    std::vector<int> field_group;
    std::vector<sb::ShapeGroup> groups;
    int nlm = 0, nk = 0;
    // fused 3D 3PCF and full 4PCF: array groups of the forward path.  The first npack carry two real m = 0
    // kernels (l_a, l_b) as K_{l_a 0} + i K_{l_b 0}, stored as kernel groups nlm .. nlm + npack - 1;
    // the others are one (l, m) each.  kmap: kernel group of each array group; rowmap: the (l, m)
    // group of part 0 and part 1 of its pair sums (-1: none).
    int npack = 0, nag = 0;
    int pack_l[2 * sb::kMaxPack] = {};
    std::vector<int> ag_kmap, ag_rowmap;
    std::vector<int> lm_src;       // 2 per (l, m): array group and part (0 complex, 1 / 2 re / im of a pair)
    const int *d_kmap = nullptr, *d_rowmap = nullptr, *d_lmsrc = nullptr;
    int kernel_groups() const { return nlm + npack; }
    int64_t max_ng = 0;
    int64_t last_ng = 0;
    // result layout
    int64_t zeta_doubles = 0;
    int32_t idx_rows = 0, idx_cols = 0;
    std::vector<int32_t> idx_table;
    sb::Full4Plan f4;
    std::vector<std::pair<int, int>> p4_pairs, p4_canon;
    std::map<std::pair<int, int>, int> p4_canon_index;
    // device tables: built on the host at creation, copied into the head of the caller's
    // persistent buffer by sb_prepare (tab_bytes bytes; the kernel spectra follow)
    std::vector<char> host_tab;
    size_t tab_bytes = 0;
    std::map<int, size_t> tw_off;
    size_t off_terms = 0, off_tptr = 0, off_laml = 0, off_stage = 0, off_pairs = 0, off_coefw = 0;
    size_t off_kmap = 0, off_rowmap = 0, off_lmsrc = 0, off_gptr = 0, off_gidx = 0, off_gcoef = 0;
    std::map<int, const float2 *> tw;
    const sb::QuadTerm *d_terms = nullptr;
    const int *d_term_ptr = nullptr, *d_lam_l = nullptr, *d_stage = nullptr, *d_pairs = nullptr;
    const int *d_gptr = nullptr, *d_gidx = nullptr;
    const double *d_gcoef = nullptr;
    int gather_nout = 0;
    int max_cols = 0;
    // workspace (caller-owned)
    char *persist = nullptr, *scratch = nullptr;
    size_t persist_need = 0, scratch_need = 0;
    size_t off_w = 0, off_dhat = 0, off_coef = 0, off_part = 0, off_tot = 0, off_grad = 0;
    size_t off_vtmp = 0, off_dsum = 0, off_gtab = 0;
    size_t off_flag = 0;          // 256 B: the non-finite counter of SB_FLAG_CHECK_FINITE
    size_t off_zt = 0;            // one field's result: the autotuner's output buffer
    uint32_t warnings = 0;        // SB_WARN_* bits
    // kernel spectra regenerated per chunk of kernel groups on every call (no cache in the
    // persistent buffer); their stored planes then sit in scratch at off_kc
    bool regen = false;
    size_t off_kc = 0;
    // half kernel store (ShapeGroup::half on the shapes it applies to): on request, when the
    // full store would pass kKernelCacheCap, and with regeneration
    bool half = false;
    // SB_FLAG_KEEP_FOR_ADJOINT: each field's coefficient arrays (the middle pass's output) at
    // off_coef + keep_off[f], the fields of a shape in its order (so every field batch of the
    // forward sits at its own stride); the backward's v arrays at off_vkeep.  kept: the arrays
    // hold the last forward's fields kept_delta and no backward has consumed them yet.
    bool keep = false;
    std::vector<size_t> keep_off;
    size_t off_vkeep = 0;
    bool kept = false;
    std::vector<const void *> kept_delta;
    // kernel groups ((l, m) multiplets) whose arrays share the scratch at once: all of them,
    // unless a 3PCF plan's full set would exceed coef_limit (then the passes run in chunks)
    uint64_t coef_limit = 48ull << 30;
    int chunk_groups = 0;
    // fields of one shape run through the passes together, up to fbatch at a time (one launch
    // per pass for all of them): as many as kBatchBytes of kernel arrays allow, at most
    // fbatch_req when the caller set it (sb_plan_set_field_batch), 1 when the passes run in chunks
    int fbatch = 1, fbatch_req = 0;
    bool prepared = false;
    // launch shapes (autotuned): cells per workgroup of the cell-parallel contractions (unfused
    // 3PCF pair sums, full 4PCF, projected 4PCF); the scratch holds the partial sums of the
    // smallest candidate of contract_tile_range
    int cpb_pair = 8192, cpb_quad = 1024, cpb_proj4 = 4096;
    int &contract_tile() { return prob.npcf == 3 ? cpb_pair : (prob.ndim == 3 ? cpb_quad : cpb_proj4); }
    int contract_tile() const { return prob.npcf == 3 ? cpb_pair : (prob.ndim == 3 ? cpb_quad : cpb_proj4); }
    void contract_tile_range(int *lo, int *hi) const {
        if (prob.npcf == 3) { *lo = 2048; *hi = 16384; }
        else if (prob.ndim == 3) { *lo = 512; *hi = 4096; }
        else { *lo = 1024; *hi = 8192; }
    }
    // a forward call runs the cell-parallel contraction on some field
    bool uses_contract() const {
        if (prob.npcf == 4 || !fused) return true;
        for (const auto &G : groups)
            if (G.rows <= 0) return true;
        return false;
    }
    const float *d_coefw = nullptr;   // weighted 3j values, every term, per canonical Lambda
    std::vector<int> coefw_off;
    bool quad_mfma = false;       // full 4PCF contraction on the matrix cores (l <= 4, <= 8 bins)
    bool fused = true;            // fused last pass + contraction for the 3PCFs (flag SB_FLAG_UNFUSED clears it)
    bool adj_fused = true;        // adjoint: last pass fused with the adjoint weights (SB_FLAG_UNFUSED clears it)
    int quad_tile = 32, proj4_tile = 64;
    std::map<std::pair<int, int>, int> fft_var;   // (length, axis) -> variant
    // untuned default: variant 0, except the register-resident 16-pencil pass along a strided axis
    // of length 1024 (about 3x the LDS-staged pass there, where autotuning takes long)
    int fft_variant(int n, int axis) const {
        auto it = fft_var.find({n, axis});
        if (it != fft_var.end()) return it->second;
        return n == 1024 && axis < prob.ndim - 1 ? 6 : 0;
    }
    // per-launch timing
    bool timing = false;
    std::vector<sb::TimedLaunch> timed;
    template <class F>
    hipError_t timed_launch(int stage, int kernel, hipStream_t s, F &&fn, int fft_n = 0, int fft_sign = 0,
                            int batch = 0, double bytes = 0.0, double flops = 0.0) {
        if (!timing) return fn();
        sb::TimedLaunch t{stage, kernel, fft_n, fft_sign, batch, bytes, flops, nullptr, nullptr};
        if (hipEventCreate(&t.a) != hipSuccess || hipEventCreate(&t.b) != hipSuccess) return fn();
        (void)hipEventRecord(t.a, s);
        const hipError_t e = fn();
        (void)hipEventRecord(t.b, s);
        timed.push_back(t);
        return e;
    }
    void release_timing() {
        for (auto &t : timed) {
            (void)hipEventDestroy(t.a);
            (void)hipEventDestroy(t.b);
        }
        timed.clear();
    }
    // graph replay cache
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<const void *> graph_delta;
    double *graph_zeta = nullptr;
    hipStream_t graph_stream = nullptr;
    void release_graph() {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        graph_exec = nullptr;
        graph = nullptr;
        graph_delta.clear();
        graph_zeta = nullptr;
    }
};

namespace sb {
sb_status fail(sb_status s, const std::string &msg);
sb_status hip_fail(hipError_t e, const char *what);
sb_status forward(sb_plan *p, const void *const *delta, double *zeta, hipStream_t s);
sb_status density_spectrum(sb_plan *p, const sb::ShapeGroup &G, const void *delta, hipStream_t s);
// Coefficients of kernel groups [g0, g0 + ng) of field f into scratch (group g0 first); the
// density spectrum must be in scratch already.  last_axis = false stops before the inverse
// transform along the last axis.  kmap (device, optional): the kernel group of each of the ng
// output groups (array groups of a packed plan) instead of g0 .. g0 + ng - 1.
sb_status coefficients(sb_plan *p, int f, int g0, int ngroups, hipStream_t s, bool last_axis = true,
                       const int *kmap = nullptr, int nf = 1);
void layout_scratch(sb_plan *p);
sb_status contract(sb_plan *p, const ShapeGroup &G, double *const *zout, int nf, hipStream_t s);
// Half kernel store (plan.hip): whether a shape keeps only the planes c_0 = 0 .. r0, the planes
// stored per kernel, and the half-store fields of an axis-0 launch.
bool half_store(const ShapeGroup &G, int ndim, int64_t r0, bool want);
int stored_planes(const ShapeGroup &G, int ndim, int64_t r0, bool want);
void mirror_args(const sb_plan *p, const ShapeGroup &G, int kgroup0, Axis0Args &a);
// SB_FLAG_CHECK_FINITE: count the NaN / Inf values of the inputs (n[i] values of dtype[i] at in[i]),
// wait for the stream and return SB_ENONFINITE when there are any; SB_OK otherwise (and at once
// when the flag is clear).
sb_status check_finite(sb_plan *p, int count, const void *const *in, const int64_t *n, const int *dtype,
                       hipStream_t s);
// FFT passes over the listed axes (in order) of arrays with extents n[0..ndim) and ncell
// cells; the first pass reads `in` with load mode `first_load`, later passes work in place
// on `out`; the last pass stores with `store` into final_out (or out).
sb_status fft_axes(sb_plan *p, const int64_t *n, int ndim, int64_t ncell, const int *axes, int naxes, int sign,
                   int first_load, const void *in, int64_t in_bs, float2 *out, int64_t out_bs, int batch,
                   hipStream_t s, int store = STORE_C, const float2 *mul = nullptr, int64_t mul_bs = 0,
                   float2 *final_out = nullptr);
sb_status fft_all_axes(sb_plan *p, const ShapeGroup &G, int sign, int first_load, const void *in, int64_t in_bs,
                       float2 *out, int64_t out_bs, int batch, hipStream_t s);
}  // namespace sb
