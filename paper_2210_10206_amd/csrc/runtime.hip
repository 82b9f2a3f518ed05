// Runtime services of the plan: per-launch timing, the launch-shape autotuner and
// HIP-graph replay of the forward pass.
#include "sb_plan.h"

#include <algorithm>
#include <vector>

using namespace sb;

extern "C" {

sb_status sb_profile(sb_plan *p, int32_t enable) {
    if (!p) return fail(SB_EINVAL, "null plan");
    p->release_timing();
    p->timing = enable != 0;
    return SB_OK;
}

sb_status sb_profile_read(sb_plan *p, int32_t max, int32_t *count, sb_launch_record *out) {
    if (!p || !count || (max > 0 && !out)) return fail(SB_EINVAL, "null argument");
    *count = (int32_t)p->timed.size();
    for (int32_t i = 0; i < max && i < (int32_t)p->timed.size(); ++i) {
        const auto &t = p->timed[i];
        hipError_t e = hipEventSynchronize(t.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float x = 0.f;
        e = hipEventElapsedTime(&x, t.a, t.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        out[i].stage = t.stage;
        out[i].kernel = t.kernel;
        out[i].fft_n = t.fft_n;
        out[i].fft_sign = t.fft_sign;
        out[i].batch = t.batch;
        out[i].bytes = t.bytes;
        out[i].flops = t.flops;
        out[i].ms = x;
    }
    return SB_OK;
}

sb_status sb_stage_times(sb_plan *p, double *fft_ms, int32_t *n_fft, double *contract_ms, int32_t *n_contract) {
    if (!p || !fft_ms || !n_fft || !contract_ms || !n_contract) return fail(SB_EINVAL, "null argument");
    double ms[STAGE_COUNT] = {0, 0, 0};
    int cnt[STAGE_COUNT] = {0, 0, 0};
    for (auto &t : p->timed) {
        hipError_t e = hipEventSynchronize(t.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float x = 0.f;
        e = hipEventElapsedTime(&x, t.a, t.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        ms[t.stage] += x;
        cnt[t.stage] += 1;
    }
    *fft_ms = ms[STAGE_FFT];
    *n_fft = cnt[STAGE_FFT];
    *contract_ms = ms[STAGE_CONTRACT];
    *n_contract = cnt[STAGE_CONTRACT];
    return SB_OK;
}

// Times every FFT variant of every (length, axis) of the plan's shapes on the
// coefficient scratch (a full-batch inverse pass, as in the forward) and keeps the
// fastest.  Contraction block sizes are chosen among a few candidates the same way.
sb_status sb_autotune(sb_plan *p, void *stream) {
    if (!p) return fail(SB_EINVAL, "null plan");
    if (!p->persist || !p->scratch) return fail(SB_EWORKSPACE, "workspace not bound");
    if (!p->prepared) return fail(SB_ESTATE, "sb_prepare has not run");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return fail(SB_EHIP, "event create");
    float2 *coef = reinterpret_cast<float2 *>(p->scratch + p->off_coef);
    const bool was_timing = p->timing;
    p->timing = false;
    for (const auto &G : p->groups) {
        for (int d = 0; d < p->prob.ndim; ++d) {
            const int n = (int)G.n[d];
            const int nv = fft_num_variants(n);
            int64_t stride = 1;
            for (int k = d + 1; k < p->prob.ndim; ++k) stride *= G.n[k];
            float best = 1e30f;
            int bestv = 0;
            for (int v = 0; v < nv; ++v) {
                FftPass ps{};
                ps.n = n;
                ps.stride = stride;
                ps.ng = G.ng;
                ps.sign = 1;
                ps.load = LOAD_C;
                ps.store = STORE_C;
                ps.in = coef;
                ps.out = coef;
                ps.in_bs = ps.out_bs = G.ng;
                // the arrays a forward pass transforms at once (fewer with packed m = 0 pairs)
                ps.batch = (p->npack > 0 ? std::min(p->chunk_groups, p->nag) : p->chunk_groups) * p->prob.nbins;
                ps.tw = p->tw.at(n);
                ps.variant = v;
                float tot = 0.f;
                for (int rep = 0; rep < 3; ++rep) {
                    (void)hipEventRecord(a, s);
                    hipError_t e = launch_fft_pass(ps, s);
                    (void)hipEventRecord(b, s);
                    if (e != hipSuccess) {
                        (void)hipEventDestroy(a);
                        (void)hipEventDestroy(b);
                        return hip_fail(e, "autotune fft");
                    }
                    (void)hipEventSynchronize(b);
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, a, b);
                    if (rep > 0) tot += ms;
                }
                if (tot < best) { best = tot; bestv = v; }
            }
            p->fft_var[{n, d}] = bestv;
        }
    }
    // contraction tile: every candidate on the first field of the largest shape; the kernels
    // read whatever the coefficient scratch holds (timing only; a forward call recomputes it)
    if (p->uses_contract() && p->chunk_groups == p->nlm) {
        int f0 = 0;
        for (int f = 0; f < p->batch; ++f)
            if (p->groups[p->field_group[f]].ng > p->groups[p->field_group[f0]].ng) f0 = f;
        double *zt = nullptr;
        if (hipMalloc(&zt, (size_t)p->zeta_doubles * sizeof(double)) != hipSuccess) {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            p->timing = was_timing;
            return fail(SB_EHIP, "autotune buffer");
        }
        int lo = 0, hi = 0;
        p->contract_tile_range(&lo, &hi);
        float best = 1e30f;
        int bestc = p->contract_tile();
        sb_status st = SB_OK;
        for (int c = lo; c <= hi && st == SB_OK; c *= 2) {
            p->contract_tile() = c;
            float tot = 0.f;
            for (int rep = 0; rep < 3 && st == SB_OK; ++rep) {
                (void)hipEventRecord(a, s);
                st = contract(p, f0, zt, s);
                (void)hipEventRecord(b, s);
                (void)hipEventSynchronize(b);
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, a, b);
                if (rep > 0) tot += ms;
            }
            if (tot < best) { best = tot; bestc = c; }
        }
        p->contract_tile() = bestc;
        (void)hipFree(zt);
        if (st != SB_OK) {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            p->timing = was_timing;
            return st;
        }
    }
    p->timing = was_timing;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    p->release_graph();
    return SB_OK;
}

int32_t sb_fft_variants(int32_t n) { return fft_supported(n) ? fft_num_variants(n) : 0; }

sb_status sb_plan_set_fft_variant(sb_plan *p, int32_t n, int32_t axis, int32_t variant) {
    if (!p) return fail(SB_EINVAL, "null plan");
    if (!fft_supported(n)) return fail(SB_EINVAL, "unsupported length");
    if (axis < 0 || axis >= p->prob.ndim) return fail(SB_EINVAL, "axis out of range");
    if (variant < 0 || variant >= fft_num_variants(n)) return fail(SB_EINVAL, "variant out of range");
    p->fft_var[{n, axis}] = variant;
    p->release_graph();
    return SB_OK;
}

sb_status sb_plan_get_fft_variant(const sb_plan *p, int32_t n, int32_t axis, int32_t *variant) {
    if (!p || !variant) return fail(SB_EINVAL, "null argument");
    if (!fft_supported(n)) return fail(SB_EINVAL, "unsupported length");
    if (axis < 0 || axis >= p->prob.ndim) return fail(SB_EINVAL, "axis out of range");
    *variant = p->fft_variant(n, axis);
    return SB_OK;
}

sb_status sb_plan_set_contract_tile(sb_plan *p, int32_t cells) {
    if (!p) return fail(SB_EINVAL, "null plan");
    int lo = 0, hi = 0;
    p->contract_tile_range(&lo, &hi);
    if (cells < lo || cells > hi || (cells & (cells - 1)) != 0)
        return fail(SB_EINVAL, "contraction tile must be a power of two within the plan's range");
    p->contract_tile() = cells;
    p->release_graph();
    return SB_OK;
}

sb_status sb_plan_get_contract_tile(const sb_plan *p, int32_t *cells, int32_t *lo, int32_t *hi) {
    if (!p || !cells) return fail(SB_EINVAL, "null argument");
    int l = 0, h = 0;
    p->contract_tile_range(&l, &h);
    *cells = p->contract_tile();
    if (lo) *lo = l;
    if (hi) *hi = h;
    return SB_OK;
}

sb_status sb_forward_graph(sb_plan *p, const void *const *delta, double *zeta, void *stream) {
    if (!p || !delta || !zeta) return fail(SB_EINVAL, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!s) return fail(SB_EINVAL, "graph replay needs a non-default stream");
    if (p->timing) return fail(SB_ESTATE, "disable per-launch timing before graph replay");
    bool same = p->graph_exec && p->graph_zeta == zeta && p->graph_stream == s &&
                (int)p->graph_delta.size() == p->batch;
    for (int f = 0; same && f < p->batch; ++f) same = p->graph_delta[f] == delta[f];
    if (!same) {
        p->release_graph();
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        const sb_status st = forward(p, delta, zeta, s);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(s, &g);
        if (st != SB_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_fail(e, "hipGraphInstantiate");
        }
        p->graph = g;
        p->graph_delta.assign(delta, delta + p->batch);
        p->graph_zeta = zeta;
        p->graph_stream = s;
    }
    const hipError_t e = hipGraphLaunch(p->graph_exec, s);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return SB_OK;
}

}  // extern "C"
