// Runtime services of the plan: per-launch timing, the launch-shape autotuner and
// HIP-graph replay of the forward pass.
#include "sb_plan.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <utility>
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

}  // extern "C"

namespace {

// Key of a plan's tuned choices in the autotuner's cache file: the device architecture and
// everything the timed launches depend on (dimensionality, correlation order, bins, lmax,
// precision, flags, outer bin edge and the distinct grid shapes).
std::string tune_key(const sb_plan *p) {
    hipDeviceProp_t prop{};
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s ndim=%d npcf=%d nbins=%d lmax=%d prec=%d flags=%u rmax=%.17g shapes=",
                  arch.c_str(), p->prob.ndim, p->prob.npcf, p->prob.nbins, p->prob.lmax, p->prob.precision,
                  p->prob.flags & ~(unsigned)SB_FLAG_CHECK_FINITE, p->edges[p->prob.nbins]);
    std::string key = buf;
    for (size_t g = 0; g < p->groups.size(); ++g) {
        if (g) key += ",";
        for (int d = 0; d < p->prob.ndim; ++d) key += (d ? "x" : "") + std::to_string(p->groups[g].n[d]);
    }
    return key;
}

// The cache is a JSON object with one entry per line:
//   "<key>": {"fft": [[n, axis, variant], ...], "contract_tile": cells},
// read_entries returns the (key, entry text) pairs of an existing file.
std::vector<std::pair<std::string, std::string>> read_entries(const char *path) {
    std::vector<std::pair<std::string, std::string>> out;
    std::FILE *f = std::fopen(path, "r");
    if (!f) return out;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
    std::fclose(f);
    size_t pos = 0;
    while (true) {
        const size_t q0 = text.find('"', pos);
        if (q0 == std::string::npos) break;
        const size_t q1 = text.find('"', q0 + 1);
        if (q1 == std::string::npos) break;
        const size_t b0 = text.find('{', q1);
        const size_t b1 = b0 == std::string::npos ? std::string::npos : text.find('}', b0);
        if (b1 == std::string::npos) break;
        out.emplace_back(text.substr(q0 + 1, q1 - q0 - 1), text.substr(b0, b1 - b0 + 1));
        pos = b1 + 1;
    }
    return out;
}

// Integers of an entry's "fft" list and its "contract_tile" value; false when malformed.
bool parse_entry(const std::string &e, std::vector<int> &fft, int *tile) {
    const size_t f0 = e.find("\"fft\""), t0 = e.find("\"contract_tile\"");
    if (f0 == std::string::npos || t0 == std::string::npos || t0 < f0) return false;
    fft.clear();
    const char *c = e.c_str() + f0 + 5, *stop = e.c_str() + t0;
    while (c < stop) {
        if (*c == '-' || (*c >= '0' && *c <= '9')) {
            char *endp = nullptr;
            fft.push_back((int)std::strtol(c, &endp, 10));
            c = endp;
        } else {
            ++c;
        }
    }
    if (fft.size() % 3 != 0) return false;
    const char *tc = e.c_str() + t0 + 15;
    while (*tc && !(*tc == '-' || (*tc >= '0' && *tc <= '9'))) ++tc;
    if (!*tc) return false;
    *tile = (int)std::strtol(tc, nullptr, 10);
    return true;
}

}  // namespace

extern "C" {

// Times every FFT variant of every (length, axis) of the plan's shapes on the coefficient
// scratch (a full-batch inverse pass, as in the forward) and keeps the fastest; the
// contraction tile is chosen among its candidates the same way, with the output written to
// the plan's scratch.  With a cache file, a stored entry for this plan's key is applied
// without timing, and new choices are added to the file.
sb_status sb_autotune(sb_plan *p, void *stream, const char *cache_path) {
    if (!p) return fail(SB_EINVAL, "null plan");
    if (!p->persist || !p->scratch) return fail(SB_EWORKSPACE, "workspace not bound");
    if (!p->prepared) return fail(SB_ESTATE, "sb_prepare has not run");
    p->kept = false;   // the timed passes run in the scratch the kept arrays live in
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::string key;
    std::vector<std::pair<std::string, std::string>> entries;
    if (cache_path && *cache_path) {
        key = tune_key(p);
        entries = read_entries(cache_path);
        for (const auto &kv : entries) {
            if (kv.first != key) continue;
            std::vector<int> fft;
            int tile = 0;
            if (!parse_entry(kv.second, fft, &tile)) return fail(SB_EINVAL, "malformed autotune cache entry");
            for (size_t i = 0; i < fft.size(); i += 3) {
                if (!fft_supported(fft[i]) || fft[i + 1] < 0 || fft[i + 1] >= p->prob.ndim || fft[i + 2] < 0 ||
                    fft[i + 2] >= fft_num_variants(fft[i]))
                    return fail(SB_EINVAL, "autotune cache entry names an unknown FFT variant");
                p->fft_var[{fft[i], fft[i + 1]}] = fft[i + 2];
            }
            int lo = 0, hi = 0;
            p->contract_tile_range(&lo, &hi);
            if (tile < lo || tile > hi || (tile & (tile - 1)) != 0)
                return fail(SB_EINVAL, "autotune cache entry has a contraction tile out of range");
            p->contract_tile() = tile;
            p->release_graph();
            return SB_OK;
        }
    }
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
                        p->timing = was_timing;
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
        double *zt = reinterpret_cast<double *>(p->scratch + p->off_zt);
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
                double *zo[1] = {zt};
                st = contract(p, p->groups[p->field_group[f0]], zo, 1, s);
                (void)hipEventRecord(b, s);
                (void)hipEventSynchronize(b);
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, a, b);
                if (rep > 0) tot += ms;
            }
            if (tot < best) { best = tot; bestc = c; }
        }
        p->contract_tile() = bestc;
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
    if (!key.empty()) {
        std::string entry = "{\"fft\": [";
        bool first = true;
        for (const auto &kv : p->fft_var) {
            entry += (first ? "[" : ", [") + std::to_string(kv.first.first) + ", " + std::to_string(kv.first.second) +
                     ", " + std::to_string(kv.second) + "]";
            first = false;
        }
        entry += "], \"contract_tile\": " + std::to_string(p->contract_tile()) + "}";
        bool found = false;
        for (auto &kv : entries)
            if (kv.first == key) { kv.second = entry; found = true; }
        if (!found) entries.emplace_back(key, entry);
        const std::string tmp = std::string(cache_path) + ".tmp";
        std::FILE *f = std::fopen(tmp.c_str(), "w");
        if (!f) return fail(SB_EINVAL, std::string("cannot write the autotune cache ") + tmp);
        std::fputs("{\n", f);
        for (size_t i = 0; i < entries.size(); ++i)
            std::fprintf(f, " \"%s\": %s%s\n", entries[i].first.c_str(), entries[i].second.c_str(),
                         i + 1 < entries.size() ? "," : "");
        std::fputs("}\n", f);
        const bool ok = std::fclose(f) == 0;
        if (!ok || std::rename(tmp.c_str(), cache_path) != 0)
            return fail(SB_EINVAL, std::string("cannot write the autotune cache ") + cache_path);
    }
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
    if (p->prob.flags & SB_FLAG_CHECK_FINITE)
        return fail(SB_ESTATE, "a plan with SB_FLAG_CHECK_FINITE waits for its stream and cannot be captured");
    p->kept = false;
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
    p->kept = false;   // set by the capture, which ran nothing
    const hipError_t e = hipGraphLaunch(p->graph_exec, s);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    if (p->keep) {   // the replay keeps the arrays of the captured fields, which are these
        p->kept = true;
        p->kept_delta.assign(delta, delta + p->batch);
    }
    return SB_OK;
}

}  // extern "C"
