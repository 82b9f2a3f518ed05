"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerance (floating point): max |Z_gpu - Z_oracle| / max |Z_oracle| <= 1e-5 for the float32
path and <= 3e-4 for split-BF16, over the whole result and over every block of its leading
index (per l, Lambda, m or (m1, m2)), each block relative to its own max |Z_oracle|
(tests/parity.py).  Gradients: max |g_gpu - g_oracle| / max |g_oracle| <= 1e-5.  Integer work
(bin counts) is compared exactly.
"""
import math
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from fieldgen import lognormal_field, linear_edges  # noqa: E402
from parity import TOL32, TOL_SPLIT, check, rel_err  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_10206_amd as pkg
    pkg.load()  # fails loudly when the HIP library is missing
    from paper_2210_10206_amd import api
    return api


def run_plan(api, fields, edges, lmax, npcf=3, dtype=torch.float32, graph=False, precision="fp32", **kw):
    shapes = [f.shape for f in fields]
    plan = api.Plan(shapes, edges, lmax, npcf=npcf, input_dtype=dtype, precision=precision, **kw)
    dev = [torch.from_numpy(np.ascontiguousarray(f)).to(device="cuda", dtype=dtype) for f in fields]
    if graph:
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            z = plan.forward(dev, stream=s, graph=True)
        s.synchronize()
    else:
        z = plan.forward(dev)
    torch.cuda.synchronize()
    return plan, dev, z.cpu().numpy()


# ------------------------------------------------------------------ 32^3 full 3PCF (float64 input)

def test_c1_full3pcf_32(sb):
    say("case: 32^3 float64 lognormal seed 0, 4 bins to 8, lmax 4, full 3PCF")
    d = lognormal_field((32, 32, 32), seed=0, sigma=1.0, dtype=np.float64)
    edges = linear_edges(8, 4)
    plan, dev, z = run_plan(sb, [d], edges, 4, dtype=torch.float64)
    ref = oracle.zeta3_full(d, edges, 4)
    assert np.max(np.abs(ref.imag)) < 1e-9 * np.max(np.abs(ref.real))
    check(z[0], ref.real, TOL32, say)
    assert list(plan.bin_counts(0)) == list(oracle.bin_counts((32, 32, 32), edges))
    plan.close()


def test_degenerate_cases(sb):
    # one bin and lmax 0 (a single kernel array; the 3PCF reduces to sum_x delta a^2), the
    # smallest supported grid, mmax 0 projected, an all-zero field and a single-cell spike (every
    # sum is exactly zero: r = 0 lies in no bin, so a^b(y) vanishes at the spike)
    say("case: degenerate inputs: 1 bin / lmax 0 at 16^3, 8^3 full 3PCF and 4PCF, 32x48 mmax 0, zero field, spike")
    d = lognormal_field((16, 16, 16), seed=31, sigma=1.0)
    e1 = linear_edges(4, 1)
    _, _, z = run_plan(sb, [d], e1, 0)
    ref = oracle.zeta3_full(d.astype(np.float64), e1, 0).real
    assert z.shape == (1, 1, 1, 1)
    check(z[0], ref, TOL32, say, "1 bin lmax 0: ")
    d8 = lognormal_field((8, 8, 8), seed=32, sigma=1.0)
    e8 = linear_edges(3, 2)
    _, _, z8 = run_plan(sb, [d8], e8, 2)
    check(z8[0], oracle.zeta3_full(d8.astype(np.float64), e8, 2).real, TOL32, say, "8^3 3PCF: ")
    _, _, z84 = run_plan(sb, [d8], e8, 2, npcf=4)
    _, ref84 = oracle.zeta4_full(d8.astype(np.float64), e8, 2)
    check(z84[0], ref84.real, TOL32, say, "8^3 4PCF: ")
    dp = lognormal_field((32, 48), seed=33, sigma=1.0)
    ep = linear_edges(6, 3)
    _, _, zp = run_plan(sb, [dp], ep, 0)
    check(zp[0], oracle.zeta3_proj(dp.astype(np.float64), ep, 0), TOL32, say, "mmax 0 projected: ")
    zero = np.zeros((24, 24, 24), np.float32)
    spike = zero.copy()
    spike[5, 7, 11] = 3.0
    e = linear_edges(8, 4)
    for npcf in (3, 4):
        plan, _, zz = run_plan(sb, [zero], e, 4, npcf=npcf)
        assert np.all(zz == 0.0), f"npcf {npcf}: nonzero sums for the zero field"
        # spike: exact sums vanish; the float32 transforms leave rounding noise in a^b(y), so the
        # bound is 1e-5 of the size the sums would have with |a| at its largest (3 x bin count)
        nmax = float(max(plan.bin_counts(0)))
        plan, _, zz = run_plan(sb, [spike], e, 4, npcf=npcf)
        bound = 1e-5 * 3.0 * (3.0 * nmax) ** (npcf - 1)
        say(f"  spike npcf {npcf}: max |Z| = {np.max(np.abs(zz)):.3e} (bound {bound:.3e})")
        assert np.max(np.abs(zz)) <= bound


def test_c1_coefficients_match_oracle(sb):
    say("case: 32^3 coefficients a^b_lm at sampled cells")
    d = lognormal_field((32, 32, 32), seed=0, sigma=1.0, dtype=np.float64)
    edges = linear_edges(8, 4)
    plan, dev, z = run_plan(sb, [d], edges, 4, dtype=torch.float64, keep_coeffs=True)
    rng = np.random.Generator(np.random.PCG64(7))
    cells = rng.choice(d.size, 64, replace=False)
    ref = oracle.coeffs_full(d, edges, 4, cells=cells)   # (ncell, nb, (lmax+1)^2)
    worst = 0.0
    for l in range(5):
        for m in range(l + 1):
            lm = l * (l + 1) // 2 + m
            for b in range(4):
                a = plan.coeffs(lm * 4 + b).reshape(-1).cpu().numpy()[cells]
                r = ref[:, b, l * l + m + l]
                scale = np.max(np.abs(ref[:, b, :]))
                worst = max(worst, float(np.max(np.abs(a - r)) / scale))
    say(f"  coefficient err (rel. to max |a| per bin) = {worst:.3e}")
    assert worst < 2e-6
    plan.close()


def test_unfused_path_matches_oracle(sb):
    say("case: 32^3 unfused path (coefficients written, separate contraction), 4 bins to 8, lmax 4")
    d = lognormal_field((32, 32, 32), seed=0, sigma=1.0)
    edges = linear_edges(8, 4)
    plan, dev, z = run_plan(sb, [d], edges, 4, fused=False)
    ref = oracle.zeta3_full(d.astype(np.float64), edges, 4)
    check(z[0], ref.real, TOL32, say)
    plan.close()


def test_ragged_noncubic_grid_with_ties(sb):
    say("case: (12, 16, 24) normal field, edges (0, 1.5, 2, 3.2, 5), lmax 3")
    rng = np.random.Generator(np.random.PCG64(11))
    d = rng.standard_normal((12, 16, 24)).astype(np.float32)
    edges = np.array([0.0, 1.5, 2.0, 3.2, 5.0])
    plan, dev, z = run_plan(sb, [d], edges, 3)
    ref = oracle.zeta3_full(d.astype(np.float64), edges, 3)
    check(z[0], ref.real, TOL32, say)
    assert list(plan.bin_counts(0)) == list(oracle.bin_counts(d.shape, edges))
    plan.close()


def test_box_truncated_kernel_24(sb):
    say("case: 24^3, 8 bins to 16 (kernel reaches the box edge), lmax 4")
    d = lognormal_field((24, 24, 24), seed=3, sigma=1.0)
    edges = linear_edges(16, 8)
    plan, dev, z = run_plan(sb, [d], edges, 4)
    assert plan.warnings() & 1, "the kernel reaches the box edge: the truncation bit must be set"
    ref = oracle.zeta3_full(d.astype(np.float64), edges, 4)
    check(z[0], ref.real, TOL32, say)
    plan.close()


def test_uneven_batch(sb):
    say("case: uneven batch 16^3, 24^3, 32^3, 8 bins to 6, lmax 4")
    fields = [lognormal_field((n, n, n), seed=i, sigma=1.0) for i, n in enumerate((16, 24, 32))]
    edges = linear_edges(6, 8)
    plan, dev, z = run_plan(sb, fields, edges, 4)
    for i, f in enumerate(fields):
        ref = oracle.zeta3_full(f.astype(np.float64), edges, 4)
        check(z[i], ref.real, TOL32, say, f"field {i} {f.shape}: ")
    plan.close()


def test_chunked_kernel_groups_match_whole(sb):
    # a scratch limit of three (l, m) groups makes the fused 3PCF and the adjoint run their
    # passes over chunks (3, 3, 3, 3, 3) of the 15 groups; results match the one-chunk plan
    say("case: 32^3, 8 bins to 6, lmax 4: chunks of 3 kernel groups vs all at once (forward + adjoint)")
    d = lognormal_field((32, 32, 32), seed=7, sigma=1.0)
    edges = linear_edges(6, 8)
    dev = [torch.from_numpy(d).cuda()]
    whole = sb.Plan([d.shape], edges, 4)
    per_group = 8 * d.size * 8
    chunked = sb.Plan([d.shape], edges, 4, scratch_limit=3 * per_group)
    assert chunked.scratch_bytes < whole.scratch_bytes
    z1 = whole.forward(dev).cpu().numpy()
    z2 = chunked.forward(dev).cpu().numpy()
    G = torch.from_numpy(np.random.Generator(np.random.PCG64(4)).standard_normal((1, 5, 8, 8))).cuda()
    g1 = whole.backward(dev, G)[0].cpu().numpy()
    g2 = chunked.backward(dev, G)[0].cpu().numpy()
    torch.cuda.synchronize()
    ref = oracle.zeta3_full(d.astype(np.float64), edges, 4).real
    say(f"  chunked vs oracle err={rel_err(z2[0], ref):.3e}; chunked vs whole max diff "
        f"{np.max(np.abs(z2 - z1)):.3e}, grad {np.max(np.abs(g2 - g1)):.3e}")
    assert np.array_equal(z1, z2)
    assert np.array_equal(g1, g2)
    check(z2[0], ref, TOL32, say)
    whole.close()
    chunked.close()


@pytest.mark.parametrize("shape,nbins,lmax", [((32, 32, 32), 4, 1), ((8, 16, 256), 10, 6), ((8, 16, 256), 3, 5),
                                              ((12, 8, 96), 8, 4), ((16, 16, 64), 16, 2)])
def test_packed_m0_arrays(sb, shape, nbins, lmax):
    # the default fused 3D 3PCF carries the real m = 0 coefficient fields two to a transform;
    # every last-pass family (LDS-staged, register-resident 256, radix-list 96) against the
    # oracle and against the plan with one transform per (l, m)
    say(f"case: {shape} full 3PCF, {nbins} bins to 8, lmax {lmax}: packed m = 0 pairs vs one per (l, m)")
    d = lognormal_field(shape, seed=50 + lmax, sigma=1.0)
    edges = linear_edges(8, nbins)
    plan, dev, z = run_plan(sb, [d], edges, lmax)
    plan0, _, z0 = run_plan(sb, [d], edges, lmax, pack=False)
    assert plan.persistent_bytes > plan0.persistent_bytes   # the packed kernels are stored besides
    ref = oracle.zeta3_full(d.astype(np.float64), edges, lmax).real
    check(z[0], ref, TOL32, say, "packed: ")
    check(z0[0], ref, TOL32, say, "unpacked: ")
    say(f"  packed vs unpacked {rel_err(z[0], z0[0]):.3e}")
    # the adjoint runs the same array groups: its gradient against the one-per-(l, m) adjoint
    G = torch.from_numpy(np.random.Generator(np.random.PCG64(60 + lmax)).standard_normal(
        (1, lmax + 1, nbins, nbins))).cuda()
    g1 = plan.backward(dev, G)[0].cpu().numpy()
    g0 = plan0.backward(dev, G)[0].cpu().numpy()
    torch.cuda.synchronize()
    gdiff = rel_err(g1, g0)
    say(f"  adjoint packed vs unpacked {gdiff:.3e}")
    assert gdiff < TOL32
    plan.close()
    plan0.close()


@pytest.mark.parametrize("shape", [(8, 64, 16), (8, 128, 16), (8, 256, 16), (8, 512, 16), (512, 8, 32),
                                   (8, 1024, 16), (1024, 8, 16), (8, 256, 64), (8, 128, 64), (8, 64, 64),
                                   (8, 160, 64), (8, 192, 32), (8, 96, 16)])
def test_every_fft_variant(sb, shape):
    # every launch shape of the passes of each axis (what the autotuner may pick) gives the
    # oracle's sums; the middle axis (a plain pass in the forward, kernel-cache and density
    # transforms too) has length 64 / 128 / 256 / 512, or 512 is the first axis (density and
    # kernel-cache transforms, stride 256); a last axis of 64 lets the 64-pencil middle-pass tiles run
    say(f"case: {shape} full 3PCF, 4 bins to 4, lmax 3, every FFT variant of every axis")
    d = lognormal_field(shape, seed=40, sigma=1.0)
    edges = linear_edges(4, 4)
    ref = oracle.zeta3_full(d.astype(np.float64), edges, 3).real
    plan = sb.Plan([d.shape], edges, 3)
    dev = [torch.from_numpy(d).cuda()]
    for axis, n in enumerate(shape):
        for v in range(plan.fft_variants(n)):
            plan.set_fft_variant(n, axis, v)
            z = plan.forward(dev).cpu().numpy()
            check(z[0], ref, TOL32, say, f"axis {axis} length {n} variant {v}: ")
        plan.set_fft_variant(n, axis, 0)
    # tuned choices round-trip through choices / set_choices
    plan.autotune(torch.cuda.current_stream())
    tuned = plan.choices()
    plan.set_choices({"fft": {k: 0 for k in tuned["fft"]}})
    assert all(v == 0 for v in plan.choices()["fft"].values())
    plan.set_choices(tuned)
    assert plan.choices() == tuned
    plan.close()


@pytest.mark.parametrize("shape", [(512, 8, 16), (8, 16, 512), (64, 16, 128), (160, 8, 192), (96, 8, 160),
                                   (192, 8, 96), (1024, 8, 16), (8, 8, 1024)])
def test_long_axes(sb, shape):
    # axis lengths of 512 (the three-stage register-resident forms) and the 64 / 128 pairs,
    # each on the axis-0 pass and on the fused last pass
    say(f"case: {shape} full 3PCF, 4 bins to 4, lmax 3")
    d = lognormal_field(shape, seed=41, sigma=1.0)
    edges = linear_edges(4, 4)
    plan, dev, z = run_plan(sb, [d], edges, 3)
    ref = oracle.zeta3_full(d.astype(np.float64), edges, 3).real
    check(z[0], ref, TOL32, say)
    plan.close()


@pytest.mark.parametrize("n", [512, 1024])
@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_fused_last_pass_long(sb, precision, n):
    # a last axis of 512 or 1024 points: the register-resident fused last pass with one exchange
    # buffer, at 10 bins (12-bin tiles) with the packed m = 0 groups (real and packed pair sums),
    # and its regenerated-kernel form
    say(f"case: 8 x 16 x {n} full 3PCF, 10 bins to 5, lmax 2, {precision}; the same regenerated")
    d = lognormal_field((8, 16, n), seed=43, sigma=1.0)
    edges = linear_edges(5, 10)
    ref = oracle.zeta3_full(d.astype(np.float64), edges, 2).real
    tol = TOL_SPLIT if precision == "split_bf16" else TOL32
    for regen in (False, True):
        plan, dev, z = run_plan(sb, [d], edges, 2, precision=precision, regen_kernels=regen)
        check(z[0], ref, tol, say, f"regenerated {regen}: ")
        plan.close()


@pytest.mark.parametrize("n", [512, 1024])
def test_fused_last_pass_long_projected(sb, n):
    # the complex pair sums of the projected 3PCF on a 512- or 1024-point last axis (12-bin tiles)
    say(f"case: 16 x {n} projected 3PCF, 9 bins to 9, mmax 4")
    d = lognormal_field((16, n), seed=44, sigma=1.0)
    edges = linear_edges(9, 9)
    _, _, z3 = run_plan(sb, [d], edges, 4, npcf=3)
    check(z3[0], oracle.zeta3_proj(d.astype(np.float64), edges, 4), TOL32, say, "proj3: ")


def test_call_order_and_argument_errors(sb):
    # error paths of the C ABI that need a plan (whose creation allocates device tables)
    import ctypes
    from paper_2210_10206_amd import _lib
    lib = _lib.load()
    say("case: C-ABI state and argument errors on a 16^3 plan")
    edges = np.array([0.0, 2.0, 4.0])
    prob = _lib.SbProblem(3, 3, 2, edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 2, 0, 0, 0)
    sh = np.array([16, 16, 16], dtype=np.int64)
    h = ctypes.c_void_p()
    assert lib.sb_plan_create(ctypes.byref(prob), 1, sh.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              ctypes.byref(h)) == 0
    d = torch.zeros((16, 16, 16), dtype=torch.float32, device="cuda")
    z = torch.zeros(64, dtype=torch.float64, device="cuda")
    ptrs = (ctypes.c_void_p * 1)(d.data_ptr())
    assert lib.sb_forward(h, ptrs, ctypes.c_void_p(z.data_ptr()), None) == -3          # not bound
    pb, sbytes = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.sb_plan_workspace(h, ctypes.byref(pb), ctypes.byref(sbytes)) == 0
    pers = torch.empty(pb.value + 256, dtype=torch.uint8, device="cuda")
    scr = torch.empty(sbytes.value + 256, dtype=torch.uint8, device="cuda")
    pp, sp = (pers.data_ptr() + 255) & ~255, (scr.data_ptr() + 255) & ~255
    assert lib.sb_plan_bind(h, ctypes.c_void_p(pp), pb.value - 1, ctypes.c_void_p(sp), sbytes.value) == -3
    assert lib.sb_plan_bind(h, ctypes.c_void_p(pp + 8), pb.value, ctypes.c_void_p(sp), sbytes.value) == -1
    assert lib.sb_plan_bind(h, ctypes.c_void_p(pp), pb.value, ctypes.c_void_p(sp), sbytes.value) == 0
    assert lib.sb_forward(h, ptrs, ctypes.c_void_p(z.data_ptr()), None) == -7          # not prepared
    assert lib.sb_plan_set_scratch_limit(h, ctypes.c_uint64(1 << 20)) == -7            # after bind
    assert lib.sb_plan_set_fft_variant(h, 7, 0, 0) == -1                              # no such length
    assert lib.sb_plan_set_fft_variant(h, 16, 0, 99) == -1                            # no such variant
    assert lib.sb_plan_set_fft_variant(h, 16, 3, 0) == -1                             # no such axis
    assert lib.sb_fft_variants(7) == 0 and lib.sb_fft_variants(16) >= 1
    assert lib.sb_prepare(h, None) == 0
    assert lib.sb_forward(h, ptrs, None, None) == -1                                  # null output
    assert lib.sb_forward(h, ptrs, ctypes.c_void_p(z.data_ptr()), None) == 0
    torch.cuda.synchronize()
    lib.sb_plan_destroy(h)
    # the adjoint exists for the full 3PCF only
    p4 = sb.Plan([(16, 16, 16)], edges, 2, npcf=4)
    with pytest.raises(Exception):
        p4.backward([d], torch.zeros((1, 100), dtype=torch.float64, device="cuda"))
    p4.close()


@pytest.mark.parametrize("shape,npcf,lmax", [((32, 32, 32), 3, 4), ((16, 24, 32), 4, 4), ((64, 96), 4, 4)])
def test_graph_replay_matches_eager(sb, shape, npcf, lmax):
    say(f"case: {shape} npcf {npcf} graph capture + replay vs eager (three replays, eager work between)")
    d = lognormal_field(shape, seed=5, sigma=1.0)
    edges = linear_edges(8, 4)
    plan = sb.Plan([d.shape], edges, lmax, npcf=npcf)
    dev = [torch.from_numpy(d).cuda()]
    eager = plan.forward_raw(dev).cpu().numpy()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    out = torch.empty((1, plan.zeta_doubles), dtype=torch.float64, device="cuda")
    for rep in range(3):
        with torch.cuda.stream(s):
            plan.forward_raw(dev, out=out, stream=s, graph=True)
        s.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, eager), f"replay {rep} differs"
        _ = plan.forward(dev)  # eager work between replays
        torch.cuda.synchronize()
    plan.close()


@pytest.mark.parametrize("nbins", [3, 8, 10, 16])
def test_last_axis_256_bin_counts(sb, nbins):
    # a contiguous axis of 256 takes the register-resident fused last pass; every padded bin
    # count (4, 8, 12, 16) of its tile
    say(f"case: (8, 16, 256) full 3PCF, {nbins} bins to 8, lmax 4")
    d = lognormal_field((8, 16, 256), seed=30 + nbins, sigma=1.0)
    edges = linear_edges(8, nbins)
    plan, dev, z = run_plan(sb, [d], edges, 4)
    ref = oracle.zeta3_full(d.astype(np.float64), edges, 4)
    check(z[0], ref.real, TOL32, say)
    plan.close()


@pytest.mark.parametrize("shape", [(16, 160), (12, 192), (24, 96), (16, 128), (16, 64)])
def test_projected_register_last_pass(sb, shape):
    say(f"case: {shape} projected 3PCF, 4 bins to 6, mmax 4")
    d = lognormal_field(shape, seed=13, sigma=1.0)
    edges = linear_edges(6, 4)
    _, _, z3 = run_plan(sb, [d], edges, 4, npcf=3)
    ref3 = oracle.zeta3_proj(d.astype(np.float64), edges, 4)
    check(z3[0], ref3, TOL32, say, "proj3: ")


def test_projected_last_axis_256(sb):
    say("case: 128 x 256 projected 3PCF, 6 bins to 12, mmax 5")
    d = lognormal_field((128, 256), seed=12, sigma=1.0)
    edges = linear_edges(12, 6)
    _, _, z3 = run_plan(sb, [d], edges, 5, npcf=3)
    ref3 = oracle.zeta3_proj(d.astype(np.float64), edges, 5)
    check(z3[0], ref3, TOL32, say, "proj3: ")


# ------------------------------------------------------------------ projected

def test_projected_small(sb):
    say("case: 64x96 projected 3PCF + 4PCF, 5 bins to 10, mmax 4")
    d = lognormal_field((64, 96), seed=2, sigma=1.0)
    edges = linear_edges(10, 5)
    _, _, z3 = run_plan(sb, [d], edges, 4, npcf=3)
    ref3 = oracle.zeta3_proj(d.astype(np.float64), edges, 4)
    check(z3[0], ref3, TOL32, say, "proj3: ")
    _, _, z4 = run_plan(sb, [d], edges, 4, npcf=4)
    pairs, ref4 = oracle.zeta4_proj(d.astype(np.float64), edges, 4)
    check(z4[0], ref4, TOL32, say, "proj4 matrix cores: ")
    _, _, z4v = run_plan(sb, [d], edges, 4, npcf=4, mfma=False)   # the vector-ALU contraction
    check(z4v[0], ref4, TOL32, say, "proj4 vector ALU: ")


# ------------------------------------------------------------------ full 4PCF

# split-BF16 keeps ~16 mantissa bits of each operand (the lo*lo term is dropped): 2^-16 per
# product, which grows to a few 1e-5 on sums that cancel (TOL_SPLIT = 3e-4)


@pytest.mark.parametrize("precision,mfma", [("fp32", True), ("split_bf16", True), ("fp32", False)])
def test_full4pcf_small(sb, precision, mfma):
    say(f"case: 24^3 full 4PCF, 4 bins to 6, lmax 4, {precision}, matrix cores {mfma}")
    d = lognormal_field((24, 24, 24), seed=4, sigma=1.0)
    edges = linear_edges(6, 4)
    plan, dev, z = run_plan(sb, [d], edges, 4, npcf=4, precision=precision, mfma=mfma)
    lams, ref = oracle.zeta4_full(d.astype(np.float64), edges, 4)
    assert [tuple(x) for x in plan.zeta_index()] == lams
    check(z[0], ref.real, TOL_SPLIT if precision == "split_bf16" else TOL32, say)
    plan.close()


@pytest.mark.parametrize("mfma,parity,lmax", [(True, "even", 4), (False, "even", 3), (True, "odd", 4), (False, "odd", 2)])
def test_full4pcf_packed_m0_arrays(sb, mfma, parity, lmax):
    # the 4PCF coefficients carry the real m = 0 fields two to an array by default; the
    # contraction kernels read those columns through the (array, part) table
    say(f"case: 24^3 full 4PCF, 4 bins to 6, lmax {lmax}, {parity} parity, matrix cores {mfma}: packed vs unpacked")
    d = lognormal_field((24, 24, 24), seed=9, sigma=1.0)
    edges = linear_edges(6, 4)
    plan, dev, z = run_plan(sb, [d], edges, lmax, npcf=4, mfma=mfma, parity=parity)
    plan0, _, z0 = run_plan(sb, [d], edges, lmax, npcf=4, mfma=mfma, parity=parity, pack=False)
    assert plan.persistent_bytes > plan0.persistent_bytes
    diff = rel_err(z[0], z0[0])
    say(f"  packed vs unpacked {diff:.3e}")
    assert diff < TOL32
    if parity == "even":
        lams, ref = oracle.zeta4_full(d.astype(np.float64), edges, lmax)
        check(z[0], ref.real, TOL32, say, "packed vs oracle: ")
    else:
        lams, ref = oracle.zeta4_full(d.astype(np.float64), edges, lmax, parity="odd")
        check(z[0], ref.imag, TOL32, say, "packed vs oracle: ")
    plan.close()
    plan0.close()


@pytest.mark.parametrize("precision,mfma", [("fp32", True), ("split_bf16", True), ("fp32", False)])
def test_full4pcf_odd_parity(sb, precision, mfma):
    # the 23 odd Lambda at lmax 4: the imaginary part of the sums (their real part vanishes)
    say(f"case: 24^3 full 4PCF odd parity, 5 bins to 6, lmax 4, {precision}, matrix cores {mfma}")
    d = lognormal_field((24, 24, 24), seed=14, sigma=1.0)
    edges = linear_edges(6, 5)
    plan, dev, z = run_plan(sb, [d], edges, 4, npcf=4, precision=precision, mfma=mfma, parity="odd")
    lams, ref = oracle.zeta4_full(d.astype(np.float64), edges, 4, parity="odd")
    assert [tuple(x) for x in plan.zeta_index()] == lams and len(lams) == 23
    assert np.max(np.abs(ref.real)) < 1e-9 * np.max(np.abs(ref.imag))
    check(z[0], ref.imag, TOL_SPLIT if precision == "split_bf16" else TOL32, say)
    plan.close()


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_full4pcf_eight_bins_ragged_blocks(sb, precision):
    # 8 bins fill all four 16-pair tiles; 12 x 16 x 24 = 4608 cells leave a half block
    say(f"case: (12,16,24) full 4PCF, 8 bins to 5, lmax 4, {precision}")
    d = lognormal_field((12, 16, 24), seed=6, sigma=1.0)
    edges = linear_edges(5, 8)
    plan, dev, z = run_plan(sb, [d], edges, 4, npcf=4, precision=precision)
    lams, ref = oracle.zeta4_full(d.astype(np.float64), edges, 4)
    check(z[0], ref.real, TOL_SPLIT if precision == "split_bf16" else TOL32, say)
    plan.close()


def test_contract_tile_candidates(sb):
    # every cells-per-workgroup choice of the three cell-parallel contractions, the range
    # check, and the autotuner's pick: the tile only reorders the FP64 partial sums
    say("case: contraction tile candidates: (12,16,24) full 4PCF 8 bins; 64x96 projected 4PCF; "
        "(16,24,32) unfused 3PCF")
    d4 = lognormal_field((12, 16, 24), seed=6, sigma=1.0)
    e4 = linear_edges(5, 8)
    _, ref4 = oracle.zeta4_full(d4.astype(np.float64), e4, 4)
    dp = lognormal_field((64, 96), seed=2, sigma=1.0)
    ep = linear_edges(10, 5)
    _, refp = oracle.zeta4_proj(dp.astype(np.float64), ep, 4)
    d3 = lognormal_field((16, 24, 32), seed=3, sigma=1.0)
    e3 = linear_edges(8, 4)
    ref3 = oracle.zeta3_full(d3.astype(np.float64), e3, 4).real
    for d, edges, kw, ref, (lo_want, hi_want) in (
            (d4, e4, dict(npcf=4), ref4.real, (512, 4096)),
            (dp, ep, dict(npcf=4), refp, (1024, 8192)),
            (d3, e3, dict(npcf=3, fused=False), ref3, (2048, 16384))):
        plan = sb.Plan([d.shape], edges, 4, **kw)
        dev = [torch.from_numpy(d).cuda()]
        cur, (lo, hi) = plan.contract_tile()
        assert (lo, hi) == (lo_want, hi_want) and lo <= cur <= hi
        c = lo
        while c <= hi:
            plan.set_contract_tile(c)
            z = plan.forward(dev)
            torch.cuda.synchronize()
            check(z.cpu().numpy()[0], ref, TOL32, say, f"{d.shape} npcf {kw['npcf']} tile {c}: ")
            c *= 2
        for bad in (lo // 2, 2 * hi, lo + 64):
            with pytest.raises(RuntimeError):
                plan.set_contract_tile(bad)
        plan.autotune(torch.cuda.current_stream())
        tuned = plan.contract_tile()[0]
        z = plan.forward(dev)
        torch.cuda.synchronize()
        check(z.cpu().numpy()[0], ref, TOL32, say, f"{d.shape} npcf {kw['npcf']} tuned tile {tuned}: ")
        assert lo <= tuned <= hi
        plan.close()


def test_full4pcf_lmax3_six_bins(sb):
    # lmax 3: a different canonical Lambda set on the matrix-core path
    say("case: 16^3 full 4PCF, 6 bins to 6, lmax 3")
    d = lognormal_field((16, 16, 16), seed=8, sigma=1.0)
    edges = linear_edges(6, 6)
    plan, dev, z = run_plan(sb, [d], edges, 3, npcf=4)
    lams, ref = oracle.zeta4_full(d.astype(np.float64), edges, 3)
    check(z[0], ref.real, TOL32, say)
    plan.close()


# ------------------------------------------------------------------ adjoint

@pytest.mark.parametrize("shape,nbins", [((8, 16, 256), 10), ((8, 12, 64), 3), ((12, 8, 160), 16), ((256, 8, 12), 6),
                                         ((8, 8, 256), 3), ((8, 12, 256), 7), ((12, 8, 256), 16)])
def test_adjoint_register_last_pass(sb, shape, nbins):
    # the register-resident adjoint last pass at last-axis lengths 256 (4, 8, 12 and 16 padded
    # bins: the skewed LDS layout), 64 and 160 (4 and 16 padded bins), and the register-resident
    # adjoint axis-0 accumulation at 256, against the oracle's gradient at 24 sampled cells
    say(f"case: {shape} adjoint, {nbins} bins to 6, lmax 3, gradient at 24 cells")
    d = lognormal_field(shape, seed=41, sigma=1.0)
    edges = linear_edges(6, nbins)
    rng = np.random.Generator(np.random.PCG64(42))
    G = rng.standard_normal((4, nbins, nbins))
    cells = np.sort(rng.choice(d.size, 24, replace=False))
    plan = sb.Plan([d.shape], edges, 3)
    g = plan.backward([torch.from_numpy(d).cuda()], torch.from_numpy(G)[None].cuda())[0]
    g = g.reshape(-1).double().cpu().numpy()[cells]
    ref = oracle.grad3_full(d.astype(np.float64), edges, 3, G, cells=cells)
    err = float(np.max(np.abs(g - ref)) / np.max(np.abs(ref)))
    say(f"  grad err={err:.3e}")
    assert err < TOL32
    plan.close()


@pytest.mark.parametrize("fused", [True, False])
def test_adjoint_matches_oracle_gradient(sb, fused):
    say(f"case: 16^3 adjoint of the full 3PCF, 4 bins to 4, lmax 3, fused last pass {fused}")
    d = lognormal_field((16, 16, 16), seed=9, sigma=1.0)
    edges = linear_edges(4, 4)
    rng = np.random.Generator(np.random.PCG64(3))
    G = rng.standard_normal((4, 4, 4))
    plan = sb.Plan([d.shape], edges, 3, fused=fused)
    dev = torch.from_numpy(d).cuda().requires_grad_(True)
    z = sb.ZetaFn.apply(dev, plan)
    loss = (z * torch.from_numpy(G).cuda()).sum()
    loss.backward()
    g = dev.grad.cpu().numpy().astype(np.float64)
    ref = oracle.grad3_full(d.astype(np.float64), edges, 3, G)
    err = rel_err(g, ref)
    say(f"  grad err={err:.3e}")
    assert err < TOL32
    plan.close()


# ------------------------------------------------------------------ split-BF16 pair sums

@pytest.mark.parametrize("shape,nbins,lmax,pack", [((16, 16, 32), 4, 3, True), ((8, 16, 256), 10, 6, True),
                                                   ((8, 16, 256), 10, 6, False), ((12, 8, 96), 8, 4, True),
                                                   ((8, 8, 512), 4, 2, True), ((16, 16, 64), 16, 2, True),
                                                   ((16, 8, 160), 6, 4, True), ((8, 12, 128), 12, 5, True)])
def test_split_bf16_full3pcf(sb, shape, nbins, lmax, pack):
    # the fused pair sums on bf16 4x4x4 MFMA with hi + lo splits, on every last-pass family
    # (LDS-staged 32 / 512, register-resident 64 / 128 / 256, radix lists 96 / 160), packed m = 0
    # pairs and one transform per (l, m)
    say(f"case: {shape} full 3PCF split-BF16 pair sums, {nbins} bins to 8, lmax {lmax}, pack {pack}")
    d = lognormal_field(shape, seed=80 + nbins, sigma=1.0)
    edges = linear_edges(8, nbins)
    plan, dev, z = run_plan(sb, [d], edges, lmax, precision="split_bf16", pack=pack)
    _, _, z32 = run_plan(sb, [d], edges, lmax, pack=pack)
    ref = oracle.zeta3_full(d.astype(np.float64), edges, lmax).real
    check(z[0], ref, TOL_SPLIT, say, "split-BF16: ")
    check(z32[0], ref, TOL32, say, "float32: ")
    plan.close()


@pytest.mark.parametrize("shape", [(16, 160), (16, 128), (64, 96), (32, 48), (8, 512)])
def test_split_bf16_projected3pcf(sb, shape):
    say(f"case: {shape} projected 3PCF split-BF16 pair sums, 4 bins to 6, mmax 4")
    d = lognormal_field(shape, seed=13, sigma=1.0)
    edges = linear_edges(6, 4)
    _, _, z3 = run_plan(sb, [d], edges, 4, npcf=3, precision="split_bf16")
    ref3 = oracle.zeta3_proj(d.astype(np.float64), edges, 4)
    check(z3[0], ref3, TOL_SPLIT, say, "split-BF16 proj3: ")


@pytest.mark.parametrize("shape,nbins,mmax", [((64, 96), 5, 4), ((32, 48), 8, 3), ((48, 32), 3, 2), ((64, 64), 10, 5),
                                              ((16, 128), 1, 2)])
def test_split_bf16_projected4pcf(sb, shape, nbins, mmax):
    # the projected-4PCF contraction on bf16 16x16x32 MFMA with hi + lo splits; N tiles of
    # 8 (b3, part) column pairs: 3, 5 and 10 bins leave part of a tile empty, 8 fill it
    say(f"case: {shape} projected 4PCF split-BF16, {nbins} bins to 8, mmax {mmax}")
    d = lognormal_field(shape, seed=90 + nbins, sigma=1.0)
    edges = linear_edges(8, nbins)
    _, _, z = run_plan(sb, [d], edges, mmax, npcf=4, precision="split_bf16")
    _, _, z32 = run_plan(sb, [d], edges, mmax, npcf=4)
    pairs, ref = oracle.zeta4_proj(d.astype(np.float64), edges, mmax)
    check(z[0], ref, TOL_SPLIT, say, "split-BF16: ")
    check(z32[0], ref, TOL32, say, "float32: ")


# ------------------------------------------------------------------ kernel regeneration, 1024 axes

@pytest.mark.parametrize("shape,nbins,lmax,limit_groups", [((32, 32, 32), 4, 4, None), ((16, 24, 32), 6, 3, 2),
                                                           ((8, 16, 256), 10, 6, 3)])
def test_regenerated_kernels_match_cached(sb, shape, nbins, lmax, limit_groups):
    # a plan that keeps no kernel spectra regenerates each chunk's planes with the same kernel
    # generation and transforms: bit-identical to the cached plan without packed pairs that keeps
    # the same planes (regeneration takes the half store where it applies)
    say(f"case: {shape} full 3PCF, {nbins} bins to 6, lmax {lmax}: regenerated kernels "
        f"(chunks of {limit_groups or 'all'} groups) vs cached")
    d = lognormal_field(shape, seed=60 + nbins, sigma=1.0)
    edges = linear_edges(6, nbins)
    kw = {} if limit_groups is None else dict(scratch_limit=limit_groups * nbins * d.size * 8)
    plan, dev, z = run_plan(sb, [d], edges, lmax, regen_kernels=True, **kw)
    plan0, _, z0 = run_plan(sb, [d], edges, lmax, pack=False, half_kernels=True, **kw)
    assert plan.persistent_bytes < plan0.persistent_bytes
    assert np.array_equal(z, z0)
    check(z[0], oracle.zeta3_full(d.astype(np.float64), edges, lmax).real, TOL32, say)
    with pytest.raises(Exception):     # no adjoint without the cached spectra
        plan.backward(dev, torch.zeros((1, lmax + 1, nbins, nbins), dtype=torch.float64, device="cuda"))
    plan.close()
    plan0.close()


@pytest.mark.parametrize("shape", [(64, 16, 16), (128, 16, 24), (256, 16, 16), (96, 16, 16), (160, 16, 16),
                                   (192, 24, 16), (512, 16, 16), (1024, 16, 16), (32, 24, 16), (48, 16, 24)])
def test_half_kernel_store(sb, shape):
    # kernel planes c_0 < 0 taken from c_0 > 0 by parity (packed m = 0 pairs by conjugation) in
    # every axis-0 kernel family: register-resident 64 / 128 / 256, radix lists 96 / 160 / 192 /
    # 512 / 1024, LDS-staged 32 / 48; the fused and unfused 3PCF, the full 4PCF and the adjoint
    say(f"case: {shape} half kernel store, 4 bins to 4, lmax 3: fused, unfused, 4PCF, adjoint")
    d = lognormal_field(shape, seed=45, sigma=1.0)
    edges = linear_edges(4, 4)
    d64 = d.astype(np.float64)
    ref3 = oracle.zeta3_full(d64, edges, 3).real
    plan, dev, z = run_plan(sb, [d], edges, 3, half_kernels=True)
    full, _, zf = run_plan(sb, [d], edges, 3)
    assert plan.persistent_bytes < full.persistent_bytes
    check(z[0], ref3, TOL32, say, "fused: ")
    check(zf[0], ref3, TOL32, say, "full store: ")
    if shape[0] <= 512:
        rng = np.random.Generator(np.random.PCG64(7))
        G = rng.standard_normal((4, 4, 4))
        cells = np.sort(rng.choice(d.size, 16, replace=False))
        g = plan.backward(dev, torch.from_numpy(G)[None].cuda())[0].reshape(-1).double().cpu().numpy()[cells]
        ref = oracle.grad3_full(d64, edges, 3, G, cells=cells)
        err = float(np.max(np.abs(g - ref)) / np.max(np.abs(ref)))
        say(f"  adjoint err={err:.3e}")
        assert err < TOL32
    plan.close()
    full.close()
    if shape[0] <= 192:
        _, _, zu = run_plan(sb, [d], edges, 3, half_kernels=True, fused=False)
        check(zu[0], ref3, TOL32, say, "unfused: ")
        _, _, z4 = run_plan(sb, [d], edges, 3, npcf=4, half_kernels=True)
        check(z4[0], oracle.zeta4_full(d64, edges, 3)[1].real, TOL32, say, "4PCF: ")


@pytest.mark.parametrize("shape,npcf", [((64, 96), 3), ((48, 64), 4), ((24, 24, 12), 3), ((16, 8, 32), 4)])
def test_half_kernel_store_not_applicable(sb, shape, npcf):
    # the half store applies to 3D shapes whose support radius stays below half of every edge:
    # on a 2D plan, or with an edge of at most 2 r0 (here r0 = 6 against edges of 12 and 8), the
    # flag leaves the plan unchanged, bit for bit (and a 16-point edge, above 2 r0, takes it)
    say(f"case: {shape} npcf {npcf}, 4 bins to 6, lmax 3: half-store flag where it does not apply")
    d = lognormal_field(shape, seed=46, sigma=1.0)
    edges = linear_edges(6, 4)
    p1, _, z1 = run_plan(sb, [d], edges, 3, npcf=npcf, half_kernels=True)
    p0, _, z0 = run_plan(sb, [d], edges, 3, npcf=npcf)
    assert p1.persistent_bytes == p0.persistent_bytes
    assert np.array_equal(z1, z0)
    p1.close()
    p0.close()
    if len(shape) == 3:
        p2, _, _ = run_plan(sb, [lognormal_field((24, 24, 16), seed=46, sigma=1.0)], edges, 3, npcf=npcf,
                            half_kernels=True)
        p3, _, _ = run_plan(sb, [lognormal_field((24, 24, 16), seed=46, sigma=1.0)], edges, 3, npcf=npcf)
        assert p2.persistent_bytes < p3.persistent_bytes
        p2.close()
        p3.close()


@pytest.mark.parametrize("shape,npcf", [((8, 16, 1024), 3), ((1024, 8, 16), 3), ((8, 1024, 16), 3), ((16, 1024), 3),
                                        ((1024, 16), 3), ((8, 8, 1024), 4), ((16, 1024), 4)])
def test_axes_of_1024(sb, shape, npcf):
    # transforms of length 1024 on every axis: the axis-0 correlation pass, the middle pass, and the
    # last pass (fused with the pair sums for the 3PCF; the 4PCF's plain pass)
    say(f"case: {shape} npcf {npcf}, 4 bins to 4, lmax 3")
    d = lognormal_field(shape, seed=44, sigma=1.0)
    edges = linear_edges(4, 4)
    plan, dev, z = run_plan(sb, [d], edges, 3, npcf=npcf)
    d64 = d.astype(np.float64)
    if len(shape) == 3:
        ref = oracle.zeta3_full(d64, edges, 3).real if npcf == 3 else oracle.zeta4_full(d64, edges, 3)[1].real
    else:
        ref = oracle.zeta3_proj(d64, edges, 3) if npcf == 3 else oracle.zeta4_proj(d64, edges, 3)[1]
    check(z[0], ref, TOL32, say)
    if npcf == 3 and len(shape) == 3 and shape[2] == 1024:
        with pytest.raises(Exception):   # the adjoint has no last pass at 1024
            plan.backward(dev, torch.zeros((1, 4, 4, 4), dtype=torch.float64, device="cuda"))
    plan.close()


# ------------------------------------------------------------------ batched launches

@pytest.mark.parametrize("kind", ["full3", "full4_mfma", "full4_split", "full4_valu", "full4_odd", "proj3", "proj4",
                                  "proj4_split", "proj4_valu"])
def test_field_batches_match_single_fields(sb, kind):
    # fields of one shape share every pass launch (the field is the launch's third grid dimension):
    # each field's sums equal those of one launch sequence per field, bit for bit, on an uneven
    # batch whose shapes interleave
    say(f"case: field batches vs one launch sequence per field, {kind}")
    full = kind.startswith("full")
    shapes = [(16, 16, 16), (24, 24, 24), (16, 16, 16), (24, 24, 24), (16, 16, 16)] if full else \
             [(64, 96), (32, 48), (64, 96), (64, 96), (32, 48)]
    fields = [lognormal_field(sh, seed=100 + i, sigma=1.0) for i, sh in enumerate(shapes)]
    edges = linear_edges(6, 4)
    kw = dict(npcf=3 if kind in ("full3", "proj3") else 4)
    if kind.endswith("split"):
        kw["precision"] = "split_bf16"
    if kind.endswith("valu"):
        kw["mfma"] = False
    if kind.endswith("odd"):
        kw["parity"] = "odd"
    lmax = 4 if full else 3
    pb, dev, zb = run_plan(sb, fields, edges, lmax, **kw)
    p1, _, z1 = run_plan(sb, fields, edges, lmax, field_batch=1, **kw)
    say(f"  fields per launch: {pb.field_batch} (batched plan), {p1.field_batch}")
    assert pb.field_batch == 3 and p1.field_batch == 1
    assert np.array_equal(zb, z1)
    # the batched plan replayed from a HIP graph, three times with eager work between
    s = torch.cuda.Stream()
    out = torch.empty((len(fields), pb.zeta_doubles), dtype=torch.float64, device="cuda")
    for rep in range(3):
        with torch.cuda.stream(s):
            pb.forward_raw(dev, out=out, stream=s, graph=True)
        s.synchronize()
        assert np.array_equal(pb.unpack(out).cpu().numpy(), zb), f"graph replay {rep}"
        _ = p1.forward(dev)
        torch.cuda.synchronize()
    # and against the oracle for one field of each shape
    for i in (0, 1):
        d64 = fields[i].astype(np.float64)
        if kind == "full3":
            ref = oracle.zeta3_full(d64, edges, lmax).real
        elif kind.startswith("full4"):
            lams, r = oracle.zeta4_full(d64, edges, lmax, parity="odd" if kind.endswith("odd") else "even")
            ref = r.imag if kind.endswith("odd") else r.real
        elif kind == "proj3":
            ref = oracle.zeta3_proj(d64, edges, lmax)
        else:
            ref = oracle.zeta4_proj(d64, edges, lmax)[1]
        check(zb[i], ref, TOL_SPLIT if kind.endswith("split") else TOL32, say, f"field {i} {shapes[i]}: ")
    pb.close()
    p1.close()
