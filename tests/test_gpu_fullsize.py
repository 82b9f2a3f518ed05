"""GPU parity at the workloads' full sizes, against oracle values stored by
tests/golden/make_golden.py (which calls only the oracle), and sampled coefficient checks
the oracle computes cell by cell.

Tolerance: max |Z_gpu - Z_oracle| / max |Z_oracle| <= 1e-5 (float32 path; 3e-4 split-BF16),
over the whole result and over every leading-index block (per l, per Lambda, per m or per
(m1, m2)), each block relative to its own max |Z_oracle| (tests/parity.py).
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from fieldgen import lognormal_field, linear_edges, c5_shapes, sparse_unit_field  # noqa: E402
from parity import TOL32, TOL_SPLIT, check, rel_err  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"stored oracle values {name} not generated")
    return np.load(path)


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_10206_amd as pkg
    pkg.load()
    from paper_2210_10206_amd import api as a
    return a


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_projected_512(api, precision):
    say(f"case: 512^2 float32 lognormal seed 0, 10 bins to 40, m up to 10: projected 3PCF + 4PCF, {precision}")
    g = golden("c2_proj_512.npz")
    d = lognormal_field((512, 512), seed=0, sigma=1.0)
    edges = linear_edges(40, 10)
    dev = [torch.from_numpy(d).cuda()]
    p3 = api.Plan([d.shape], edges, 10, npcf=3, precision=precision)
    z3 = p3.forward(dev)[0].cpu().numpy()
    p4 = api.Plan([d.shape], edges, 10, npcf=4, precision=precision)
    z4 = p4.forward(dev)[0].cpu().numpy()
    torch.cuda.synchronize()
    assert [tuple(x) for x in p4.zeta_index()] == [tuple(x) for x in g["pairs"]]
    tol = TOL_SPLIT if precision == "split_bf16" else TOL32
    check(z3, g["zeta3"], tol, say, "proj3 (m blocks): ")
    check(z4, g["zeta4"], tol, say, "proj4 ((m1, m2) blocks): ")
    p3.close()
    p4.close()


@pytest.mark.parametrize("precision,mfma,tol", [("fp32", True, TOL32), ("split_bf16", True, TOL_SPLIT),
                                                ("fp32", False, TOL32)])
def test_full4pcf_128_batch_fields(api, precision, mfma, tol):
    say(f"case: fields 0 and 1 of the 16-field 128^3 batch, 8 bins to 24, even Lambda, lmax 4, "
        f"{precision}, matrix cores {mfma}")
    gs = [golden(f"c4_full4_128_field{i}.npz") for i in (0, 1)]
    fields = [lognormal_field((128,) * 3, seed=i, sigma=float(gs[i]["sigma"])) for i in (0, 1)]
    edges = linear_edges(24, 8)
    plan = api.Plan([f.shape for f in fields], edges, 4, npcf=4, precision=precision, mfma=mfma)
    z = plan.forward([torch.from_numpy(f).cuda() for f in fields]).cpu().numpy()
    torch.cuda.synchronize()
    assert [tuple(x) for x in plan.zeta_index()] == [tuple(x) for x in gs[0]["lams"]]
    for i in (0, 1):
        ref = gs[i]["zeta4"]
        assert np.max(np.abs(ref.imag)) < 1e-9 * np.max(np.abs(ref.real))
        check(z[i], ref.real, tol, say, f"field {i} (Lambda blocks): ")
    plan.close()


def test_uneven_batch_sizes(api):
    say("case: one field of each edge 64/96/128/160/192 and a second 64^3 field in one uneven plan, "
        "8 bins to 16, lmax 4")
    edges_list = c5_shapes()
    first = {}
    for i, n in enumerate(edges_list):
        first.setdefault(n, i)
    items = sorted(first.items())
    items.append((64, [i for i, n in enumerate(edges_list) if n == 64][1]))
    fields = [lognormal_field((n,) * 3, seed=i, sigma=1.0) for n, i in items]
    refs = [golden(f"c5_full3_{n}_field{i}.npz")["zeta3"].real for n, i in items]
    edges = linear_edges(16, 8)
    plan = api.Plan([f.shape for f in fields], edges, 4, npcf=3)
    z = plan.forward([torch.from_numpy(f).cuda() for f in fields]).cpu().numpy()
    torch.cuda.synchronize()
    for (n, i), zi, ref in zip(items, z, refs):
        check(zi, ref, TOL32, say, f"{n}^3 (field {i}, l blocks): ")
    plan.close()


@pytest.mark.parametrize("seed,sigma,precision", [(0, 0.5, "fp32"), (1, 1.5, "fp32"), (0, 0.5, "split_bf16"),
                                                   (1, 1.5, "split_bf16")])
def test_full3pcf_256(api, seed, sigma, precision):
    say(f"case: 256^3 full 3PCF seed {seed} sigma {sigma}, 10 bins to 32, lmax 6, {precision} pair sums")
    g = golden(f"c3_full3_256_seed{seed}.npz")
    d = lognormal_field((256,) * 3, seed=seed, sigma=sigma)
    edges = linear_edges(32, 10)
    plan = api.Plan([d.shape], edges, 6, npcf=3, precision=precision)
    z = plan.forward([torch.from_numpy(d).cuda()])[0].cpu().numpy()
    torch.cuda.synchronize()
    ref = g["zeta3"].real
    check(z, ref, TOL_SPLIT if precision == "split_bf16" else TOL32, say, "l blocks: ")
    # and per zeta_l^{b1 b2} entry, relative to max |Z_l| of its l
    per_entry = np.abs(z - ref) / np.max(np.abs(ref), axis=(1, 2), keepdims=True)
    say(f"  worst entry (relative to its l block) {np.max(per_entry):.3e}")
    plan.close()


def test_full3pcf_512_sparse_field(api):
    """512^3 (kernel arrays in chunks of (l, m) groups next to the 39 GiB compact cache) on a
    non-periodic field: 16384 unit-weight cells scattered over the whole box, 10 bins to 32,
    lmax 6.  The sums only involve the occupied cells, which the oracle evaluates directly
    (its sum restricted to them is the whole sum)."""
    say("case: 16384 particles on 512^3, 10 bins to 32, lmax 6: full 3PCF vs the oracle at the occupied cells")
    d = sparse_unit_field((512,) * 3, 16384, seed=512)
    cells = np.flatnonzero(d.reshape(-1))
    edges = linear_edges(32, 10)
    dev = torch.from_numpy(d.astype(np.float32)).cuda()
    plan = api.Plan([d.shape], edges, 6, npcf=3)
    say(f"  512^3 plan: persistent {plan.persistent_bytes / 2**30:.1f} GiB, scratch {plan.scratch_bytes / 2**30:.1f} GiB")
    z = plan.forward([dev])[0].cpu().numpy()
    torch.cuda.synchronize()
    plan.close()
    del plan, dev
    torch.cuda.empty_cache()
    say("  oracle at the occupied cells")
    ref = oracle.zeta3_full(d, edges, 6, cells=cells).real
    check(z, ref, TOL32, say, "l blocks: ")


def test_full3pcf_1024_sparse_field(api):
    """1024^3: the kernel spectra are not cached (they would take about 169 GB): each chunk of
    (l, m) groups regenerates its kernel planes, and the length-1024 last axis runs the plain
    last pass and the pair contraction.  16384 unit-weight cells scattered over the box, 10 bins
    to 32, lmax 6, against the oracle at the occupied cells."""
    say("case: 16384 particles on 1024^3, 10 bins to 32, lmax 6: full 3PCF vs the oracle at the occupied cells")
    torch.cuda.empty_cache()
    d = sparse_unit_field((1024,) * 3, 16384, seed=1024)
    cells = np.flatnonzero(d.reshape(-1))
    edges = linear_edges(32, 10)
    dev = torch.from_numpy(d.astype(np.float32)).cuda()
    plan = api.Plan([d.shape], edges, 6, npcf=3)
    say(f"  1024^3 plan: persistent {plan.persistent_bytes / 2**30:.3f} GiB, scratch {plan.scratch_bytes / 2**30:.1f} GiB")
    z = plan.forward([dev])[0].cpu().numpy()
    torch.cuda.synchronize()
    plan.close()
    del plan, dev
    torch.cuda.empty_cache()
    say("  oracle at the occupied cells")
    ref = oracle.zeta3_full(d, edges, 6, cells=cells).real
    del d
    check(z, ref, TOL32, say, "l blocks: ")


def test_coefficients_256_sampled(api):
    say("case: 256^3 coefficients at 24 sampled cells vs the oracle, 10 bins to 32, lmax 6")
    d = lognormal_field((256,) * 3, seed=0, sigma=0.5)
    edges = linear_edges(32, 10)
    plan = api.Plan([d.shape], edges, 6, npcf=3, keep_coeffs=True)
    plan.forward([torch.from_numpy(d).cuda()])
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(21))
    cells = np.sort(rng.choice(d.size, 24, replace=False))
    ref = oracle.coeffs_full(d.astype(np.float64), edges, 6, cells=cells)
    worst = 0.0
    for l in range(7):
        for m in range(l + 1):
            lm = l * (l + 1) // 2 + m
            for b in range(10):
                a = plan.coeffs(lm * 10 + b).reshape(-1)[torch.from_numpy(cells).cuda()].cpu().numpy()
                r = ref[:, b, l * l + m + l]
                worst = max(worst, float(np.max(np.abs(a - r)) / np.max(np.abs(ref[:, b, :]))))
    say(f"  coefficient err (rel. to max |a| per bin) = {worst:.3e}")
    assert worst < 2e-6
    plan.close()


def test_particles_on_grid_full_128(api):
    """The validation set-up of Sec. 2.5 with our own draws: 104 unit-weight cells on a 128^3
    grid (delta = the weight grid), 10 linear bins; the sums only involve the occupied cells,
    which the oracle evaluates directly (its sum restricted to those cells is the whole sum)."""
    say("case: 104 particles on 128^3, 10 bins to 20: full 3PCF (lmax 4) and even 4PCF (lmax 2)")
    d = sparse_unit_field((128,) * 3, 104, seed=2210)
    cells = np.flatnonzero(d.reshape(-1))
    edges = linear_edges(20, 10)
    dev = [torch.from_numpy(d.astype(np.float32)).cuda()]
    p3 = api.Plan([d.shape], edges, 4, npcf=3)
    z3 = p3.forward(dev)[0].cpu().numpy()
    p3.close()
    r3 = oracle.zeta3_full(d, edges, 4, cells=cells).real
    p4 = api.Plan([d.shape], edges, 2, npcf=4)
    z4 = p4.forward(dev)[0].cpu().numpy()
    p4.close()
    lams, r4 = oracle.zeta4_full(d, edges, 2, cells=cells)
    check(z3, r3, TOL32, say, "3PCF: ")
    check(z4, r4.real, TOL32, say, f"4PCF ({len(lams)} Lambda): ")


def test_particles_on_grid_projected_256(api):
    """41 unit-weight cells on a 256^2 grid, 10 linear bins (the projected validation set-up
    of Sec. 2.5 with our own draw): projected 3PCF and 4PCF, m up to 4."""
    say("case: 41 particles on 256^2, 10 bins to 30, mmax 4: projected 3PCF and 4PCF")
    d = sparse_unit_field((256, 256), 41, seed=41)
    cells = np.flatnonzero(d.reshape(-1))
    edges = linear_edges(30, 10)
    dev = [torch.from_numpy(d.astype(np.float32)).cuda()]
    p3 = api.Plan([d.shape], edges, 4, npcf=3)
    z3 = p3.forward(dev)[0].cpu().numpy()
    p3.close()
    r3 = oracle.zeta3_proj(d, edges, 4, cells=cells)
    p4 = api.Plan([d.shape], edges, 4, npcf=4)
    z4 = p4.forward(dev)[0].cpu().numpy()
    p4.close()
    pairs, r4 = oracle.zeta4_proj(d, edges, 4, cells=cells)
    check(z3, r3, TOL32, say, "proj3: ")
    check(z4, r4, TOL32, say, "proj4: ")

