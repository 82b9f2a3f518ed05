"""GPU parity at the workloads' full sizes, against oracle values stored by
tests/golden/make_golden.py (which calls only the oracle), and sampled coefficient checks
the oracle computes cell by cell.

Tolerance: max |Z_gpu - Z_oracle| / max |Z_oracle| <= 1e-5 (float32 path), also reported
per leading-index block (per l, per Lambda, per m or per (m1, m2)).
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from fieldgen import lognormal_field, linear_edges, c5_shapes, sparse_unit_field  # noqa: E402

TOL32 = 1e-5
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(got, ref):
    return float(np.max(np.abs(np.asarray(got) - np.asarray(ref))) / np.max(np.abs(ref)))


def worst_block(got, ref):
    """Largest per-block error, each block relative to its own max |ref|."""
    out = 0.0
    for i in range(ref.shape[0]):
        m = np.max(np.abs(ref[i]))
        if m > 0:
            out = max(out, float(np.max(np.abs(got[i] - ref[i])) / m))
    return out


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


def test_projected_512(api):
    say("case: 512^2 float32 lognormal seed 0, 10 bins to 40, m up to 10: projected 3PCF + 4PCF")
    g = golden("c2_proj_512.npz")
    d = lognormal_field((512, 512), seed=0, sigma=1.0)
    edges = linear_edges(40, 10)
    dev = [torch.from_numpy(d).cuda()]
    p3 = api.Plan([d.shape], edges, 10, npcf=3)
    z3 = p3.forward(dev)[0].cpu().numpy()
    p4 = api.Plan([d.shape], edges, 10, npcf=4)
    z4 = p4.forward(dev)[0].cpu().numpy()
    torch.cuda.synchronize()
    assert [tuple(x) for x in p4.zeta_index()] == [tuple(x) for x in g["pairs"]]
    e3, e4 = rel_err(z3, g["zeta3"]), rel_err(z4, g["zeta4"])
    say(f"  proj3 err={e3:.3e} (worst m block {worst_block(z3, g['zeta3']):.3e}); "
        f"proj4 err={e4:.3e} (worst (m1,m2) block {worst_block(z4, g['zeta4']):.3e})")
    assert e3 < TOL32 and e4 < TOL32
    p3.close()
    p4.close()


@pytest.mark.parametrize("precision,mfma,tol", [("fp32", True, TOL32), ("split_bf16", True, 3e-4),
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
        e = rel_err(z[i], ref.real)
        say(f"  field {i}: err={e:.3e} (worst Lambda block {worst_block(z[i], ref.real):.3e})")
        assert e < tol
    plan.close()


def test_uneven_batch_sizes(api):
    say("case: one field of each edge 64/96/128/160/192 in one uneven plan, 8 bins to 16, lmax 4")
    edges_list = c5_shapes()
    first = {}
    for i, n in enumerate(edges_list):
        first.setdefault(n, i)
    items = sorted(first.items())
    fields = [lognormal_field((n,) * 3, seed=i, sigma=1.0) for n, i in items]
    refs = [golden(f"c5_full3_{n}_field{i}.npz")["zeta3"].real for n, i in items]
    edges = linear_edges(16, 8)
    plan = api.Plan([f.shape for f in fields], edges, 4, npcf=3)
    z = plan.forward([torch.from_numpy(f).cuda() for f in fields]).cpu().numpy()
    torch.cuda.synchronize()
    for (n, i), zi, ref in zip(items, z, refs):
        e = rel_err(zi, ref)
        say(f"  {n}^3 (field {i}): err={e:.3e} (worst l block {worst_block(zi, ref):.3e})")
        assert e < TOL32
    plan.close()


@pytest.mark.parametrize("seed,sigma", [(0, 0.5), (1, 1.5)])
def test_full3pcf_256(api, seed, sigma):
    say(f"case: 256^3 full 3PCF seed {seed} sigma {sigma}, 10 bins to 32, lmax 6")
    g = golden(f"c3_full3_256_seed{seed}.npz")
    d = lognormal_field((256,) * 3, seed=seed, sigma=sigma)
    edges = linear_edges(32, 10)
    plan = api.Plan([d.shape], edges, 6, npcf=3)
    z = plan.forward([torch.from_numpy(d).cuda()])[0].cpu().numpy()
    torch.cuda.synchronize()
    ref = g["zeta3"].real
    e = rel_err(z, ref)
    say(f"  err={e:.3e} (worst l block {worst_block(z, ref):.3e})")
    assert e < TOL32
    plan.close()


def test_full3pcf_512_tiled(api):
    """512^3 (kernel arrays in chunks of (l, m) groups next to the 38 GB compact cache): the
    2 x 2 x 2 periodic tiling of a 256^3 field has the same coefficients at every cell as the
    256^3 field (every kernel offset is shorter than the 256 period), so its sums are exactly
    8 times the 256^3 sums."""
    say("case: 512^3 = 2x2x2 tiling of the 256^3 sigma 0.5 seed 0 field, 10 bins to 32, lmax 6")
    d = lognormal_field((256,) * 3, seed=0, sigma=0.5)
    edges = linear_edges(32, 10)
    p256 = api.Plan([d.shape], edges, 6, npcf=3)
    z256 = p256.forward([torch.from_numpy(d).cuda()])[0].cpu().numpy()
    p256.close()
    del p256
    torch.cuda.empty_cache()
    big = torch.from_numpy(d).cuda().repeat(2, 2, 2).contiguous()
    p512 = api.Plan([tuple(big.shape)], edges, 6, npcf=3)
    say(f"  512^3 plan: persistent {p512.persistent_bytes / 2**30:.1f} GiB, scratch {p512.scratch_bytes / 2**30:.1f} GiB")
    z512 = p512.forward([big])[0].cpu().numpy()
    torch.cuda.synchronize()
    p512.close()
    e = rel_err(z512, 8.0 * z256)
    say(f"  max |Z_512 - 8 Z_256| / max |8 Z_256| = {e:.3e}")
    assert e < TOL32


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
    """The validation set-up of Sec. 3.2 with our own draws: 104 unit-weight cells on a 128^3
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
    e3, e4 = rel_err(z3, r3), rel_err(z4, r4.real)
    say(f"  3PCF err={e3:.3e}; 4PCF err={e4:.3e} ({len(lams)} Lambda)")
    assert e3 < TOL32 and e4 < TOL32


def test_particles_on_grid_projected_256(api):
    """41 unit-weight cells on a 256^2 grid, 10 linear bins (the projected validation set-up
    of Sec. 3.2 with our own draw): projected 3PCF and 4PCF, m up to 4."""
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
    e3, e4 = rel_err(z3, r3), rel_err(z4, r4)
    say(f"  proj3 err={e3:.3e}; proj4 err={e4:.3e}")
    assert e3 < TOL32 and e4 < TOL32

