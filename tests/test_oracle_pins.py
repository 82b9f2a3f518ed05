"""Pins for the FP64 oracle: brute force, closed forms, invariants (CPU only)."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle.api import support
from fieldgen import lognormal_field, linear_edges, sparse_unit_field
import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------- binning

def test_bin_counts_integer_edges_match_enumeration():
    for shape, R, nb in [((32, 32, 32), 8, 4), ((512, 512), 40, 10), ((128,) * 3, 24, 8),
                         ((64,) * 3, 16, 8), ((24,) * 3, 16, 8), ((9, 10, 11), 4, 4)]:
        edges = linear_edges(R, nb)
        eint = [int(round(e)) for e in edges]
        assert all(float(a) == b for a, b in zip(eint, edges))
        off_bf, bins_bf = bf.int_offsets(shape, eint)
        counts = oracle.bin_counts(shape, edges)
        assert list(counts) == list(np.bincount(bins_bf, minlength=nb)), shape


def test_bin_counts_fixture():
    """Exact per-bin cell counts of the five workloads (fixture from an exact
    integer enumeration, including the rational edges 3.2 b of the 256^3 case)."""
    with open(os.path.join(GOLDEN, "bin_counts.json")) as f:
        fx = json.load(f)
    for case in fx["cases"]:
        c = oracle.bin_counts(tuple(case["shape"]), linear_edges(case["rmax"], case["nbins"]))
        assert list(c) == case["counts"], case["name"]


def test_ties_on_edges_go_to_lower_bin():
    # |r| = 2 exactly sits on edge e_1 = 2 of edges (0, 2, 4): it belongs to bin 0 = (0, 2].
    off, bins, _ = support((16, 16, 16), [0.0, 2.0, 4.0])
    r2 = (off.astype(np.int64) ** 2).sum(axis=1)
    assert np.all(bins[r2 == 4] == 0)
    assert np.all(bins[r2 == 16] == 1)
    assert not np.any(r2 == 0)


# ---------------------------------------------------------------- 3j symbols

def test_threej_closed_form_and_orthogonality():
    for l in range(7):
        for m in range(-l, l + 1):
            assert abs(oracle.threej(l, l, 0, m, -m, 0) - (-1) ** (l - m) / math.sqrt(2 * l + 1)) < 1e-15
    for l1, l2 in itertools.product(range(5), range(5)):
        for l3 in range(abs(l1 - l2), l1 + l2 + 1):
            for m3 in range(-l3, l3 + 1):
                s = sum(oracle.threej(l1, l2, l3, m1, m2, m3) ** 2
                        for m1 in range(-l1, l1 + 1) for m2 in range(-l2, l2 + 1) if m1 + m2 + m3 == 0)
                assert abs(s - 1.0 / (2 * l3 + 1)) < 1e-14


def test_threej_against_sympy():
    from sympy.physics.wigner import wigner_3j
    for l1, l2, l3 in [(1, 1, 2), (2, 3, 3), (4, 4, 4), (3, 4, 5), (6, 6, 6), (2, 2, 4)]:
        for m1 in range(-l1, l1 + 1):
            for m2 in range(-l2, l2 + 1):
                m3 = -m1 - m2
                if abs(m3) > l3:
                    continue
                assert abs(oracle.threej(l1, l2, l3, m1, m2, m3) - float(wigner_3j(l1, l2, l3, m1, m2, m3))) < 1e-15


def test_lambda_and_pair_tables():
    lams = oracle.lambdas(4)
    assert len(lams) == 42
    assert len(oracle.lambdas(4, "both")) == 65
    assert lams[0] == (0, 0, 0) and lams[1] == (0, 1, 1)
    assert len(oracle.mpairs(10)) == 331
    assert oracle.mpairs(1) == [(-1, 0), (-1, 1), (0, -1), (0, 0), (0, 1), (1, -1), (1, 0)]


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("shape", [(8, 8, 8), (7, 8, 9)])
def test_zeta3_full_vs_legendre_bruteforce(shape, rng):
    d = rng.standard_normal(shape)
    d -= d.mean()
    edges = [0, 1, 2, 3]
    Z = oracle.zeta3_full(d, [float(e) for e in edges], 4)
    B = bf.zeta3_legendre(d, edges, 4)
    assert rel(Z.real, B) < 1e-12
    assert np.max(np.abs(Z.imag)) < 1e-12 * np.max(np.abs(Z.real))


@pytest.mark.parametrize("lam", [(1, 1, 2), (2, 2, 2), (1, 2, 3), (2, 1, 1), (1, 1, 1), (0, 0, 0)])
def test_zeta4_full_vs_quadruplets(lam, rng):
    # (1,1,1) is totally antisymmetric in the bins, so it needs three bins to be non-zero
    shape, edges = ((7, 7, 7), [0, 1, 2, 3]) if lam == (1, 1, 1) else ((6, 6, 6), [0, 1, 2])
    d = rng.standard_normal(shape)
    d -= d.mean()
    parity = "even" if sum(lam) % 2 == 0 else "odd"
    lams, Z = oracle.zeta4_full(d, [float(e) for e in edges], 3, parity=parity)
    Zl = Z[lams.index(lam)]
    B = bf.zeta4_quadruplets(d, edges, lam)
    assert rel(Zl, B) < 1e-12
    if parity == "even":
        assert np.max(np.abs(Zl.imag)) < 1e-12 * np.max(np.abs(Zl.real))
    else:
        assert np.max(np.abs(Zl.real)) < 1e-12 * np.max(np.abs(Zl.imag))


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_zeta4_0ll_vs_legendre(l, rng):
    d = rng.standard_normal((7, 7, 7))
    d -= d.mean()
    lams, Z = oracle.zeta4_full(d, [0.0, 1.0, 2.0], 3)
    B = bf.zeta4_0ll_legendre(d, [0, 1, 2], l)
    assert rel(Z[lams.index((0, l, l))].real, B) < 1e-12


def test_zeta3_proj_vs_pairs(rng):
    d = rng.standard_normal((10, 12))
    d -= d.mean()
    Z = oracle.zeta3_proj(d, [0.0, 1.0, 2.0, 3.0], 4)
    B = bf.zeta3_proj_pairs(d, [0, 1, 2, 3], 4)
    assert rel(Z, B) < 1e-12


def test_zeta4_proj_vs_triples(rng):
    d = rng.standard_normal((10, 12))
    d -= d.mean()
    pairs, Z = oracle.zeta4_proj(d, [0.0, 1.0, 2.0, 3.0], 3)
    for (m1, m2) in [(2, 1), (-3, 1), (0, 0), (1, -3), (3, -3), (-2, -1)]:
        B = bf.zeta4_proj_triples(d, [0, 1, 2, 3], m1, m2)
        assert rel(Z[pairs.index((m1, m2))], B) < 1e-12, (m1, m2)


def test_particle_field_agrees_with_counting(rng):
    """Sparse unit-weight cells (the particle-on-grid inputs of the validation section)."""
    d = sparse_unit_field((12, 12, 12), 60, seed=5)
    Z = oracle.zeta3_full(d, [0.0, 1.0, 2.0, 3.0], 3)
    B = bf.zeta3_legendre(d, [0, 1, 2, 3], 3)
    assert rel(Z.real, B) < 1e-12


# ---------------------------------------------------------------- closed forms

def test_constant_field_closed_form():
    c = 1.7
    N = 16
    d = np.full((N, N, N), c)
    edges = linear_edges(6, 3)
    Z = oracle.zeta3_full(d, edges, 6).real
    counts = oracle.bin_counts((N, N, N), edges)
    # l = 0: every a_00^b = c N_b / sqrt(4 pi)
    expect0 = N ** 3 * c ** 3 * np.outer(counts, counts) / (4 * math.pi)
    assert rel(Z[0], expect0) < 1e-13
    # cubic lattice shells: the lattice sums of Y_lm vanish for l = 1, 2, 3, 5
    for l in (1, 2, 3, 5):
        assert np.max(np.abs(Z[l])) < 1e-10 * np.max(np.abs(Z[0]))
    assert np.max(np.abs(Z[4])) > 1e-6 * np.max(np.abs(Z[0]))


def test_constant_field_projected():
    c = 0.8
    N = 20
    d = np.full((N, N), c)
    edges = linear_edges(6, 3)
    Z = oracle.zeta3_proj(d, edges, 6)
    counts = oracle.bin_counts((N, N), edges)
    assert rel(Z[0].real, N * N * c ** 3 * np.outer(counts, counts)) < 1e-13
    for m in (1, 2, 3, 5, 6):
        assert np.max(np.abs(Z[m])) < 1e-10 * np.max(np.abs(Z[0]))


def test_homogeneity_and_translation(rng):
    d = rng.standard_normal((8, 8, 8))
    edges = [0.0, 1.5, 3.0]
    Z = oracle.zeta3_full(d, edges, 3).real
    assert rel(oracle.zeta3_full(2.5 * d, edges, 3).real, 2.5 ** 3 * Z) < 1e-13
    assert rel(oracle.zeta3_full(np.roll(d, (1, 3, -2), axis=(0, 1, 2)), edges, 3).real, Z) < 1e-13
    lams, Z4 = oracle.zeta4_full(d, edges, 2)
    _, Z4b = oracle.zeta4_full(-1.5 * d, edges, 2)
    assert rel(Z4b.real, 1.5 ** 4 * Z4.real) < 1e-13


def cubic_symmetries():
    for perm in itertools.permutations(range(3)):
        for flips in itertools.product([False, True], repeat=3):
            yield perm, flips


def apply_sym(d, perm, flips):
    e = np.transpose(d, perm)
    for ax, f in enumerate(flips):
        if f:
            e = np.roll(np.flip(e, axis=ax), 1, axis=ax)  # x -> -x about cell 0
    return np.ascontiguousarray(e)


def test_full_invariance_under_cubic_group(rng):
    d = rng.standard_normal((8, 8, 8))
    edges = [0.0, 1.5, 3.0]
    Z3 = oracle.zeta3_full(d, edges, 4).real
    lams, Z4 = oracle.zeta4_full(d, edges, 2)
    for perm, flips in cubic_symmetries():
        e = apply_sym(d, perm, flips)
        assert rel(oracle.zeta3_full(e, edges, 4).real, Z3) < 1e-12
    for perm, flips in list(cubic_symmetries())[::7]:
        e = apply_sym(d, perm, flips)
        assert rel(oracle.zeta4_full(e, edges, 2)[1].real, Z4.real) < 1e-12


def test_projected_rotation_and_flip(rng):
    d = rng.standard_normal((12, 12))
    edges = [0.0, 1.5, 3.0]
    Z3 = oracle.zeta3_proj(d, edges, 5)
    pairs, Z4 = oracle.zeta4_proj(d, edges, 3)
    rot = np.ascontiguousarray(np.rot90(d))  # 90 degree rotation of the grid
    assert rel(oracle.zeta3_proj(rot, edges, 5), Z3) < 1e-12
    assert rel(oracle.zeta4_proj(rot, edges, 3)[1], Z4) < 1e-12
    flip = np.ascontiguousarray(np.roll(np.flip(d, axis=1), 1, axis=1))  # y -> -y
    assert rel(oracle.zeta3_proj(flip, edges, 5), np.conj(Z3)) < 1e-12
    assert rel(oracle.zeta4_proj(flip, edges, 3)[1], np.conj(Z4)) < 1e-12
    # Hermitian in (b1, b2), real diagonal
    assert rel(np.transpose(Z3, (0, 2, 1)), np.conj(Z3)) < 1e-12


def test_4pcf_with_l3_zero_is_weighted_3pcf(rng):
    """Lambda = (l, l, 0): the 3j sum collapses to (-1)^l / sqrt(2l+1) times a 3PCF-like
    sum with weight delta(x) a^b3_00(x) = delta(x) S^b3(x) / sqrt(4 pi)."""
    d = rng.standard_normal((8, 8, 8))
    d -= d.mean()
    edges = [0.0, 1.5, 3.0]
    lams, Z4 = oracle.zeta4_full(d, edges, 3)
    a = oracle.coeffs_full(d, edges, 3, cells=np.arange(d.size))
    dd = d.reshape(-1)
    for l in range(4):
        lam = (l, l, 0)
        got = Z4[lams.index(lam)].real
        exp = np.zeros_like(got)
        for b3 in range(2):
            w = dd * a[:, b3, 0]
            for m in range(-l, l + 1):
                j = l * l + m + l
                jm = l * l - m + l
                # a_{l,-m} enters the 3j sum; the closed form uses it directly
                exp[:, :, b3] += ((-1) ** (l - m) / math.sqrt(2 * l + 1) *
                                  np.einsum("x,xi,xj->ij", w, a[:, :, j], a[:, :, jm])).real
        assert rel(got, exp) < 1e-12


def test_coefficient_symmetry_negative_m(rng):
    """a_{l,-m} = (-1)^m conj(a_lm) and c_{-m} = conj(c_m) for a real field (eq. c_m def)."""
    d = rng.standard_normal((8, 8, 8))
    a = oracle.coeffs_full(d, [0.0, 2.0, 3.0], 3, cells=np.arange(0, 512, 7))
    for l in range(4):
        for m in range(1, l + 1):
            assert np.max(np.abs(a[:, :, l * l - m + l] - (-1) ** m * np.conj(a[:, :, l * l + m + l]))) < 1e-13
    d2 = rng.standard_normal((10, 10))
    c = oracle.coeffs_proj(d2, [0.0, 2.0, 3.0], 4, cells=np.arange(100))
    for m in range(1, 5):
        assert np.max(np.abs(c[:, :, 4 - m] - np.conj(c[:, :, 4 + m]))) < 1e-13


# ---------------------------------------------------------------- gradient

def test_grad3_central_differences_exact(rng):
    """The 3PCF sum is a cubic form without delta(y)^3 terms (r = 0 is in no bin), so central
    differences are exact up to rounding for any step h."""
    d = rng.standard_normal((6, 6, 6))
    edges = [0.0, 1.0, 2.0]
    lmax = 2
    G = rng.standard_normal((lmax + 1, 2, 2))
    g = oracle.grad3_full(d, edges, lmax, G)
    L = lambda f: float(np.sum(G * oracle.zeta3_full(f, edges, lmax).real))  # noqa: E731
    for y in [0, 17, 100, 215]:
        for h in (1e-3, 0.3):
            e = np.zeros(d.size)
            e[y] = h
            e = e.reshape(d.shape)
            fd = (L(d + e) - L(d - e)) / (2 * h)
            assert abs(fd - g.reshape(-1)[y]) < 1e-9 * max(1.0, abs(fd)), (y, h)


def test_grad3_box_truncated_kernel(rng):
    """24^3 with 8 bins out to r = 16 > N/2: kernels reach the box edge (offset set is the
    zero-centred cube); the gradient is still exact under central differences."""
    d = lognormal_field((12, 12, 12), seed=3, sigma=1.0, dtype=np.float64)
    edges = linear_edges(8, 4)
    lmax = 2
    G = rng.standard_normal((lmax + 1, 4, 4))
    g = oracle.grad3_full(d, edges, lmax, G)
    L = lambda f: float(np.sum(G * oracle.zeta3_full(f, edges, lmax).real))  # noqa: E731
    for y in [5, 901]:
        e = np.zeros(d.size)
        e[y] = 1e-3
        e = e.reshape(d.shape)
        fd = (L(d + e) - L(d - e)) / 2e-3
        assert abs(fd - g.reshape(-1)[y]) < 1e-8 * max(1.0, abs(fd))


def test_grad3_at_cells_matches_whole_field(rng):
    """The gradient evaluated at a subset of cells (coefficients only where needed) equals
    the whole-field gradient at those cells."""
    d = rng.standard_normal((8, 6, 10))
    edges = [0.0, 1.5, 2.5, 3.0]
    lmax = 3
    G = rng.standard_normal((lmax + 1, 3, 3))
    full = oracle.grad3_full(d, edges, lmax, G).reshape(-1)
    cells = np.array([0, 7, 61, 200, 479])
    sub = oracle.grad3_full(d, edges, lmax, G, cells=cells)
    assert np.allclose(sub, full[cells], rtol=1e-12, atol=1e-12 * np.max(np.abs(full)))


def test_grad3_fd_24_box_truncated():
    """The adjoint finite-difference case of the uneven-batch workload: 24^3 lognormal field,
    8 bins out to r = 16 (> N/2, kernels reach the box edge), lmax 4, central differences
    with h = 1e-3 at 16 random cells against the gradient at those cells."""
    d = lognormal_field((24, 24, 24), seed=24, sigma=1.0, dtype=np.float64)
    edges = linear_edges(16, 8)
    lmax = 4
    g_rng = np.random.Generator(np.random.PCG64(240))
    G = g_rng.standard_normal((lmax + 1, 8, 8))
    cells = np.sort(g_rng.choice(d.size, 16, replace=False))
    g = oracle.grad3_full(d, edges, lmax, G, cells=cells)
    L = lambda f: float(np.sum(G * oracle.zeta3_full(f, edges, lmax).real))  # noqa: E731
    h = 1e-3
    for y, gy in zip(cells, g):
        e = np.zeros(d.size)
        e[y] = h
        e = e.reshape(d.shape)
        fd = (L(d + e) - L(d - e)) / (2 * h)
        assert abs(fd - gy) < 1e-7 * max(1.0, np.max(np.abs(g))), (y, fd, gy)


# ---------------------------------------------------------------- normalization (Sec. 2.5)

def test_normalization_constant_field_closed_form():
    """delta = c everywhere: the l = 0 sums are N_g c^3 n_b1 n_b2 / (4 pi) (counts n_b), the N
    of Sec. 2.5 is N_g (1 + c) ((1 + c) n_b1) ((1 + c) n_b2), so the normalized l = 0 3PCF is
    c^3 / (4 pi (1 + c)^3) for every bin pair."""
    c = 0.7
    d = np.full((10, 10, 10), c)
    edges = [0.0, 1.0, 2.0, 3.5]
    z = oracle.zeta3_full(d, edges, 1).real
    N = oracle.normalization(d, edges, 3)
    assert np.allclose(z[0] / N, c ** 3 / (4 * np.pi * (1 + c) ** 3), rtol=1e-12)
    # the 4PCF with Lambda = (0, 0, 0): 3j = 1, sums N_g c^4 n n n / (4 pi)^(3/2) over
    # N = N_g (1 + c)^4 n n n
    lams, z4 = oracle.zeta4_full(d, edges, 0)
    N4 = oracle.normalization(d, edges, 4)
    assert np.allclose(z4[0].real / N4, c ** 4 / ((4 * np.pi) ** 1.5 * (1 + c) ** 4), rtol=1e-12)



def test_correlation_core_equals_the_cell_by_cell_loop():
    """The C core's correlation visits cells in blocks of 512 and offsets in runs of at most 64
    of one bin, cells outermost within a run (a loop interchange only).  Against the plain
    definition a^b_j(x) = sum_{r in b} B_j(r) delta(x + r), each product and sum rounded in
    float64 in offset order, written here cell by cell in numpy: bit-identical, on a grid of
    several cell blocks with bins of several offset runs, and at an unordered cell list."""
    from oracle import api as oapi
    rng = np.random.Generator(np.random.PCG64(2024))
    shape = (12, 10, 14)                                     # 1680 cells: blocks of 512, 512, 512, 144
    d = rng.standard_normal(shape)
    edges = np.array([0.0, 1.5, 2.6, 4.0])                   # 32, 82 and 194 offsets: runs of 64
    off, bins, counts = oapi.support(shape, edges)
    assert counts.max() > 128
    B = oapi.basis_full(off, 2)
    ref = np.zeros((d.size, 3, B.shape[1]), dtype=np.complex128)
    coords = np.stack(np.unravel_index(np.arange(d.size), shape), axis=1)
    for o in range(off.shape[0]):   # offsets in table order; the same running totals for every cell
        nbr = np.ravel_multi_index(((coords + off[o]) % np.array(shape)).T, shape)
        v = d.reshape(-1)[nbr]
        b = bins[o]
        ref[:, b, :].real = ref[:, b, :].real + B[o].real[None, :] * v[:, None]
        ref[:, b, :].imag = ref[:, b, :].imag + B[o].imag[None, :] * v[:, None]
    got = oapi.coeffs_full(d, edges, 2)
    assert np.array_equal(got.real, ref.real) and np.array_equal(got.imag, ref.imag)
    cells = rng.permutation(d.size)[:700]
    got_c = oapi.coeffs_full(d, edges, 2, cells=cells)
    assert np.array_equal(got_c, ref[cells])


def test_grid_sum_accumulation_error_is_negligible():
    """The oracle adds per-cell contributions in float64, sequentially within each thread's
    cell range, then the thread totals in order.  Against an exactly rounded sum (math.fsum)
    of the per-cell contributions, the difference stays at the float64 level, far below the
    1e-5 parity bound."""
    import math
    from oracle import api as oapi
    d = lognormal_field((16, 16, 16), seed=77, sigma=1.0, dtype=np.float64)
    edges = np.array([0.0, 2.0, 4.0])
    z = oracle.zeta3_full(d, edges, 2, nthreads=3).real
    a = oapi.coeffs_full(d, edges, 2)                       # (cells, bins, (lmax+1)^2), bit-exact per cell
    exact = np.zeros_like(z)
    for l in range(3):
        cols = slice(l * l, (l + 1) ** 2)
        for b1 in range(2):
            for b2 in range(2):
                terms = d.reshape(-1) * np.sum(a[:, b1, cols] * np.conj(a[:, b2, cols]), axis=1).real
                exact[l, b1, b2] = math.fsum(terms)
    scale = np.max(np.abs(exact))
    assert np.max(np.abs(z - exact)) <= 1e-12 * scale


def test_kernels_have_parity_under_inversion():
    """The binned kernels conj(Y_lm(r^)) on the support of a bin change by (-1)^l under r -> -r,
    and the support of every bin is symmetric, when 2 r0 stays below every edge: the identity
    the half kernel store uses to take the planes c_0 < 0 from c_0 > 0.  At an edge of 2 r0 the
    zero-centred offsets of that axis lose the symmetry (-r0 is kept, +r0 folds onto it), which
    is why plans keep every plane there."""
    from oracle.api import basis_full
    lmax = 4
    off, bins, _ = support((16, 20, 18), linear_edges(6, 3))   # r0 = 6, 2 r0 = 12 < every edge
    key = {tuple(o): b for o, b in zip(off.tolist(), bins.tolist())}
    neg = -off
    assert all(key.get(tuple(o)) == b for o, b in zip(neg.tolist(), bins.tolist()))
    B, Bn = basis_full(off, lmax), basis_full(neg, lmax)
    for l in range(lmax + 1):
        cols = slice(l * l, (l + 1) ** 2)
        np.testing.assert_allclose(Bn[:, cols], (-1) ** l * B[:, cols], rtol=0, atol=1e-13)
    off12, _, _ = support((12, 20, 18), linear_edges(6, 3))  # an edge of exactly 2 r0
    keys12 = {tuple(o) for o in off12.tolist()}
    assert any(tuple(-o) not in keys12 for o in off12)
