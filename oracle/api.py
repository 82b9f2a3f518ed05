"""Python side of the FP64 oracle: supports, bases, term tables, C-core wrappers.

Test infrastructure only (see the package docstring).

Conventions (each one a reading of the paper, listed with its reason in the
repository's design notes):

* Grid coordinates are zero-centred, c(i) = i for 2i < N and i - N otherwise
  (the "coordinates centered on zero" of the notes to Alg. 1 and Alg. 2).
* Offset r lies in bin b iff e_b < |r| <= e_{b+1} (the mask of Alg. 1 and
  Alg. 2), decided exactly on the given float64 edges; r = 0 is in no bin.
* 3D axes (x, y, z) = (array axis 0, 1, 2); Y_lm is orthonormal with the
  Condon-Shortley phase; the 3D basis is conj(Y_lm(r^)) (eq. almconv).
* 2D axes (x, y) = (array axis 0, 1), phi = atan2(y, x); the basis is
  e^{-i m phi} (eqs. c_m def and the kernel K^b_m of Sec. 2.2).
* a and c are correlations, delta(x + r) (eq. almconv and its footnote).
"""
from __future__ import annotations

import ctypes
import os
from fractions import Fraction

import numpy as np
from scipy.special import sph_harm_y

from .threej import threej

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        # SB_ORACLE_LIB names another build of the same core (the sanitizer build of
        # build.build(sanitize=True)); the default one is compiled on first use.
        path = os.environ.get("SB_ORACLE_LIB") or os.path.join(_HERE, "_liboracle.so")
        if not os.path.exists(path):
            if "SB_ORACLE_LIB" in os.environ:
                raise FileNotFoundError(path)
            from .build import build
            build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int, ctypes.c_int64
        lib.oc_coeffs.argtypes = [i32, P, P, i64, P, P, i32, i32, P, i64, P, P, i32]
        lib.oc_coeffs.restype = i32
        lib.oc_zeta.argtypes = [i32, P, P, i64, P, P, i32, i32, P, i32, i32, P, P, P, i64, P, P, i32]
        lib.oc_zeta.restype = i32
        lib.oc_grad3.argtypes = [i32, P, P, i64, P, P, i32, i32, P, i32, P, P, P, P, P, i64, P, P, i32]
        lib.oc_grad3.restype = i32
        lib.oc_max_threads.restype = i32
        _LIB = lib
    return _LIB


def max_threads() -> int:
    return int(_lib().oc_max_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Support of the radial bins (mask of Alg. 1 / Alg. 2)
# --------------------------------------------------------------------------

def _centred(n: int) -> np.ndarray:
    return np.array([i if 2 * i < n else i - n for i in range(n)], dtype=np.int64)


def support(shape, edges):
    """Offsets of every radial bin.

    Returns (off, bins, counts): off is an (n_off, ndim) int32 array of offsets
    r, bins the bin index of each (sorted by bin, then lexicographically), and
    counts the number of offsets per bin.  Bin b holds e_b < |r| <= e_{b+1},
    decided by comparing the integer |r|^2 with the exact rational square of
    each float64 edge."""
    shape = tuple(int(s) for s in shape)
    edges = [float(e) for e in edges]
    nb = len(edges) - 1
    e2 = [Fraction(e) ** 2 for e in edges]
    emax = max(edges)
    axes = []
    for n in shape:
        c = _centred(n)
        axes.append(c[np.abs(c) <= int(np.floor(emax))])
    grids = np.meshgrid(*axes, indexing="ij")
    off = np.stack([g.ravel() for g in grids], axis=1)
    r2 = np.sum(off * off, axis=1)
    binmap = {}
    for v in np.unique(r2):
        v = int(v)
        b_of = -1
        for b in range(nb):
            if e2[b] < v <= e2[b + 1]:
                b_of = b
                break
        binmap[v] = b_of
    bins = np.array([binmap[int(v)] for v in r2], dtype=np.int64)
    keep = (bins >= 0) & (r2 > 0)
    off, bins = off[keep], bins[keep]
    order = np.lexsort(tuple(off[:, d] for d in reversed(range(off.shape[1]))) + (bins,))
    off, bins = off[order], bins[order]
    counts = np.bincount(bins, minlength=nb)
    return (np.ascontiguousarray(off.astype(np.int32)), np.ascontiguousarray(bins.astype(np.int32)),
            counts.astype(np.int64))


def bin_counts(shape, edges) -> np.ndarray:
    """Number of grid offsets in each bin (the N_cells in bin of eqn radial_binning)."""
    return support(shape, edges)[2]


# --------------------------------------------------------------------------
# Bases
# --------------------------------------------------------------------------

def _full_index(l: int, m: int) -> int:
    return l * l + (m + l)


def basis_full(off: np.ndarray, lmax: int) -> np.ndarray:
    """conj(Y_lm(r^)) for l = 0..lmax, m = -l..l at every offset: (n_off, (lmax+1)^2).

    Column l*l + (m + l).  Y_lm from scipy.special.sph_harm_y (polar angle
    first), which includes the Condon-Shortley phase."""
    x, y, z = (off[:, d].astype(np.float64) for d in range(3))
    r = np.sqrt(x * x + y * y + z * z)
    theta = np.arccos(np.clip(z / r, -1.0, 1.0))
    phi = np.arctan2(y, x)
    out = np.empty((off.shape[0], (lmax + 1) ** 2), dtype=np.complex128)
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            out[:, _full_index(l, m)] = np.conj(sph_harm_y(l, m, theta, phi))
    return out


def basis_proj(off: np.ndarray, mmax: int) -> np.ndarray:
    """e^{-i m phi} for m = -mmax..mmax at every offset: (n_off, 2 mmax + 1), column m + mmax."""
    phi = np.arctan2(off[:, 1].astype(np.float64), off[:, 0].astype(np.float64))
    out = np.empty((off.shape[0], 2 * mmax + 1), dtype=np.complex128)
    for m in range(-mmax, mmax + 1):
        out[:, m + mmax] = np.exp(-1j * m * phi)
    return out


# --------------------------------------------------------------------------
# Term tables
# --------------------------------------------------------------------------

def lambdas(lmax: int, parity: str = "even"):
    """Lambda = (l1, l2, l3) in the loop order of Alg. 6: l1 and l2 over 0..lmax,
    l3 from |l1 - l2| to min(l1 + l2, lmax).  parity selects even, odd or both sums."""
    out = []
    for l1 in range(lmax + 1):
        for l2 in range(lmax + 1):
            for l3 in range(abs(l1 - l2), min(l1 + l2, lmax) + 1):
                odd = (l1 + l2 + l3) % 2 == 1
                if parity == "even" and odd:
                    continue
                if parity == "odd" and not odd:
                    continue
                out.append((l1, l2, l3))
    return out


def mpairs(mmax: int):
    """(m1, m2) pairs of the projected 4PCF: m1 outer over -mmax..mmax, m2 inner,
    kept when |m1 + m2| <= mmax (m3 = -(m1 + m2), eq. proj_4pcf_coeff)."""
    return [(m1, m2) for m1 in range(-mmax, mmax + 1) for m2 in range(-mmax, mmax + 1)
            if abs(m1 + m2) <= mmax]


def _terms_full4(lmax: int, parity: str):
    lams = lambdas(lmax, parity)
    ptr, js, ws = [0], [], []
    for (l1, l2, l3) in lams:
        for m1 in range(-l1, l1 + 1):
            for m2 in range(-l2, l2 + 1):
                m3 = -(m1 + m2)
                if abs(m3) > l3:
                    continue
                w = threej(l1, l2, l3, m1, m2, m3)
                if w == 0.0:
                    continue
                js.append((_full_index(l1, m1), _full_index(l2, m2), _full_index(l3, m3)))
                ws.append(w)
        ptr.append(len(ws))
    return lams, np.array(ptr, np.int32), np.array(js, np.int32).reshape(-1, 3), np.array(ws, np.float64)


# --------------------------------------------------------------------------
# C-core wrappers
# --------------------------------------------------------------------------

def _prep(delta, edges):
    d = np.ascontiguousarray(np.asarray(delta, dtype=np.float64))
    shape = np.array(d.shape, dtype=np.int64)
    off, bins, counts = support(d.shape, edges)
    return d, shape, off, bins, counts


def _cells(cells):
    if cells is None:
        return 0, None
    c = np.ascontiguousarray(np.asarray(cells, dtype=np.int64).ravel())
    return c.size, c


def _coeffs(d, shape, off, bins, nb, basis, cells, nthreads):
    ncell, c = _cells(cells)
    if c is None:
        c = np.arange(d.size, dtype=np.int64)
        ncell = d.size
    B = np.ascontiguousarray(basis.astype(np.complex128))
    out = np.zeros((ncell, nb, B.shape[1]), dtype=np.complex128)
    _lib().oc_coeffs(d.ndim, _ptr(shape), _ptr(d), off.shape[0], _ptr(off), _ptr(bins), nb,
                     B.shape[1], _ptr(B), ncell, _ptr(c), _ptr(out), int(nthreads))
    return out


def coeffs_full(delta, edges, lmax, cells=None, nthreads=0):
    """a^b_lm(x) (eq. almconv, unnormalised mask) at the given flat cell indices:
    (ncells, nbins, (lmax+1)^2), column l*l + m + l."""
    d, shape, off, bins, _ = _prep(delta, edges)
    return _coeffs(d, shape, off, bins, len(edges) - 1, basis_full(off, lmax), cells, nthreads)


def coeffs_proj(delta, edges, mmax, cells=None, nthreads=0):
    """c^b_m(x) (eqs. c_m def, discretize_cmb, unnormalised mask): (ncells, nbins, 2 mmax + 1), column m + mmax."""
    d, shape, off, bins, _ = _prep(delta, edges)
    return _coeffs(d, shape, off, bins, len(edges) - 1, basis_proj(off, mmax), cells, nthreads)


def _zeta(d, shape, off, bins, nb, basis, mode, ptr, js, ws, cells, nthreads):
    ncell, c = _cells(cells)
    B = np.ascontiguousarray(basis.astype(np.complex128))
    ng = len(ptr) - 1
    per = nb * nb if mode == 3 else nb * nb * nb
    out = np.zeros(ng * per, dtype=np.complex128)
    js = np.ascontiguousarray(js.astype(np.int32).ravel())
    ws = np.ascontiguousarray(np.asarray(ws, np.float64)) if ws is not None else np.zeros(1)
    rc = _lib().oc_zeta(d.ndim, _ptr(shape), _ptr(d), off.shape[0], _ptr(off), _ptr(bins), nb,
                        B.shape[1], _ptr(B), mode, ng, _ptr(ptr), _ptr(js), _ptr(ws),
                        ncell, _ptr(c) if c is not None else None, _ptr(out), int(nthreads))
    if rc != 0:
        raise MemoryError("oracle contraction failed")
    return out.reshape((ng,) + (nb,) * (2 if mode == 3 else 3))


def zeta3_full(delta, edges, lmax, cells=None, nthreads=0):
    """Full 3PCF sums Z[l, b1, b2] = sum_x delta sum_{m=-l..l} a^b1_lm conj(a^b2_lm).

    This is the grid sum of Alg. 5 (eq. alm_to_zeta_clean without the
    (-1)^l / sqrt(2l+1) prefactor) over all m instead of m >= 0 with S += S*.
    Complex output: the imaginary part is zero up to rounding."""
    d, shape, off, bins, _ = _prep(delta, edges)
    ptr = np.array([l * l for l in range(lmax + 2)], np.int32)
    js = np.arange((lmax + 1) ** 2, dtype=np.int32)
    return _zeta(d, shape, off, bins, len(edges) - 1, basis_full(off, lmax), 3, ptr, js, None,
                 cells, nthreads)


def zeta3_proj(delta, edges, mmax, cells=None, nthreads=0):
    """Projected 3PCF sums Z[m, b1, b2] = sum_x delta c^b1_m conj(c^b2_m), m = 0..mmax
    (the grid sum of Alg. 7 over all ordered bin pairs)."""
    d, shape, off, bins, _ = _prep(delta, edges)
    ptr = np.arange(mmax + 2, dtype=np.int32)
    js = np.array([m + mmax for m in range(mmax + 1)], np.int32)
    return _zeta(d, shape, off, bins, len(edges) - 1, basis_proj(off, mmax), 3, ptr, js, None,
                 cells, nthreads)


def zeta4_full(delta, edges, lmax, parity="even", cells=None, nthreads=0):
    """Full 4PCF sums Z[Lambda, b1, b2, b3] = sum_x delta sum_M 3j(Lambda; M) a^b1 a^b2 a^b3.

    E(Lambda) C^Lambda_M equals the plain 3j for both parities (Sec. 2.3), and the
    sum runs over every (m1, m2) with |m1 + m2| <= l3: the full form that Alg. 6
    halves with m3 >= 0 and the 2 S(m3) Re[...] weighting.  Returns (lams, Z)."""
    d, shape, off, bins, _ = _prep(delta, edges)
    lams, ptr, js, ws = _terms_full4(lmax, parity)
    Z = _zeta(d, shape, off, bins, len(edges) - 1, basis_full(off, lmax), 4, ptr, js, ws,
              cells, nthreads)
    return lams, Z


def zeta4_proj(delta, edges, mmax, cells=None, nthreads=0):
    """Projected 4PCF sums Z[p, b1, b2, b3] = sum_x delta c^b1_m1 c^b2_m2 c^b3_m3, m3 = -(m1 + m2),
    (m1, m2) = mpairs(mmax)[p] (eq. proj_4pcf_coeff, all ordered bin triples).
    c for negative m is the direct sum with e^{-i m phi}.  Returns (pairs, Z)."""
    d, shape, off, bins, _ = _prep(delta, edges)
    pairs = mpairs(mmax)
    ptr = np.arange(len(pairs) + 1, dtype=np.int32)
    js = np.array([(m1 + mmax, m2 + mmax, -(m1 + m2) + mmax) for (m1, m2) in pairs], np.int32)
    ws = np.ones(len(pairs))
    Z = _zeta(d, shape, off, bins, len(edges) - 1, basis_proj(off, mmax), 4, ptr, js, ws,
              cells, nthreads)
    return pairs, Z


def grad3_full(delta, edges, lmax, G, cells=None, nthreads=0):
    """d/d delta(y) of L = sum_{l,b1,b2} G[l,b1,b2] Z[l,b1,b2] for the full 3PCF sums.

    Derivative of the trilinear sum of zeta3_full: the direct term
    sum G a^b1 conj(a^b2) at y plus, for every neighbour x = y - r, the terms
    through d a^b(x) / d delta(y) = conj(Y_lm(r^)) for r in bin b.  Returns the
    real gradient (the imaginary part is rounding noise and is dropped after a check):
    the whole field, or the values at the flat cell indices `cells` (then the coefficients
    are evaluated only at those cells and their neighbours y - r)."""
    d, shape, off, bins, _ = _prep(delta, edges)
    nb = len(edges) - 1
    B = basis_full(off, lmax)
    if cells is None:
        ys, amap = None, None
        a_all = np.ascontiguousarray(_coeffs(d, shape, off, bins, nb, B, None, nthreads))
        ny = d.size
    else:
        ys = np.ascontiguousarray(np.asarray(cells, dtype=np.int64).ravel())
        ny = ys.size
        # every x = y - r (and y itself), as flat indices
        coords = np.stack(np.unravel_index(ys, d.shape), axis=1)
        nbr = (coords[:, None, :] - off[None, :, :]) % np.array(d.shape)
        need = np.unique(np.concatenate([ys, np.ravel_multi_index(nbr.reshape(-1, d.ndim).T, d.shape)]))
        amap = np.full(d.size, -1, dtype=np.int64)
        amap[need] = np.arange(need.size, dtype=np.int64)
        a_all = np.ascontiguousarray(_coeffs(d, shape, off, bins, nb, B, need, nthreads))
    ptr = np.array([l * l for l in range(lmax + 2)], np.int32)
    js = np.arange((lmax + 1) ** 2, dtype=np.int32)
    Gd = np.ascontiguousarray(np.asarray(G, np.float64).reshape(lmax + 1, nb, nb))
    out = np.zeros(ny, dtype=np.complex128)
    Bc = np.ascontiguousarray(B)
    _lib().oc_grad3(d.ndim, _ptr(shape), _ptr(d), off.shape[0], _ptr(off), _ptr(bins), nb,
                    B.shape[1], _ptr(Bc), lmax + 1, _ptr(ptr), _ptr(js), _ptr(Gd), _ptr(a_all),
                    None if amap is None else _ptr(amap), int(ny), None if ys is None else _ptr(ys),
                    _ptr(out), int(nthreads))
    scale = max(1.0, float(np.max(np.abs(out.real))))
    if np.max(np.abs(out.imag)) > 1e-9 * scale:
        raise AssertionError("oracle gradient has a non-negligible imaginary part")
    return out.real.reshape(d.shape) if cells is None else out.real


def normalization(delta, edges, npcf):
    """The N of Sec. 2.5 with unit cells (box side = grid resolution, the paper's validation
    set-up): N = N_gal prod_{n=1}^{N-1} (nbar V_bin,n), N_gal = sum over cells of (delta + 1),
    nbar = N_gal / N_g, V_bin = number of cells in the bin (cell volume or area 1).  Returned
    with the broadcast shape of the bin axes of the result: (nb, nb) for npcf 3, (nb, nb, nb)
    for npcf 4; the raw sums divided by it are the normalized coefficients."""
    d = np.asarray(delta, dtype=np.float64)
    ngal = float(np.sum(d + 1.0))
    nbar = ngal / d.size
    v = nbar * bin_counts(d.shape, edges).astype(np.float64)
    if npcf == 3:
        return ngal * np.multiply.outer(v, v)
    return ngal * np.multiply.outer(np.multiply.outer(v, v), v)

