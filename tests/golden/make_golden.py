"""Write the oracle's expected values for the workloads too large to recompute in a test.

Calls only the FP64 oracle (``oracle/``) and the seeded field generator
(``fieldgen``).  Usage:  python tests/golden/make_golden.py {c2,c3,c4,c5} [--threads N]

  c2  512^2 projected field, 10 bins to 40, m up to 10: projected 3PCF and 4PCF sums
  c3  the two 256^3 full-3PCF fields (sigma 0.5 seed 0, sigma 1.5 seed 1),
      10 bins to 32 (edges 3.2 b), lmax 6                      (about an hour per field)
  c4  fields 0 and 1 of the 16-field 128^3 batch, 8 bins to 24, even Lambda, lmax 4
  c5  one field of each grid edge of the uneven 48-field batch, 8 bins to 16, lmax 4
  c5g the same fields: gradient of sum G Z (G seeded normal) at 32 seeded cells each
  c5x a sixth field of the uneven batch: the second field of edge 64
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from fieldgen import lognormal_field, linear_edges, c4_batch, c5_shapes  # noqa: E402


def _save(name, **arrays):
    path = os.path.join(HERE, name)
    np.savez(path, **arrays)
    print("wrote", path, flush=True)


def make_c2(nt):
    d = lognormal_field((512, 512), seed=0, sigma=1.0)
    edges = linear_edges(40, 10)
    t = time.time()
    z3 = oracle.zeta3_proj(d.astype(np.float64), edges, 10, nthreads=nt)
    pairs, z4 = oracle.zeta4_proj(d.astype(np.float64), edges, 10, nthreads=nt)
    _save("c2_proj_512.npz", zeta3=z3, zeta4=z4, pairs=np.array(pairs), edges=edges,
          seconds=time.time() - t)


def make_c3(nt, seeds=(0, 1)):
    sig = {0: 0.5, 1: 1.5}
    for s in seeds:
        d = lognormal_field((256, 256, 256), seed=s, sigma=sig[s])
        edges = linear_edges(32, 10)
        t = time.time()
        z = oracle.zeta3_full(d.astype(np.float64), edges, 6, nthreads=nt)
        _save(f"c3_full3_256_seed{s}.npz", zeta3=z, edges=edges, sigma=sig[s], seconds=time.time() - t)


def make_c4(nt, fields=(0, 1)):
    n = 128
    aux = np.random.Generator(np.random.PCG64(10 ** 6))
    sigmas = aux.uniform(0.5, 2.0, size=16)
    for i in fields:
        d = lognormal_field((n, n, n), seed=i, sigma=float(sigmas[i]))
        edges = linear_edges(24, 8)
        t = time.time()
        lams, z = oracle.zeta4_full(d.astype(np.float64), edges, 4, nthreads=nt)
        _save(f"c4_full4_128_field{i}.npz", zeta4=z, lams=np.array(lams), edges=edges,
              sigma=sigmas[i], seconds=time.time() - t)


def make_c5(nt):
    edges_list = c5_shapes()
    seen = {}
    for i, n in enumerate(edges_list):
        if n not in seen:
            seen[n] = i
    for n, i in sorted(seen.items()):
        d = lognormal_field((n, n, n), seed=i, sigma=1.0)
        edges = linear_edges(16, 8)
        t = time.time()
        z = oracle.zeta3_full(d.astype(np.float64), edges, 4, nthreads=nt)
        _save(f"c5_full3_{n}_field{i}.npz", zeta3=z, edges=edges, field=i, seconds=time.time() - t)


def make_c5g(nt):
    edges_list = c5_shapes()
    seen = {}
    for i, n in enumerate(edges_list):
        if n not in seen:
            seen[n] = i
    for n, i in sorted(seen.items()):
        d = lognormal_field((n, n, n), seed=i, sigma=1.0)
        edges = linear_edges(16, 8)
        rng = np.random.Generator(np.random.PCG64(5500 + i))
        G = rng.standard_normal((5, 8, 8))
        cells = np.sort(rng.choice(d.size, 32, replace=False))
        t = time.time()
        g = oracle.grad3_full(d.astype(np.float64), edges, 4, G, cells=cells, nthreads=nt)
        _save(f"c5_grad3_{n}_field{i}.npz", grad=g, cells=cells, G=G, edges=edges, field=i,
              seconds=time.time() - t)


def c5_extra_field():
    """(edge, index) of the sixth checked field of the uneven batch: the second one of edge 64."""
    idx = [i for i, n in enumerate(c5_shapes()) if n == 64]
    return 64, idx[1]


def make_c5x(nt):
    n, i = c5_extra_field()
    d = lognormal_field((n, n, n), seed=i, sigma=1.0)
    edges = linear_edges(16, 8)
    t = time.time()
    z = oracle.zeta3_full(d.astype(np.float64), edges, 4, nthreads=nt)
    _save(f"c5_full3_{n}_field{i}.npz", zeta3=z, edges=edges, field=i, seconds=time.time() - t)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["c2", "c3", "c4", "c5", "c5g", "c5x"])
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--seeds", type=int, nargs="*", default=None)
    a = ap.parse_args()
    if a.what == "c3":
        make_c3(a.threads, tuple(a.seeds) if a.seeds else (0, 1))
    else:
        {"c2": make_c2, "c4": make_c4, "c5": make_c5, "c5g": make_c5g, "c5x": make_c5x}[a.what](a.threads)
