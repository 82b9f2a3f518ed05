"""Error measures of the parity tests (no GPU code; imported by the GPU test modules).

The error of a result against the FP64 oracle is max |Z_gpu - Z_oracle| / max |Z_oracle|,
taken over the whole result and over every block of its leading index (per l, per Lambda,
per m, per (m1, m2)), each block relative to its own max |Z_oracle|.  Both must stay within
the bound: 1e-5 for the float32 path, 3e-4 for split-BF16.
"""
import numpy as np

TOL32 = 1e-5
TOL_SPLIT = 3e-4


def rel_err(got, ref):
    got, ref = np.asarray(got), np.asarray(ref)
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def block_errs(got, ref):
    """Per-block errors along the leading axis, each relative to that block's max |ref|."""
    got, ref = np.asarray(got), np.asarray(ref)
    out = []
    for i in range(ref.shape[0]):
        m = float(np.max(np.abs(ref[i])))
        out.append(float(np.max(np.abs(got[i] - ref[i]))) / m if m > 0 else float(np.max(np.abs(got[i]))))
    return out


def worst_block(got, ref):
    return max(block_errs(got, ref))


def check(got, ref, tol, say=print, label=""):
    """Assert the whole-result and the per-block error within tol; returns (err, worst block)."""
    e, wb = rel_err(got, ref), worst_block(got, ref)
    say(f"  {label}err={e:.3e} worst block={wb:.3e} (bound {tol:g})")
    assert e < tol, f"{label}whole-result error {e:.3e} >= {tol:g}"
    assert wb < tol, f"{label}worst block error {wb:.3e} >= {tol:g}"
    return e, wb
