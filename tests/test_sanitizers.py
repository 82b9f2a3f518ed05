"""Host-side AddressSanitizer and UndefinedBehaviorSanitizer runs (CPU only).

* The oracle's C core, built by gcc with -fsanitize=address,undefined, runs the oracle pins that
  reach it (coefficients, the 3PCF and 4PCF sums, the adjoint of the 3PCF).
* The host half of the HIP library (plan creation, bin and index tables, scratch layouts,
  argument validation and the status strings), built with the same checks on its host code
  (device code unchanged, build.build(sanitize=True)), runs the CPU ABI tests and the plan sweep
  below.

Each run is a child process with the sanitizer runtime preloaded; a finding aborts it with a
nonzero status and the sanitizer's report.  Leak checking is off: the Python interpreter keeps
its own allocations to the end.
"""
import ctypes
import glob
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=99",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _child(env_extra, args, timeout=900):
    env = dict(os.environ)
    env.update(SAN_ENV)
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider", *args],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    return out


def _sources_newer_than(path, roots):
    if not os.path.exists(path):
        return True
    t = os.path.getmtime(path)
    for root in roots:
        for f in glob.glob(os.path.join(root, "*")):
            if os.path.getmtime(f) > t:
                return True
    return False


def test_oracle_core_under_asan_and_ubsan(tmp_path):
    from oracle.build import build
    lib = build(sanitize=True, out=str(tmp_path / "liboracle_san.so"))
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()
    # the finite-difference gradient case on 24^3 is left out: it only repeats the calls of the
    # small gradient case, ten times slower under the checks
    out = _child({"SB_ORACLE_LIB": lib, "LD_PRELOAD": asan},
                 [os.path.join("tests", "test_oracle_pins.py"), "-k", "not grad3_fd_24"])
    assert " passed" in out


def _sanitized_hip_library():
    from paper_2210_10206_amd import build as hipbuild
    out = os.path.join(hipbuild.HERE, "_build_sanitize", "libsarabande_hip.so")
    if _sources_newer_than(out, [hipbuild.CSRC, hipbuild.INCLUDE]):
        out = hipbuild.build(jobs=min(8, os.cpu_count() or 1), sanitize=True)
    return out


def _clang_asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        pytest.skip("clang AddressSanitizer runtime not found under /opt/rocm/llvm")
    return found[-1]


def test_plan_host_code_under_asan_and_ubsan():
    lib = _sanitized_hip_library()
    rt = _clang_asan_runtime()
    out = _child({"SB_LIB_PATH": lib, "LD_PRELOAD": rt},
                 [os.path.join("tests", "test_abi.py"),
                  os.path.join("tests", "test_sanitizers.py") + "::test_host_plan_sweep"])
    assert " passed" in out


def _problem(lib_mod, ndim, npcf, edges, lmax, prec=0, dtype=0, flags=0):
    e = np.ascontiguousarray(edges, dtype=np.float64)
    p = lib_mod.SbProblem(ndim, npcf, len(e) - 1, e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), lmax, prec,
                          dtype, flags)
    return p, e


def test_host_plan_sweep():
    """Every host-side query over a sweep of plan shapes: the kinds of correlation, lmax and bin
    counts to their limits, uneven batches, the path flags, the regenerated-kernel and 1024
    plans, field batching and scratch limits.  Run plainly in the CPU suite and under the
    sanitizers by test_plan_host_code_under_asan_and_ubsan."""
    from paper_2210_10206_amd import _lib
    lib = _lib.load()
    i32, i64, sz, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_uint32
    for s in range(-8, 2):
        assert lib.sb_status_str(s)
    for n in range(0, 1030):
        lib.sb_fft_variants(n)
    cases = []
    for ndim in (2, 3):
        for npcf in (3, 4):
            lmaxes = (0, 1, 4, 10) if ndim == 3 else (0, 3, 16)
            for lmax in lmaxes:
                for nb in (1, 3, 8, 16):
                    if npcf == 4 and (nb > 10 or (ndim == 3 and lmax > 6)):
                        continue
                    for flags in ((0, 1, 2, 4, 16, 32, 128) if npcf == 3 else (0, 4, 8, 32, 128)):
                        if flags == 8 and ndim == 2:
                            continue
                        cases.append((ndim, npcf, lmax, nb, flags))
    shapes3 = [[(32, 32, 32)], [(16, 24, 32), (32, 32, 32), (16, 24, 32), (48, 40, 36)], [(64, 64, 64)] * 3]
    shapes2 = [[(64, 64)], [(32, 48), (64, 64), (32, 48)]]
    made = 0
    for ndim, npcf, lmax, nb, flags in cases:
        edges = np.linspace(0.5, 7.5, nb + 1)
        prob, e = _problem(_lib, ndim, npcf, edges, lmax, flags=flags)
        for shapes in (shapes3 if ndim == 3 else shapes2):
            sh = np.ascontiguousarray(np.array(shapes, dtype=np.int64).ravel())
            h = ctypes.c_void_p()
            rc = lib.sb_plan_create(ctypes.byref(prob), len(shapes), sh.ctypes.data_as(ctypes.POINTER(i64)),
                                    ctypes.byref(h))
            if rc != 0:
                assert not h.value and lib.sb_last_error()
                continue
            made += 1
            pb, sb = sz(), sz()
            assert lib.sb_plan_workspace(h, ctypes.byref(pb), ctypes.byref(sb)) == 0
            nz = np.zeros(len(shapes), dtype=np.int64)
            assert lib.sb_zeta_size(h, nz.ctypes.data_as(ctypes.POINTER(i64))) == 0
            rows, cols, tab = i32(), i32(), ctypes.POINTER(i32)()
            assert lib.sb_zeta_index(h, ctypes.byref(rows), ctypes.byref(cols), ctypes.byref(tab)) == 0
            if rows.value:
                assert sum(tab[k] for k in range(rows.value * cols.value)) >= 0
            for f in range(len(shapes)):
                cnt = np.zeros(nb, dtype=np.int64)
                assert lib.sb_bin_counts(h, f, cnt.ctypes.data_as(ctypes.POINTER(i64))) == 0
            assert lib.sb_bin_counts(h, len(shapes), None) != 0
            w = u32()
            assert lib.sb_plan_warnings(h, ctypes.byref(w)) == 0
            for fb in (1, 2, 64):
                lib.sb_plan_set_field_batch(h, fb)
                got = i32()
                assert lib.sb_plan_get_field_batch(h, ctypes.byref(got)) == 0
                assert lib.sb_plan_workspace(h, ctypes.byref(pb), ctypes.byref(sb)) == 0
            lib.sb_plan_set_scratch_limit(h, 1 << 20)
            lib.sb_plan_workspace(h, ctypes.byref(pb), ctypes.byref(sb))
            lib.sb_plan_set_scratch_limit(h, 0)
            t1, t2, t3 = i32(), i32(), i32()
            lib.sb_plan_get_contract_tile(h, ctypes.byref(t1), ctypes.byref(t2), ctypes.byref(t3))
            lib.sb_plan_set_contract_tile(h, 64)
            v = i32()
            lib.sb_plan_get_fft_variant(h, 0, 0, ctypes.byref(v))
            lib.sb_plan_set_fft_variant(h, 0, 0, 0)
            lib.sb_plan_destroy(h)
    assert made > 100
    # the large grids: regenerated kernel planes at 1024^3 and 512^3 at lmax 10, and a 2D 1024^2 plan
    for ndim, shape, lmax in ((3, (1024, 1024, 1024), 6), (3, (512, 512, 512), 10), (2, (1024, 1024), 10)):
        prob, e = _problem(_lib, ndim, 3, np.linspace(0, 32, 11), lmax)
        sh = np.array(shape, dtype=np.int64)
        h = ctypes.c_void_p()
        assert lib.sb_plan_create(ctypes.byref(prob), 1, sh.ctypes.data_as(ctypes.POINTER(i64)), ctypes.byref(h)) == 0
        pb, sb = sz(), sz()
        assert lib.sb_plan_workspace(h, ctypes.byref(pb), ctypes.byref(sb)) == 0
        lib.sb_plan_destroy(h)
    lib.sb_plan_destroy(None)
