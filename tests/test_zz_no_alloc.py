"""sb_forward_noalloc (the forward pass with its working arrays in the library's fixed device
array, for callers that cannot allocate) against sb_forward through the C ABI: two calls in a
row, the second with a smaller input, each equal to sb_forward bit for bit (same kernels, same
order) and within the float32 bound of the oracle."""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from fieldgen import lognormal_field, linear_edges  # noqa: E402
from parity import TOL32, check  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problem(lib_mod, ndim, npcf, edges, lmax):
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.float64))
    p = lib_mod.SbProblem(ndim, npcf, len(e) - 1, e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), lmax, 0, 0, 0)
    return p, e


def _plan_persistent_only(lib_mod, lib, shape, edges, lmax, npcf):
    """A C plan bound to a persistent buffer only (no scratch) and prepared."""
    prob, e = _problem(lib_mod, len(shape), npcf, edges, lmax)
    sh = np.ascontiguousarray(np.array(shape, dtype=np.int64))
    h = ctypes.c_void_p()
    assert lib.sb_plan_create(ctypes.byref(prob), 1, sh.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              ctypes.byref(h)) == 0, lib.sb_last_error()
    pb, sbytes = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.sb_plan_workspace(h, ctypes.byref(pb), ctypes.byref(sbytes)) == 0
    pers = torch.empty(pb.value + 256, dtype=torch.uint8, device="cuda")
    pp = (pers.data_ptr() + 255) & ~255
    assert lib.sb_plan_bind(h, ctypes.c_void_p(pp), pb.value, None, 0) == 0, lib.sb_last_error()
    assert lib.sb_prepare(h, None) == 0, lib.sb_last_error()
    return h, pers, sbytes.value, e


@pytest.fixture(scope="module")
def libs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2210_10206_amd import _lib, api
    return _lib, _lib.load(), api


@pytest.mark.parametrize("npcf", [3, 4])
def test_forward_noalloc_matches_forward(libs, npcf):
    lib_mod, lib, api = libs
    cases = [((32, 32, 32), linear_edges(8, 4), 4, 1), ((16, 24, 16), linear_edges(6, 3), 2, 2)]
    if npcf == 4:
        cases = [((24, 24, 24), linear_edges(6, 4), 4, 3), ((16, 16, 16), linear_edges(4, 3), 2, 4)]
    for shape, edges, lmax, seed in cases:     # the second call has the smaller input
        say(f"case: sb_forward_noalloc vs sb_forward, {shape} npcf {npcf}, {len(edges) - 1} bins, lmax {lmax}")
        d = lognormal_field(shape, seed=seed, sigma=1.0)
        dev = torch.from_numpy(d).cuda()
        ref_plan = api.Plan([shape], edges, lmax, npcf=npcf)
        want = ref_plan.forward_raw([dev]).cpu().numpy()
        h, pers, need, e = _plan_persistent_only(lib_mod, lib, shape, edges, lmax, npcf)
        say(f"  scratch need {need / 2**20:.1f} MiB")
        got = torch.full((1, ref_plan.zeta_doubles), float("nan"), dtype=torch.float64, device="cuda")
        ptrs = (ctypes.c_void_p * 1)(dev.data_ptr())
        s = torch.cuda.current_stream()
        assert lib.sb_forward(h, ptrs, ctypes.c_void_p(got.data_ptr()), ctypes.c_void_p(s.cuda_stream)) == -3
        assert lib.sb_forward_noalloc(h, ptrs, ctypes.c_void_p(got.data_ptr()),
                                      ctypes.c_void_p(s.cuda_stream)) == 0, lib.sb_last_error()
        g = got.cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(g, want), f"max diff {np.max(np.abs(g - want))}"
        z = ref_plan.unpack(got)[0].cpu().numpy()
        if npcf == 3:
            ref = oracle.zeta3_full(d.astype(np.float64), edges, lmax).real
        else:
            ref = oracle.zeta4_full(d.astype(np.float64), edges, lmax)[1].real
        check(z, ref, TOL32, say)
        lib.sb_plan_destroy(h)
        ref_plan.close()


def test_forward_noalloc_rejects_a_plan_beyond_the_array(libs):
    lib_mod, lib, api = libs
    say("case: sb_forward_noalloc on a 128^3 plan whose scratch exceeds the fixed array")
    shape = (128, 128, 128)
    h, pers, need, e = _plan_persistent_only(lib_mod, lib, shape, linear_edges(8, 4), 4, 3)
    assert need > 64 << 20
    dev = torch.zeros(shape, dtype=torch.float32, device="cuda")
    z = torch.zeros(1000, dtype=torch.float64, device="cuda")
    ptrs = (ctypes.c_void_p * 1)(dev.data_ptr())
    assert lib.sb_forward_noalloc(h, ptrs, ctypes.c_void_p(z.data_ptr()), None) == -3
    assert b"64" in lib.sb_last_error() or b"67108864" in lib.sb_last_error()
    lib.sb_plan_destroy(h)
