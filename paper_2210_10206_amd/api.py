"""Python front end: ``Plan`` (one C plan plus its torch-owned device workspace),
``measure`` (the paper's measure/calc_zeta flow of Sec. 3.3) and ``ZetaFn`` (autograd).

Torch supplies device memory and the stream; every step of the computation runs
in the HIP library.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import SbProblem, check


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _aligned_buffer(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns 512-byte aligned blocks; keep a margin anyway
    t = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=device)
    return t


def _aligned_ptr(t: torch.Tensor) -> int:
    p = t.data_ptr()
    return (p + 255) & ~255


class Plan:
    """A plan for a batch of fields (shapes may differ).

    shapes     : list of grid shapes, each of length ndim (3 full, 2 projected)
    keep_coeffs: keep the coefficient arrays of the last field readable through coeffs()
    fused      : 3PCFs: contract inside the last FFT pass (False = the plain unfused path)
    bin_edges  : nbins + 1 increasing radii in cells; bin b = (e_b, e_{b+1}]
    lmax       : l_max in 3D, m_max in 2D
    npcf       : 3 or 4
    precision  : "fp32" or "split_bf16" (contraction arithmetic of the 4PCF paths)
    input_dtype: torch.float32 or torch.float64 (the density arrays' dtype)
    mfma       : full 4PCF: use the matrix-core contraction where it exists (l <= 4, <= 8 bins);
                 projected 4PCF: the matrix-core contraction (False = the vector-ALU kernel)
    parity     : full 4PCF: "even" (Alg. 6) or "odd" Lambda (the imaginary part of those sums)
    pack       : full 3PCF (fused path) and full 4PCF: carry the real m = 0 coefficient fields two
                 to a complex transform (False = one transform per (l, m))
    scratch_limit: bytes of kernel arrays a 3PCF plan keeps at once (default 48 GiB); above it
                 the passes run over chunks of (l, m) groups (sb_plan_set_scratch_limit)
    check_finite: scan the inputs of every call for NaN / Inf first (SB_FLAG_CHECK_FINITE)
    regen_kernels: fused 3PCF: keep no kernel spectra, regenerate them per call in scratch
                 (SB_FLAG_REGEN_KERNELS; automatic when the cache would exceed 64 GiB)
    half_kernels: 3D: keep only the axis-0 planes c_0 >= 0 of each kernel spectrum and take the
                 others by parity (SB_FLAG_HALF_KERNELS; automatic when the full cache would exceed
                 64 GiB, and with regen_kernels); half the persistent buffer, same traffic
    field_batch: fields of one shape per launch of each pass (sb_plan_set_field_batch): None or 0 =
                 as many as 32 GiB of kernel arrays allow, 1 = one launch sequence per field
    keep_for_adjoint: fused 3D 3PCF: every forward keeps each field's arrays before the last axis
                 in scratch, and a backward on the same fields reads them instead of recomputing
                 them (SB_FLAG_KEEP_FOR_ADJOINT; the scratch holds every field's arrays at once)
    """

    def __init__(self, shapes, bin_edges, lmax, npcf=3, precision="fp32", input_dtype=torch.float32,
                 device=None, stream=None, prepare=True, keep_coeffs=False, fused=True, mfma=True,
                 scratch_limit=None, parity="even", pack=True, check_finite=False, regen_kernels=False,
                 field_batch=None, half_kernels=False, keep_for_adjoint=False):
        self.lib = _lib.load()
        shapes = [tuple(int(x) for x in s) for s in shapes]
        ndim = len(shapes[0])
        if any(len(s) != ndim for s in shapes):
            raise ValueError("all shapes must have the same number of dimensions")
        self.shapes, self.ndim, self.npcf, self.lmax = shapes, ndim, int(npcf), int(lmax)
        self.edges = np.ascontiguousarray(np.asarray(bin_edges, dtype=np.float64))
        self.nbins = len(self.edges) - 1
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.input_dtype = input_dtype
        prec = {"fp32": _lib.SB_PREC_FP32, "split_bf16": _lib.SB_PREC_SPLIT_BF16}[precision]
        self.precision = precision
        self._prob = SbProblem(ndim, self.npcf, self.nbins,
                               self.edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self.lmax, prec,
                               _lib.SB_IN_F64 if input_dtype == torch.float64 else _lib.SB_IN_F32,
                               (_lib.SB_FLAG_KEEP_COEFFS if keep_coeffs else 0) | (0 if fused else _lib.SB_FLAG_UNFUSED)
                               | (0 if mfma else _lib.SB_FLAG_NO_MFMA)
                               | (_lib.SB_FLAG_ODD_PARITY if parity == "odd" else 0)
                               | (0 if pack else _lib.SB_FLAG_NO_PACK)
                               | (_lib.SB_FLAG_CHECK_FINITE if check_finite else 0)
                               | (_lib.SB_FLAG_REGEN_KERNELS if regen_kernels else 0)
                               | (_lib.SB_FLAG_HALF_KERNELS if half_kernels else 0)
                               | (_lib.SB_FLAG_KEEP_FOR_ADJOINT if keep_for_adjoint else 0))
        if parity not in ("even", "odd"):
            raise ValueError("parity must be 'even' or 'odd'")
        self.parity = parity
        sh = np.ascontiguousarray(np.array(shapes, dtype=np.int64).ravel())
        self._shapes_arr = sh
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(self.lib.sb_plan_create(ctypes.byref(self._prob), len(shapes),
                                          sh.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(handle)),
                  "sb_plan_create")
        self.handle = handle
        if scratch_limit is not None:
            check(self.lib.sb_plan_set_scratch_limit(self.handle, ctypes.c_uint64(int(scratch_limit))),
                  "sb_plan_set_scratch_limit")
        if field_batch is not None:
            check(self.lib.sb_plan_set_field_batch(self.handle, int(field_batch)), "sb_plan_set_field_batch")
        fb = ctypes.c_int32()
        check(self.lib.sb_plan_get_field_batch(self.handle, ctypes.byref(fb)), "sb_plan_get_field_batch")
        self.field_batch = fb.value
        pb, sbytes = ctypes.c_size_t(), ctypes.c_size_t()
        check(self.lib.sb_plan_workspace(self.handle, ctypes.byref(pb), ctypes.byref(sbytes)), "sb_plan_workspace")
        self.persistent_bytes, self.scratch_bytes = pb.value, sbytes.value
        self._persist = _aligned_buffer(pb.value, self.device)
        self._scratch = _aligned_buffer(sbytes.value, self.device)
        check(self.lib.sb_plan_bind(self.handle, ctypes.c_void_p(_aligned_ptr(self._persist)), pb.value,
                                    ctypes.c_void_p(_aligned_ptr(self._scratch)), sbytes.value), "sb_plan_bind")
        n = ctypes.c_int64()
        check(self.lib.sb_zeta_size(self.handle, ctypes.byref(n)), "sb_zeta_size")
        self.zeta_doubles = n.value
        self.prepared = False
        if prepare:
            self.prepare(stream)

    # ------------------------------------------------------------------ lifecycle
    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            self.lib.sb_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def prepare(self, stream=None):
        with torch.cuda.device(self.device):
            check(self.lib.sb_prepare(self.handle, _stream_ptr(stream)), "sb_prepare")
        self.prepared = True

    def autotune(self, stream=None, cache_path=None):
        """Time the launch shapes (sb_autotune); cache_path: JSON file of tuned choices, read
        when it holds this plan's entry, extended otherwise."""
        path = None if cache_path is None else str(cache_path).encode()
        with torch.cuda.device(self.device):
            check(self.lib.sb_autotune(self.handle, _stream_ptr(stream), path), "sb_autotune")

    # ------------------------------------------------------------------ layout
    def zeta_index(self):
        rows, cols = ctypes.c_int32(), ctypes.c_int32()
        tab = ctypes.POINTER(ctypes.c_int32)()
        check(self.lib.sb_zeta_index(self.handle, ctypes.byref(rows), ctypes.byref(cols), ctypes.byref(tab)),
              "sb_zeta_index")
        arr = np.array([tab[i] for i in range(rows.value * cols.value)], dtype=np.int32)
        return arr.reshape(rows.value, cols.value)

    def bin_counts(self, field: int = 0):
        out = np.zeros(self.nbins, dtype=np.int64)
        check(self.lib.sb_bin_counts(self.handle, int(field), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
              "sb_bin_counts")
        return out

    def warnings(self) -> int:
        """SB_WARN_* bits of the plan (SB_WARN_BOX_TRUNCATED: the outer edge reaches half a grid
        edge, so the zero-centred kernel support is cut by the box)."""
        bits = ctypes.c_uint32()
        check(self.lib.sb_plan_warnings(self.handle, ctypes.byref(bits)), "sb_plan_warnings")
        return bits.value

    def zeta_shape(self):
        rows = self.zeta_index().shape[0]
        nb = self.nbins
        tail = (nb, nb) if self.npcf == 3 else (nb, nb, nb)
        return (rows,) + tail

    def _check_fields(self, deltas):
        if len(deltas) != len(self.shapes):
            raise ValueError(f"expected {len(self.shapes)} fields, got {len(deltas)}")
        for d, s in zip(deltas, self.shapes):
            if tuple(d.shape) != s:
                raise ValueError(f"field shape {tuple(d.shape)} does not match the plan's {s}")
            if d.device != self.device or not d.is_contiguous() or d.dtype != self.input_dtype:
                raise ValueError("fields must be contiguous device tensors of the plan's dtype and device")

    def _ptrs(self, tensors):
        arr = (ctypes.c_void_p * len(tensors))(*[ctypes.c_void_p(t.data_ptr()) for t in tensors])
        return arr

    # ------------------------------------------------------------------ compute
    def forward_raw(self, deltas, out=None, stream=None, graph=False):
        """Raw result buffer: (batch, zeta_doubles) float64 on the device."""
        self._check_fields(deltas)
        if out is None:
            out = torch.empty((len(deltas), self.zeta_doubles), dtype=torch.float64, device=self.device)
        ptrs = self._ptrs(deltas)
        fn = self.lib.sb_forward_graph if graph else self.lib.sb_forward
        with torch.cuda.device(self.device):
            check(fn(self.handle, ptrs, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
                  "sb_forward_graph" if graph else "sb_forward")
        return out

    def forward(self, deltas, stream=None, graph=False):
        """List of fields -> tensor (batch, rows, nb, nb[, nb]); complex for projected outputs."""
        raw = self.forward_raw(deltas, stream=stream, graph=graph)
        return self.unpack(raw)

    def unpack(self, raw):
        b = raw.shape[0]
        shp = self.zeta_shape()
        if self.ndim == 2:
            return torch.view_as_complex(raw.reshape((b,) + shp + (2,)))
        return raw.reshape((b,) + shp)

    def normalize_raw(self, deltas, raw, stream=None, want_norm=False):
        """Divide a raw result buffer (batch, zeta_doubles), in place on the device, by the N of
        Sec. 2.5 of each field (sb_normalize); optionally return the factors (batch, nb, nb[, nb])."""
        self._check_fields(deltas)
        if tuple(raw.shape) != (len(self.shapes), self.zeta_doubles) or raw.dtype != torch.float64 \
                or raw.device != self.device or not raw.is_contiguous():
            raise ValueError("raw must be the contiguous (batch, zeta_doubles) float64 result of this plan")
        nt = self.nbins ** (self.npcf - 1)
        norm = torch.empty((len(self.shapes), nt), dtype=torch.float64, device=self.device) if want_norm else None
        with torch.cuda.device(self.device):
            check(self.lib.sb_normalize(self.handle, self._ptrs(deltas), ctypes.c_void_p(raw.data_ptr()),
                                        ctypes.c_void_p(norm.data_ptr() if norm is not None else None),
                                        _stream_ptr(stream)), "sb_normalize")
        if norm is not None:
            return norm.reshape((len(self.shapes),) + (self.nbins,) * (self.npcf - 1))
        return None

    def backward(self, deltas, grad_zeta, stream=None):
        """d loss / d delta for the full 3PCF given d loss / d Z (batch, lmax+1, nb, nb) float64."""
        self._check_fields(deltas)
        gz = grad_zeta.to(device=self.device, dtype=torch.float64).contiguous()
        if gz.numel() != len(self.shapes) * self.zeta_doubles:
            raise ValueError(f"grad_zeta has {gz.numel()} values; this plan needs "
                             f"{len(self.shapes)} x {self.zeta_doubles}")
        grads = [torch.empty(s, dtype=torch.float32, device=self.device) for s in self.shapes]
        with torch.cuda.device(self.device):
            check(self.lib.sb_backward(self.handle, self._ptrs(deltas), ctypes.c_void_p(gz.data_ptr()),
                                       self._ptrs(grads), _stream_ptr(stream)), "sb_backward")
        return grads

    def coeffs(self, k: int, shape=None):
        """Coefficient array k (= lm * nbins + b) of the last field, as a complex64 view."""
        ptr = ctypes.c_void_p()
        check(self.lib.sb_coeffs(self.handle, int(k), ctypes.byref(ptr)), "sb_coeffs")
        shape = tuple(shape or self.shapes[-1])
        n = int(np.prod(shape))
        off = ptr.value - self._scratch.data_ptr()
        return self._scratch[off: off + 8 * n].view(torch.complex64).reshape(shape)

    def fft_variants(self, n: int) -> int:
        return int(self.lib.sb_fft_variants(int(n)))

    def set_fft_variant(self, n: int, axis: int, variant: int):
        check(self.lib.sb_plan_set_fft_variant(self.handle, int(n), int(axis), int(variant)),
              "sb_plan_set_fft_variant")

    def contract_tile(self):
        """Cells per workgroup of the cell-parallel contraction and its allowed range (lo, hi)."""
        c, lo, hi = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(self.lib.sb_plan_get_contract_tile(self.handle, ctypes.byref(c), ctypes.byref(lo), ctypes.byref(hi)),
              "sb_plan_get_contract_tile")
        return c.value, (lo.value, hi.value)

    def set_contract_tile(self, cells: int):
        check(self.lib.sb_plan_set_contract_tile(self.handle, int(cells)), "sb_plan_set_contract_tile")

    def choices(self):
        """The tuned launch shapes of this plan: {"fft": {"n,axis": variant} for every (length,
        axis) of its shapes, "contract_tile": cells per workgroup}; set_choices() restores them
        (e.g. tuned once, saved as JSON)."""
        fft = {}
        for shape in self.shapes:
            for axis, n in enumerate(shape):
                v = ctypes.c_int32()
                check(self.lib.sb_plan_get_fft_variant(self.handle, int(n), axis, ctypes.byref(v)),
                      "sb_plan_get_fft_variant")
                fft[f"{n},{axis}"] = v.value
        return {"fft": fft, "contract_tile": self.contract_tile()[0]}

    def set_choices(self, choices):
        for key, v in choices.get("fft", {}).items():
            n, axis = (int(x) for x in key.split(","))
            self.set_fft_variant(n, axis, int(v))
        if "contract_tile" in choices:
            self.set_contract_tile(choices["contract_tile"])

    def profile(self, enable: bool):
        check(self.lib.sb_profile(self.handle, int(bool(enable))), "sb_profile")

    def launch_records(self):
        """Per-launch records of the profiled calls: list of dicts (stage, fft_n, fft_sign,
        batch, bytes, flops, ms)."""
        n = ctypes.c_int32()
        check(self.lib.sb_profile_read(self.handle, 0, ctypes.byref(n), None), "sb_profile_read")
        arr = (_lib.SbLaunchRecord * max(n.value, 1))()
        check(self.lib.sb_profile_read(self.handle, n.value, ctypes.byref(n), arr), "sb_profile_read")
        keys = ["stage", "kernel", "fft_n", "fft_sign", "batch", "bytes", "flops", "ms"]
        return [{k: getattr(arr[i], k) for k in keys} for i in range(n.value)]

    def stage_times(self):
        f, c = ctypes.c_double(), ctypes.c_double()
        nf, nc = ctypes.c_int32(), ctypes.c_int32()
        check(self.lib.sb_stage_times(self.handle, ctypes.byref(f), ctypes.byref(nf), ctypes.byref(c),
                                      ctypes.byref(nc)), "sb_stage_times")
        return {"fft_ms": f.value, "fft_launches": nf.value, "contract_ms": c.value, "contract_launches": nc.value}


def normalization(plan: Plan, deltas, field: int = 0) -> np.ndarray:
    """The N of Sec. 2.5 of one field (sb_normalize: N_gal = sum (delta + 1) on the device, unit
    cells, V_bin = cells in bin, nbar = N_gal / N_g), shaped like the result's bin axes."""
    raw = torch.zeros((len(plan.shapes), plan.zeta_doubles), dtype=torch.float64, device=plan.device)
    norm = plan.normalize_raw(deltas, raw, want_norm=True)
    return norm[field].cpu().numpy()


def measure(delta, bin_edges, lmax, projected=False, npcf=3, precision="fp32", normalized=False):
    """One field: the raw grid sums of Alg. 5-8 (see include/sarabande_hip.h for the layouts).

    delta: a 3D (full) or 2D (projected) torch tensor on a GPU, or a numpy array (copied to
    the current GPU).  Returns (zeta, index) where index lists l, (l1,l2,l3), m or (m1,m2)
    of the result's leading axis.  normalized=True divides by the N of Sec. 2.5."""
    if isinstance(delta, np.ndarray):
        delta = torch.from_numpy(np.ascontiguousarray(delta)).cuda()
    if delta.dtype not in (torch.float32, torch.float64):
        delta = delta.float()
    delta = delta.contiguous()
    if (delta.dim() == 2) != bool(projected):
        raise ValueError("projected=True needs a 2D field, projected=False a 3D field")
    plan = Plan([tuple(delta.shape)], bin_edges, lmax, npcf=npcf, precision=precision,
                input_dtype=delta.dtype, device=delta.device)
    raw = plan.forward_raw([delta])
    if normalized:
        plan.normalize_raw([delta], raw)
    z = plan.unpack(raw)[0]
    idx = plan.zeta_index()
    torch.cuda.synchronize(delta.device)
    plan.close()
    return z, idx


class ZetaFn(torch.autograd.Function):
    """Full 3PCF sums Z[l][b1][b2] of one field with a hand-written adjoint (sb_backward)."""

    @staticmethod
    def forward(ctx, delta, plan: Plan):
        if plan.ndim != 3 or plan.npcf != 3:
            raise ValueError("ZetaFn supports the full 3PCF")
        d = delta.detach().contiguous()
        z = plan.forward([d])[0]
        ctx.plan = plan
        ctx.save_for_backward(d)
        return z

    @staticmethod
    def backward(ctx, gz):
        (d,) = ctx.saved_tensors
        g = ctx.plan.backward([d], gz.unsqueeze(0))[0]
        return g.to(d.dtype), None
