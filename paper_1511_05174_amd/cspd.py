"""Thin Python binding of the cspd C-ABI (include/cspd.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory and streams.  If the compiled
library is missing, importing the functions raises -- there is no fallback.

Names follow the C entry points:
  cspd_plan, cspd_plan_destroy, cspd_plan_device_bytes,
  cspd_omp_full, cspd_omp_cross_scale,
  cspd_graph_cross_scale, cspd_graph_launch, cspd_graph_destroy,
  cspd_autotune, cspd_tuned_kernel, cspd_set_tuned_kernel,
  cspd_patch_count, cspd_extract_patches, cspd_aggregate_patches,
  cspd_ksvd_update,
  cspd_serve_create, cspd_serve_submit, cspd_serve_poll, cspd_serve_destroy,
  cspd_last_error, cspd_version.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcspd.so")
MAX_SCALES = 4
NOALLOC_SCRATCH_BYTES = 32 << 20     # CSPD_NOALLOC_SCRATCH_BYTES

OK, E_INVALID, E_SHAPE, E_NOMEM, E_DEVICE, E_BUSY, E_NOTFOUND, E_CAPACITY, E_UNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
PHI = {"identity": 0, "dense": 1, "mask": 2}
DTYPES = {"f64": 0, "f32": 1}
CORR = {"native": 0, "bf16": 1, "f16": 2}


class CspdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cspd error {code}: {msg}")
        self.code = code


class PlanDesc(C.Structure):
    _fields_ = [
        ("n_scales", C.c_int32),
        ("dim", C.c_int32 * MAX_SCALES),
        ("atoms", C.c_int32 * MAX_SCALES),
        ("dict", C.c_void_p * MAX_SCALES),
        ("up_map", C.c_void_p * MAX_SCALES),
        ("phi_kind", C.c_int32),
        ("m", C.c_int32),
        ("phi", C.c_void_p),
        ("dtype", C.c_int32),
        ("corr_mode", C.c_int32),
        ("rescore_m", C.c_int32),
        ("k_max", C.c_int32),
        ("device", C.c_int32),
        ("n_phases", C.c_int32),
    ]


class Job(C.Structure):
    _fields_ = [
        ("plan", C.c_void_p),
        ("B", C.c_int64),
        ("y", C.c_void_p),
        ("mask", C.c_void_p),
        ("k_fine", C.c_void_p),
        ("k_fine_uniform", C.c_int32),
        ("k_scale", C.c_int32 * MAX_SCALES),
        ("full", C.c_int32),
        ("support", C.c_void_p),
        ("coef", C.c_void_p),
        ("k_used", C.c_void_p),
        ("xhat", C.c_void_p),
        ("on_device", C.c_int32),
    ]


class PatchGrid(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32),
        ("dims", C.c_int32 * 4),
        ("patch", C.c_int32 * 4),
        ("stride", C.c_int32 * 4),
    ]


class JobStats(C.Structure):
    _fields_ = [
        ("submit_ns", C.c_int64),
        ("admit_ns", C.c_int64),
        ("start_ns", C.c_int64),
        ("finish_ns", C.c_int64),
        ("patches", C.c_int64),
        ("batched_with", C.c_int32),
        ("status", C.c_int32),
        ("server_resident_bytes", C.c_int64),
    ]


# Every symbol the header declares, with its ctypes signature.
SIGNATURES = {
    "cspd_plan": (C.c_int32, [C.POINTER(PlanDesc), C.POINTER(C.c_void_p)]),
    "cspd_plan_destroy": (None, [C.c_void_p]),
    "cspd_plan_device_bytes": (C.c_int64, [C.c_void_p]),
    "cspd_omp_full": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "cspd_omp_cross_scale": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_void_p]),
    "cspd_omp_cross_scale_phased": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                                C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                                C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "cspd_omp_cross_scale_noalloc": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                                 C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                                 C.c_void_p, C.c_void_p, C.c_void_p]),
    "cspd_graph_cross_scale": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "cspd_graph_launch": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "cspd_graph_destroy": (None, [C.c_void_p]),
    "cspd_autotune": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_int32, C.c_int32, C.c_void_p]),
    "cspd_tuned_kernel": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "cspd_set_tuned_kernel": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                          C.c_int32]),
    "cspd_serve_create": (C.c_int32, [C.c_int32, C.c_int64, C.c_int32, C.POINTER(C.c_void_p)]),
    "cspd_serve_submit": (C.c_int32, [C.c_void_p, C.POINTER(Job), C.POINTER(C.c_uint64)]),
    "cspd_serve_poll": (C.c_int32, [C.c_void_p, C.c_uint64, C.c_int64, C.POINTER(JobStats)]),
    "cspd_serve_destroy": (None, [C.c_void_p]),
    "cspd_patch_count": (C.c_int64, [C.POINTER(PatchGrid)]),
    "cspd_extract_patches": (C.c_int32, [C.POINTER(PatchGrid), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p]),
    "cspd_aggregate_patches": (C.c_int32, [C.POINTER(PatchGrid), C.c_void_p, C.c_void_p, C.c_void_p]),
    "cspd_ksvd_update": (C.c_int32, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                     C.c_void_p, C.c_int32, C.c_void_p]),
    "cspd_profile_enable": (C.c_int32, [C.c_int32]),
    "cspd_profile_read": (C.c_int32, [C.c_int32, C.c_char_p, C.c_int32, C.POINTER(C.c_int64),
                                      C.POINTER(C.c_double)]),
    "cspd_profile_reset": (None, []),
    "cspd_last_error": (C.c_char_p, []),
    "cspd_version": (C.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libcspd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"cspd: {path} is missing; build it with paper_1511_05174_amd/build.py")
    # PyTorch ships its own HIP runtime.  Importing torch first makes the
    # library bind to that instance (same soname), so the process holds one
    # runtime and torch's device pointers and streams are valid here.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        raise CspdError(rc, load().cspd_last_error().decode())


def cspd_last_error() -> str:
    return load().cspd_last_error().decode()


def cspd_version() -> str:
    return load().cspd_version().decode()


class Plan:
    """Owns a cspd_plan_t; destroyed with the object."""

    def __init__(self, handle: int, dims, atoms, m, phi_kind, dtype, k_max, device):
        self.handle = handle
        self.dims = list(dims)
        self.atoms = list(atoms)
        self.m = m
        self.phi_kind = phi_kind
        self.dtype = dtype
        self.k_max = k_max
        self.device = device

    @property
    def n_scales(self):
        return len(self.dims)

    @property
    def n(self):
        return self.dims[-1]

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.cspd_plan_destroy(h)


def cspd_plan(dims: Sequence[int], atoms: Sequence[int], dicts, up_maps, phi_kind: str, m: int,
              phi=None, dtype: str = "f32", corr_mode: str = "native", rescore_m: int = 0,
              k_max: int = 16, device: int = 0) -> Plan:
    """Build a resident plan.  dicts[s] is a (T_s, N_s) float64 array (the
    column-major N_s x T_s dictionary); up_maps[s] an int32 array of length
    N_{s+1}; phi a (M, N) float64 array for the dense operator, or (P, M, N)
    for P operators chosen per patch (cspd_omp_cross_scale_phased)."""
    lib = load()
    S = len(dims)
    d = PlanDesc()
    d.n_scales = S
    keep = []
    for s in range(S):
        d.dim[s] = int(dims[s])
        d.atoms[s] = int(atoms[s])
        a = np.ascontiguousarray(dicts[s], dtype=np.float64)
        keep.append(a)
        d.dict[s] = a.ctypes.data
        if s < S - 1:
            u = np.ascontiguousarray(up_maps[s], dtype=np.int32)
            keep.append(u)
            d.up_map[s] = u.ctypes.data
    d.phi_kind = PHI[phi_kind]
    d.m = int(m)
    d.n_phases = 1
    if phi is not None:
        p = np.ascontiguousarray(phi, dtype=np.float64)
        if p.ndim == 3:                  # one operator per phase
            d.n_phases = p.shape[0]
        keep.append(p)
        d.phi = p.ctypes.data
    d.dtype = DTYPES[dtype]
    d.corr_mode = CORR[corr_mode]
    d.rescore_m = int(rescore_m)
    d.k_max = int(k_max)
    d.device = int(device)
    h = C.c_void_p()
    _check(lib.cspd_plan(C.byref(d), C.byref(h)))
    return Plan(h.value, dims, atoms, m, phi_kind, dtype, k_max, device)


def plan_from_workload(w, dtype: Optional[str] = None, corr_mode: str = "native", k_max: int = 16,
                       device: int = 0, rescore_m: int = 0) -> Plan:
    return cspd_plan(w.dims, w.atoms, w.dicts, w.up_maps, w.phi_kind, w.m, w.phi,
                     dtype=dtype or w.dtype, corr_mode=corr_mode, rescore_m=rescore_m, k_max=k_max,
                     device=device)


def cspd_plan_destroy(plan: Plan):
    h, plan.handle = plan.handle, None
    if h:
        load().cspd_plan_destroy(h)


def cspd_plan_device_bytes(plan: Plan) -> int:
    return int(load().cspd_plan_device_bytes(plan.handle))


def _torch():
    import torch
    return torch


def _tdtype(plan: Plan):
    torch = _torch()
    return torch.float64 if plan.dtype == "f64" else torch.float32


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _outputs(plan, B, support, coef, k_used, xhat, want_xhat):
    torch = _torch()
    dev = torch.device("cuda", plan.device)
    if support is None:
        support = torch.empty((B, plan.k_max), dtype=torch.int32, device=dev)
    if coef is None:
        coef = torch.empty((B, plan.k_max), dtype=_tdtype(plan), device=dev)
    if k_used is None:
        k_used = torch.empty((B,), dtype=torch.int32, device=dev)
    if xhat is None and want_xhat:
        xhat = torch.empty((B, plan.n), dtype=_tdtype(plan), device=dev)
    return support, coef, k_used, xhat


def _check_inputs(plan, y, mask, k):
    torch = _torch()
    if y.dim() != 2 or y.shape[1] != plan.m or not y.is_contiguous() or y.dtype != _tdtype(plan):
        raise ValueError(f"y must be a contiguous ({'{B}'}, {plan.m}) {_tdtype(plan)} tensor")
    if mask is not None and (mask.dtype != torch.uint8 or tuple(mask.shape) != (y.shape[0], plan.n)
                             or not mask.is_contiguous()):
        raise ValueError("mask must be a contiguous (B, N) uint8 tensor")
    if k is not None and (k.dtype != torch.int32 or tuple(k.shape) != (y.shape[0],) or not k.is_contiguous()):
        raise ValueError("k must be a contiguous (B,) int32 tensor")


def cspd_omp_full(plan: Plan, y, mask=None, k=None, k_uniform: int = 0, support=None, coef=None,
                  k_used=None, xhat=None, want_xhat: bool = True, stream=None):
    """Algorithm 1 over D_high; returns (support, coef, k_used, xhat)."""
    _check_inputs(plan, y, mask, k)
    B = y.shape[0]
    support, coef, k_used, xhat = _outputs(plan, B, support, coef, k_used, xhat, want_xhat)
    _check(load().cspd_omp_full(plan.handle, B, _ptr(y), _ptr(mask), _ptr(k), int(k_uniform),
                                _ptr(support), _ptr(coef), _ptr(k_used), _ptr(xhat), _stream(stream)))
    return support, coef, k_used, xhat


def cspd_omp_cross_scale(plan: Plan, y, mask=None, k_scale: Sequence[int] = (), k_fine=None,
                         k_fine_uniform: int = 0, support=None, coef=None, k_used=None, xhat=None,
                         support_coarse=None, want_xhat: bool = True, stream=None):
    """Zero-tree OMP over all scales; returns (support, coef, k_used, xhat)."""
    _check_inputs(plan, y, mask, k_fine)
    B = y.shape[0]
    support, coef, k_used, xhat = _outputs(plan, B, support, coef, k_used, xhat, want_xhat)
    ks = (C.c_int32 * MAX_SCALES)(*([int(v) for v in k_scale] + [0] * (MAX_SCALES - len(k_scale))))
    _check(load().cspd_omp_cross_scale(plan.handle, B, _ptr(y), _ptr(mask), ks, _ptr(k_fine),
                                       int(k_fine_uniform), _ptr(support), _ptr(coef), _ptr(k_used),
                                       _ptr(xhat), _ptr(support_coarse), _stream(stream)))
    return support, coef, k_used, xhat


def cspd_omp_cross_scale_phased(plan: Plan, phase, y, mask=None, k_scale: Sequence[int] = (), k_fine=None,
                                k_fine_uniform: int = 0, support=None, coef=None, k_used=None, xhat=None,
                                support_coarse=None, want_xhat: bool = True, stream=None):
    """Zero-tree OMP with each patch's operator chosen by phase (device int32[B])."""
    _check_inputs(plan, y, mask, k_fine)
    B = y.shape[0]
    support, coef, k_used, xhat = _outputs(plan, B, support, coef, k_used, xhat, want_xhat)
    ks = (C.c_int32 * MAX_SCALES)(*([int(v) for v in k_scale] + [0] * (MAX_SCALES - len(k_scale))))
    _check(load().cspd_omp_cross_scale_phased(plan.handle, B, _ptr(phase), _ptr(y), _ptr(mask), ks, _ptr(k_fine),
                                              int(k_fine_uniform), _ptr(support), _ptr(coef), _ptr(k_used),
                                              _ptr(xhat), _ptr(support_coarse), _stream(stream)))
    return support, coef, k_used, xhat


def cspd_omp_cross_scale_noalloc(plan: Plan, y, mask=None, k_scale: Sequence[int] = (), k_fine=None,
                                 k_fine_uniform: int = 0, support=None, coef=None, k_used=None, xhat=None,
                                 support_coarse=None, want_xhat: bool = True, stream=None):
    """cspd_omp_cross_scale on the library's static workspace (the C call
    allocates nothing; outputs the caller does not pass are allocated here,
    by torch, before the call)."""
    _check_inputs(plan, y, mask, k_fine)
    B = y.shape[0]
    support, coef, k_used, xhat = _outputs(plan, B, support, coef, k_used, xhat, want_xhat)
    ks = (C.c_int32 * MAX_SCALES)(*([int(v) for v in k_scale] + [0] * (MAX_SCALES - len(k_scale))))
    _check(load().cspd_omp_cross_scale_noalloc(plan.handle, B, _ptr(y), _ptr(mask), ks, _ptr(k_fine),
                                               int(k_fine_uniform), _ptr(support), _ptr(coef), _ptr(k_used),
                                               _ptr(xhat), _ptr(support_coarse), _stream(stream)))
    return support, coef, k_used, xhat


class Graph:
    """A captured call (cspd_graph_t) and the tensors it reads and writes."""

    def __init__(self, handle, keep):
        self.handle = handle
        self.keep = keep            # buffers the graph refers to stay alive with it

    def __del__(self):
        try:
            cspd_graph_destroy(self)
        except Exception:
            pass


def cspd_graph_cross_scale(plan: Plan, y, mask=None, k_scale: Sequence[int] = (), k_fine=None,
                           k_fine_uniform: int = 0, support=None, coef=None, k_used=None, xhat=None,
                           support_coarse=None, want_xhat: bool = True):
    """Capture a cross-scale call into a HIP graph; returns (graph, support,
    coef, k_used, xhat).  Replays read y / mask / k_fine as they are then."""
    _check_inputs(plan, y, mask, k_fine)
    B = y.shape[0]
    support, coef, k_used, xhat = _outputs(plan, B, support, coef, k_used, xhat, want_xhat)
    ks = (C.c_int32 * MAX_SCALES)(*([int(v) for v in k_scale] + [0] * (MAX_SCALES - len(k_scale))))
    h = C.c_void_p()
    _check(load().cspd_graph_cross_scale(plan.handle, B, _ptr(y), _ptr(mask), ks, _ptr(k_fine),
                                         int(k_fine_uniform), _ptr(support), _ptr(coef), _ptr(k_used),
                                         _ptr(xhat), _ptr(support_coarse), C.byref(h)))
    g = Graph(h.value, (plan, y, mask, k_fine, support, coef, k_used, xhat, support_coarse))
    return g, support, coef, k_used, xhat


def cspd_graph_launch(graph: Graph, stream=None):
    _check(load().cspd_graph_launch(graph.handle, _stream(stream)))


def cspd_graph_destroy(graph: Graph):
    h, graph.handle = graph.handle, None
    if h:
        load().cspd_graph_destroy(h)


TUNED_KINDS = {0: "rules", 1: "first_mfma", 2: "vec", 3: "gram", 4: "mfma_gram", 5: "gemm_gram"}


def cspd_autotune(plan: Plan, y, mask=None, k_scale: Sequence[int] = (), k_fine=None,
                  k_fine_uniform: int = 0, reps: int = 3, stream=None):
    """Time every kernel variant of each scale on this batch and keep the
    fastest in the plan (blocks until done)."""
    _check_inputs(plan, y, mask, k_fine)
    ks = (C.c_int32 * MAX_SCALES)(*([int(v) for v in k_scale] + [0] * (MAX_SCALES - len(k_scale))))
    _check(load().cspd_autotune(plan.handle, y.shape[0], _ptr(y), _ptr(mask), ks, _ptr(k_fine),
                                int(k_fine_uniform), int(reps), _stream(stream)))


def cspd_tuned_kernel(plan: Plan, scale: int, bucket: int):
    """(kind name, nc, ppw, cand) of the plan's tuned kernel for a scale and
    sparsity bucket (0: K <= 4, 1: K <= 8, 2: K <= 16)."""
    kind, nc, ppw, cand = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(load().cspd_tuned_kernel(plan.handle, int(scale), int(bucket), C.byref(kind), C.byref(nc),
                                    C.byref(ppw), C.byref(cand)))
    return TUNED_KINDS.get(kind.value, str(kind.value)), nc.value, ppw.value, cand.value


def cspd_set_tuned_kernel(plan: Plan, scale: int, bucket: int, kind, nc: int = 1, ppw: int = 1, cand: int = 0):
    """Pin a kernel variant (kind name or number; \"rules\" clears)."""
    if isinstance(kind, str):
        kind = {v: k for k, v in TUNED_KINDS.items()}[kind]
    _check(load().cspd_set_tuned_kernel(plan.handle, int(scale), int(bucket), int(kind), int(nc), int(ppw),
                                        int(cand)))


def patch_grid(dims: Sequence[int], patch: Sequence[int], stride: Sequence[int]) -> PatchGrid:
    """A cspd_patch_grid for a signal of len(dims) axes (1..4)."""
    if not (len(dims) == len(patch) == len(stride)) or not 1 <= len(dims) <= 4:
        raise ValueError("dims, patch and stride need the same length, 1..4")
    g = PatchGrid()
    g.ndim = len(dims)
    for i, (d, q, t) in enumerate(zip(dims, patch, stride)):
        g.dims[i], g.patch[i], g.stride[i] = int(d), int(q), int(t)
    return g


def cspd_patch_count(grid: PatchGrid) -> int:
    n = int(load().cspd_patch_count(C.byref(grid)))
    if n < 0:
        raise CspdError(E_SHAPE, cspd_last_error())
    return n


def cspd_extract_patches(grid: PatchGrid, signal, mask=None, y=None, patch_mask=None, want_mask: bool = True,
                         stream=None):
    """Patches of a device float signal (and of its uint8 mask); returns
    (y, patch_mask)."""
    torch = _torch()
    n = cspd_patch_count(grid)
    vol = int(np.prod([grid.patch[i] for i in range(grid.ndim)]))
    dims = tuple(grid.dims[i] for i in range(grid.ndim))
    if signal.dtype != torch.float32 or tuple(signal.shape) != dims or not signal.is_contiguous():
        raise ValueError(f"signal must be a contiguous float32 tensor of shape {dims}")
    if mask is not None and (mask.dtype != torch.uint8 or tuple(mask.shape) != dims or not mask.is_contiguous()):
        raise ValueError(f"mask must be a contiguous uint8 tensor of shape {dims}")
    if y is None:
        y = torch.empty((n, vol), dtype=torch.float32, device=signal.device)
    if patch_mask is None and want_mask:
        patch_mask = torch.empty((n, vol), dtype=torch.uint8, device=signal.device)
    _check(load().cspd_extract_patches(C.byref(grid), _ptr(signal), _ptr(mask), _ptr(y), _ptr(patch_mask),
                                       _stream(stream)))
    return y, patch_mask


def cspd_aggregate_patches(grid: PatchGrid, estimates, out=None, stream=None):
    """Mean of the covering patches' estimates at every sample; returns the
    signal tensor."""
    torch = _torch()
    n = cspd_patch_count(grid)
    vol = int(np.prod([grid.patch[i] for i in range(grid.ndim)]))
    dims = tuple(grid.dims[i] for i in range(grid.ndim))
    if estimates.dtype != torch.float32 or tuple(estimates.shape) != (n, vol) or not estimates.is_contiguous():
        raise ValueError(f"estimates must be a contiguous float32 tensor of shape {(n, vol)}")
    if out is None:
        out = torch.empty(dims, dtype=torch.float32, device=estimates.device)
    _check(load().cspd_aggregate_patches(C.byref(grid), _ptr(estimates), _ptr(out), _stream(stream)))
    return out


def cspd_ksvd_update(x, dict_rows, support, coef, stream=None):
    """One K-SVD dictionary-update sweep in place: x (P, N) float32, dict_rows
    (T, N) float32 (one atom per row), support (P, k) int32, coef (P, k)
    float32 -- all contiguous device tensors."""
    torch = _torch()
    P, N = x.shape
    T = dict_rows.shape[0]
    k = support.shape[1]
    for name, t, shape, dt in (("x", x, (P, N), torch.float32), ("dict_rows", dict_rows, (T, N), torch.float32),
                               ("support", support, (P, k), torch.int32), ("coef", coef, (P, k), torch.float32)):
        if t.dtype != dt or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dt} tensor of shape {shape}")
    _check(load().cspd_ksvd_update(_ptr(x), P, N, _ptr(dict_rows), T, _ptr(support), _ptr(coef), k,
                                   _stream(stream)))


def cspd_profile_enable(on: bool = True):
    _check(load().cspd_profile_enable(1 if on else 0))


def cspd_profile_reset():
    load().cspd_profile_reset()


def cspd_profile_read():
    """{label: (launches, total_ms)} for every kernel recorded since the last reset."""
    lib = load()
    out = {}
    n = lib.cspd_profile_read(-1, None, 0, None, None)
    for i in range(n):
        buf = C.create_string_buffer(128)
        cnt = C.c_int64()
        ms = C.c_double()
        lib.cspd_profile_read(i, buf, 128, C.byref(cnt), C.byref(ms))
        out[buf.value.decode()] = (int(cnt.value), float(ms.value))
    return out


class Server:
    """Owns a cspd_server_t and the host buffers of its pending jobs."""

    def __init__(self, handle):
        self.handle = handle
        self.pending = {}

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.cspd_serve_destroy(h)


def cspd_serve_create(device: int = 0, hbm_budget_bytes: int = 16 << 30, max_slots: int = 4) -> Server:
    h = C.c_void_p()
    _check(load().cspd_serve_create(int(device), int(hbm_budget_bytes), int(max_slots), C.byref(h)))
    return Server(h.value)


def cspd_serve_submit(server: Server, plan: Plan, y: np.ndarray, mask: Optional[np.ndarray] = None,
                      k_fine: Optional[np.ndarray] = None, k_fine_uniform: int = 0,
                      k_scale: Sequence[int] = (), full: bool = False, want_coef: bool = True,
                      want_xhat: bool = True, out: Optional[dict] = None) -> int:
    """Queue a job on host arrays; returns its id.  Outputs are collected by
    cspd_serve_poll.  `out` may hold caller-owned output arrays ("support",
    "k_used", and "coef" / "xhat" when wanted; e.g. views of pinned memory);
    the others are allocated here."""
    ndt = np.float64 if plan.dtype == "f64" else np.float32
    y = np.ascontiguousarray(y, dtype=ndt)
    B = y.shape[0]
    if y.shape != (B, plan.m):
        raise ValueError(f"y must be (B, {plan.m})")
    bufs = {"y": y}
    if mask is not None:
        bufs["mask"] = np.ascontiguousarray(mask, dtype=np.uint8)
    if k_fine is not None:
        bufs["k_fine"] = np.ascontiguousarray(k_fine, dtype=np.int32)
    shapes = {"support": ((B, plan.k_max), np.int32), "k_used": ((B,), np.int32)}
    if want_coef:
        shapes["coef"] = ((B, plan.k_max), ndt)
    if want_xhat:
        shapes["xhat"] = ((B, plan.n), ndt)
    out = out or {}
    for name, (shape, dt) in shapes.items():
        a = out.get(name)
        if a is None:
            a = np.empty(shape, dtype=dt)
        elif a.shape != shape or a.dtype != dt or not a.flags.c_contiguous or not a.flags.writeable:
            raise ValueError(f"out[{name!r}] must be a writeable contiguous {shape} {np.dtype(dt).name} array")
        bufs[name] = a
    j = Job()
    j.plan = plan.handle
    j.B = B
    for name in ("y", "mask", "k_fine", "support", "coef", "k_used", "xhat"):
        if name in bufs:
            setattr(j, name, bufs[name].ctypes.data)
    j.k_fine_uniform = int(k_fine_uniform)
    for i, v in enumerate(k_scale):
        j.k_scale[i] = int(v)
    j.full = 1 if full else 0
    jid = C.c_uint64()
    _check(load().cspd_serve_submit(server.handle, C.byref(j), C.byref(jid)))
    server.pending[jid.value] = (bufs, plan)
    return jid.value


def cspd_serve_submit_device(server: Server, plan: Plan, y, mask=None, k_fine=None, k_fine_uniform: int = 0,
                             k_scale: Sequence[int] = (), full: bool = False, support=None, coef=None,
                             k_used=None, xhat=None, want_xhat: bool = True) -> int:
    """Queue a job whose inputs and outputs are device tensors on the
    server's device (run in place, no copies); returns its id.  Outputs not
    passed are allocated here; cspd_serve_poll returns them."""
    _check_inputs(plan, y, mask, k_fine)
    B = y.shape[0]
    support, coef, k_used, xhat = _outputs(plan, B, support, coef, k_used, xhat, want_xhat)
    j = Job()
    j.plan = plan.handle
    j.B = B
    j.y = y.data_ptr()
    j.mask = None if mask is None else mask.data_ptr()
    j.k_fine = None if k_fine is None else k_fine.data_ptr()
    j.k_fine_uniform = int(k_fine_uniform)
    for i, v in enumerate(k_scale):
        j.k_scale[i] = int(v)
    j.full = 1 if full else 0
    j.support = support.data_ptr()
    j.coef = None if coef is None else coef.data_ptr()
    j.k_used = k_used.data_ptr()
    j.xhat = None if xhat is None else xhat.data_ptr()
    j.on_device = 1
    # the server's streams do not wait for the caller's: finish the inputs first
    _torch().cuda.synchronize(y.device)
    jid = C.c_uint64()
    _check(load().cspd_serve_submit(server.handle, C.byref(j), C.byref(jid)))
    bufs = {"y": y, "mask": mask, "k_fine": k_fine, "support": support, "coef": coef, "k_used": k_used,
            "xhat": xhat}
    server.pending[jid.value] = ({k: v for k, v in bufs.items() if v is not None}, plan)
    return jid.value


def cspd_serve_poll(server: Server, job_id: int, timeout_us: int = -1):
    """Returns (outputs dict, stats dict) once the job has finished, or None
    while it is pending (E_BUSY).  Raises on failure or an unknown id."""
    st = JobStats()
    rc = load().cspd_serve_poll(server.handle, C.c_uint64(job_id), int(timeout_us), C.byref(st))
    if rc == E_BUSY:
        return None
    if rc != OK:
        server.pending.pop(job_id, None)
        _check(rc)
    bufs, _plan = server.pending.pop(job_id)
    stats = {f: getattr(st, f) for f, _ in JobStats._fields_}
    out = {k: v for k, v in bufs.items() if k in ("support", "coef", "k_used", "xhat")}
    return out, stats


def cspd_serve_destroy(server: Server):
    h, server.handle = server.handle, None
    if h:
        load().cspd_serve_destroy(h)
    server.pending.clear()
