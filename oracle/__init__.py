"""FP64 CPU oracle for full and cross-scale (zero-tree) OMP -- test infrastructure.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
and never imports it.  The arithmetic lives in ``cspd_oracle.c`` (plain C,
FP64, Householder-QR least squares, OpenMP over independent patches); this
module only compiles it, marshals numpy arrays and returns numpy arrays.

Functions:
  build()                -> path of the compiled shared object
  omp(w_like, ...)       -> dict with supports, coefs, k_used, xhat, trace
  omp_full(...)          -> Algorithm 1 over the finest dictionary
  omp_cross_scale(...)   -> Algorithm 2, chained over all scales
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cspd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
MAX_SCALES = 4
PHI_KINDS = {"identity": 0, "dense": 1, "mask": 2}


class _Model(C.Structure):
    _fields_ = [
        ("n_scales", C.c_int32),
        ("dim", C.c_int32 * MAX_SCALES),
        ("atoms", C.c_int32 * MAX_SCALES),
        ("dict", C.c_void_p * MAX_SCALES),
        ("up_map", C.c_void_p * MAX_SCALES),
        ("phi_kind", C.c_int32),
        ("m", C.c_int32),
        ("phi", C.c_void_p),
        ("n_phases", C.c_int32),
    ]


def build(src: str = _SRC, out: str = _LIB, extra_flags: Sequence[str] = ()) -> str:
    """Compile the oracle with gcc (always recompiles)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-std=c11", "-shared", "-fPIC", *extra_flags, "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_lib_cache = {}


def load(path: str = _LIB):
    if path in _lib_cache:
        return _lib_cache[path]
    if not os.path.exists(path):
        build(out=path)
    lib = C.CDLL(path)
    lib.oracle_omp.restype = C.c_int
    lib.oracle_omp.argtypes = [C.POINTER(_Model), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
    lib.oracle_max_threads.restype = C.c_int
    _lib_cache[path] = lib
    return lib


def max_threads(lib_path: str = _LIB) -> int:
    return int(load(lib_path).oracle_max_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def omp(dims, atoms, dicts, up_maps, phi_kind, m, phi, y, mask, k_scales, k_fine=None,
        full=False, forced=None, kstride=None, with_trace=False, n_threads=0,
        phase=None, lib_path: str = _LIB):
    """Run the oracle on a batch.

    dims/atoms/dicts/up_maps describe the scales (coarse -> fine); dicts[s] is
    a (T_s, N_s) array (atom-contiguous).  y is (B, M); mask (B, N) uint8 or
    None.  k_scales has one K per scale; k_fine (B,) overrides the finest K.
    Returns per-scale supports / coefs (B, S, kstride), k_used (B, S), xhat
    (B, N) and, on request, the per-step trace (B, S, kstride, 4) holding the
    best score, the runner-up score, the picked score and the step-1 maximum.
    """
    lib = load(lib_path)
    S = len(dims)
    keep = []
    md = _Model()
    md.n_scales = S
    for s in range(S):
        md.dim[s] = int(dims[s])
        md.atoms[s] = int(atoms[s])
        d = np.ascontiguousarray(dicts[s], dtype=np.float64)
        assert d.shape == (atoms[s], dims[s])
        keep.append(d)
        md.dict[s] = d.ctypes.data
        if s < S - 1:
            u = np.ascontiguousarray(up_maps[s], dtype=np.int32)
            assert u.shape == (dims[s + 1],)
            keep.append(u)
            md.up_map[s] = u.ctypes.data
    md.phi_kind = PHI_KINDS[phi_kind]
    md.m = int(m)
    md.n_phases = 1
    if phi is not None:
        p = np.ascontiguousarray(phi, dtype=np.float64)
        if p.ndim == 3:                 # one dense operator per phase
            md.n_phases = p.shape[0]
            assert p.shape[1:] == (m, dims[-1])
        keep.append(p)
        md.phi = p.ctypes.data
    y = np.ascontiguousarray(y, dtype=np.float64)
    B = y.shape[0]
    assert y.shape == (B, m)
    if mask is not None:
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
    ks = np.ascontiguousarray(k_scales, dtype=np.int32)
    assert ks.shape == (S,)
    kf = None if k_fine is None else np.ascontiguousarray(k_fine, dtype=np.int32)
    kmax = int(max(ks.max() if S else 0, 0 if kf is None or kf.size == 0 else kf.max(), 1))
    kstride = kmax if kstride is None else kstride
    fz = None
    if forced is not None:
        fz = np.ascontiguousarray(forced, dtype=np.int32)
        assert fz.shape == (B, S, kstride)
    sup = np.full((B, S, kstride), -1, dtype=np.int32)
    cf = np.zeros((B, S, kstride), dtype=np.float64)
    ku = np.zeros((B, S), dtype=np.int32)
    xh = np.zeros((B, dims[-1]), dtype=np.float64)
    tr = np.zeros((B, S, kstride, 4), dtype=np.float64) if with_trace else None
    ph = None
    if phase is not None:
        ph = np.ascontiguousarray(phase, dtype=np.int32)
        assert ph.shape == (B,)
    rc = lib.oracle_omp(C.byref(md), B, _ptr(y), _ptr(mask), _ptr(ks), _ptr(kf), int(bool(full)),
                        _ptr(fz), kstride, _ptr(sup), _ptr(cf), _ptr(ku), _ptr(xh), _ptr(tr),
                        int(n_threads), _ptr(ph))
    if rc != 0:
        raise ValueError("oracle rejected the shapes")
    out = {"supports": sup, "coefs": cf, "k_used": ku, "xhat": xh,
           "support": sup[:, -1], "coef": cf[:, -1], "k_fine_used": ku[:, -1]}
    if with_trace:
        out["trace"] = tr
    return out


def _from_workload(w, **kw):
    kw.setdefault("phase", getattr(w, "phase", None))
    return dict(dims=w.dims, atoms=w.atoms, dicts=w.dicts, up_maps=w.up_maps,
                phi_kind=w.phi_kind, m=w.m, phi=w.phi, y=w.y, mask=w.mask,
                k_scales=w.k_scales, k_fine=w.k_fine, **kw)


def omp_cross_scale(w, **kw):
    """Zero-tree OMP (Algorithm 2 chained over the scales) on a workload."""
    return omp(**_from_workload(w, **kw))


def omp_full(w, **kw):
    """Algorithm 1 over the finest dictionary only, every atom a candidate."""
    return omp(full=True, **_from_workload(w, **kw))


def snr_db(x: np.ndarray, xhat: np.ndarray) -> float:
    """Batch SNR 20 log10(||X|| / ||X - Xhat||) (Section IV-A's definition)."""
    return float(20.0 * np.log10(np.linalg.norm(x) / np.linalg.norm(x - xhat)))
