"""Helpers for the GPU tests: run the HIP path through the C-ABI binding and
bring results back as numpy arrays."""
from __future__ import annotations

import numpy as np

from paper_1511_05174_amd import cspd


def torch_mod():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a visible MI355X")
    return torch


def dtype_of(w_or_name):
    torch = torch_mod()
    name = w_or_name if isinstance(w_or_name, str) else w_or_name.dtype
    return (torch.float64, np.float64) if name == "f64" else (torch.float32, np.float32)


def inputs(w, dtype=None):
    """Device tensors for a workload; also returns the host copy of y in the
    compute precision (the oracle is fed the same rounded measurements)."""
    torch = torch_mod()
    tdt, ndt = dtype_of(dtype or w.dtype)
    y_host = np.ascontiguousarray(w.y.astype(ndt))
    y = torch.from_numpy(y_host).cuda()
    mask = None if w.mask is None else torch.from_numpy(np.ascontiguousarray(w.mask)).cuda()
    kf = None if w.k_fine is None else torch.from_numpy(np.ascontiguousarray(w.k_fine, dtype=np.int32)).cuda()
    return y, mask, kf, y_host.astype(np.float64)


def run_cross(plan, w, k_scales=None, dtype=None):
    torch = torch_mod()
    ks = list(k_scales if k_scales is not None else w.k_scales)
    y, mask, kf, yh = inputs(w, dtype)
    B = y.shape[0]
    ncoarse = int(sum(ks[:-1]))
    sc = torch.full((B, max(ncoarse, 1)), -7, dtype=torch.int32, device=y.device)
    sup, coef, ku, xh = cspd.cspd_omp_cross_scale(plan, y, mask, ks[:-1], kf, ks[-1],
                                                  support_coarse=sc if ncoarse else None)
    torch.cuda.synchronize()
    return dict(support=sup.cpu().numpy(), coef=coef.double().cpu().numpy(),
                k_used=ku.cpu().numpy(), xhat=xh.double().cpu().numpy(),
                support_coarse=sc.cpu().numpy()[:, :ncoarse], y64=yh)


def run_full(plan, w, k=None, dtype=None):
    torch = torch_mod()
    y, mask, kf, yh = inputs(w, dtype)
    kk = w.k_scales[-1] if k is None else k
    sup, coef, ku, xh = cspd.cspd_omp_full(plan, y, mask, kf, kk)
    torch.cuda.synchronize()
    return dict(support=sup.cpu().numpy(), coef=coef.double().cpu().numpy(),
                k_used=ku.cpu().numpy(), xhat=xh.double().cpu().numpy(), y64=yh)


def with_y(w, y64):
    """The workload with its measurements replaced (same dictionaries)."""
    import dataclasses
    return dataclasses.replace(w, y=y64)
