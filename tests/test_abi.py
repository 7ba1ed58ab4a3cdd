"""The C-ABI library loads, exports every symbol include/cspd.h declares, and
rejects malformed plans before touching a device (CPU only)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1511_05174_amd import cspd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cspd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(cspd_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["cspd_plan", "cspd_omp_full", "cspd_omp_cross_scale", "cspd_serve_submit",
                     "cspd_serve_poll", "cspd_plan_destroy", "cspd_serve_create",
                     "cspd_serve_destroy", "cspd_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = cspd.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(cspd.SIGNATURES), "binding and header disagree"


def _desc(**over):
    rng = np.random.default_rng(0)
    d0 = rng.standard_normal((8, 4))
    d1 = rng.standard_normal((32, 16))
    up = (np.arange(16) // 4).astype(np.int32)
    args = dict(dims=[4, 16], atoms=[8, 32], dicts=[d0, d1], up_maps=[up], phi_kind="identity",
                m=16, phi=None, dtype="f32", k_max=8)
    args.update(over)
    return args


@pytest.mark.parametrize("over,code", [
    (dict(atoms=[8, 30]), cspd.E_SHAPE),                       # T_1 not a multiple of T_0
    (dict(m=12), cspd.E_SHAPE),                                # identity needs M = N
    (dict(phi_kind="dense", m=12, phi=None), cspd.E_INVALID),  # dense without Phi
    (dict(k_max=0), cspd.E_SHAPE),
    (dict(k_max=65), cspd.E_UNSUPPORTED),                     # above the full search's 64
    (dict(k_max=32, dtype="f64"), cspd.E_UNSUPPORTED),        # K > 16: FP32 full search only
    (dict(k_max=32, phi_kind="mask"), cspd.E_UNSUPPORTED),    # ... over a shared operator
    (dict(up_maps=[np.full(16, 7, dtype=np.int32)]), cspd.E_SHAPE),   # outside [0, N_0)
    (dict(up_maps=[np.zeros(16, dtype=np.int32)]), cspd.E_SHAPE),     # not onto
    (dict(dtype="f64", corr_mode="bf16"), cspd.E_INVALID),
    (dict(dims=[1, 1], atoms=[1, 1 << 22], dicts=[np.ones((1, 1)), np.ones((1 << 22, 1))],
          up_maps=[np.zeros(1, dtype=np.int32)], m=1, k_max=1), cspd.E_SHAPE),   # 2^22 children per atom
])
def test_plan_validation(over, code):
    with pytest.raises(cspd.CspdError) as ei:
        cspd.cspd_plan(**_desc(**over))
    assert ei.value.code == code
    assert cspd.cspd_last_error()


def test_version():
    assert "gfx950" in cspd.cspd_version()


def test_one_hip_runtime_in_process():
    """torch and the library share a single HIP runtime instance."""
    import torch  # noqa: F401
    cspd.load()
    maps = open("/proc/self/maps").read().splitlines()
    paths = {l.split()[-1] for l in maps if "libamdhip64" in l}
    assert len(paths) == 1, paths
