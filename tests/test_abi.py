"""Host-side checks of the C-ABI library: it loads, exports every entry point the header
declares, sizes its workspace and rejects invalid or unsupported configurations.  None of these
calls touches a GPU (workspace == NULL is the size query)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from pflbm_inputs import plates_bridge, uniform_fluid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    from paper_1902_10432_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_1902_10432_amd import build
        build.build()
    binding.load_library()
    return binding


def test_header_symbols_exported(B):
    hdr = open(os.path.join(ROOT, "include", "pf_lbm.h")).read()
    declared = set(re.findall(r"\b(pf_lbm_[a-z_]+)\s*\(", hdr))
    assert {"pf_lbm_init", "pf_lbm_step", "pf_lbm_forces", "pf_lbm_fields"} <= declared
    lib = C.CDLL(B.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(B.EXPORTED)


def _cfg(B, w, precision="fp64", **over):
    from paper_1902_10432_amd.simulation import make_bodies, make_config
    p = dict(w.params)
    p.update(over)
    cfg, sig = make_config(p, len(w.bodies), precision)
    return cfg, sig, make_bodies(w.bodies)


def test_workspace_query_scales_with_precision(B):
    w = plates_bridge()
    sizes = {}
    for prec in ("fp64", "fp32", "fp16"):
        cfg, sig, bodies = _cfg(B, w, prec)
        rc, _, need = B.pf_lbm_init(cfg, 2, bodies, w.rho0.reshape(-1), w.phi0.reshape(-1), 0, 0, 0)
        assert rc == B.PF_LBM_OK, B.pf_lbm_last_error(None)
        sizes[prec] = need
    N = 32 ** 3
    # two population copies dominate: 2 * 19 * N * sizeof(real)
    assert sizes["fp64"] >= 2 * 19 * N * 8
    assert sizes["fp32"] >= 2 * 19 * N * 4
    assert sizes["fp32"] < 0.6 * sizes["fp64"]
    # FP16 storage halves the population copies again (phase fields stay FP64)
    assert sizes["fp16"] >= 2 * 19 * N * 2
    assert sizes["fp16"] < sizes["fp32"] - 2 * 19 * N * 2 + 4096


@pytest.mark.parametrize("field,value,code", [
    ("tau", 0.5, "EINVAL"), ("rho0", 0.0, "EINVAL"), ("eta", -1.0, "EINVAL"),
    ("RA", 2.5, "EUNSUPPORTED"), ("nx", 0, "EINVAL"), ("solid_threshold", 1.5, "EINVAL"),
])
def test_invalid_configs_rejected(B, field, value, code):
    w = plates_bridge()
    cfg, sig, bodies = _cfg(B, w)
    setattr(cfg, {"RA": "R_A"}.get(field, field), value)
    rc, _, _ = B.pf_lbm_init(cfg, 2, bodies, w.rho0.reshape(-1), w.phi0.reshape(-1), 0, 0, 0)
    assert rc == getattr(B, "PF_LBM_" + code)
    assert B.pf_lbm_last_error(None)


def test_unsupported_lattice_and_precision(B):
    w = uniform_fluid((4, 4, 4))
    cfg, sig, bodies = _cfg(B, w)
    cfg.lattice = 15
    rc, _, _ = B.pf_lbm_init(cfg, 0, bodies, w.rho0.reshape(-1), None, 0, 0, 0)
    assert rc == B.PF_LBM_EUNSUPPORTED and "D3Q27" in B.pf_lbm_last_error(None)
    # D3Q27 is accepted and needs room for 27 populations per node in both copies
    sizes = {}
    for lat in (19, 27):
        cfg.lattice = lat
        rc, _, need = B.pf_lbm_init(cfg, 0, bodies, w.rho0.reshape(-1), None, 0, 0, 0)
        assert rc == B.PF_LBM_OK
        sizes[lat] = need
    assert sizes[27] - sizes[19] >= 2 * 8 * 64 * 8
    cfg.lattice = 19
    cfg.precision = 7
    rc, _, _ = B.pf_lbm_init(cfg, 0, bodies, w.rho0.reshape(-1), None, 0, 0, 0)
    assert rc == B.PF_LBM_EUNSUPPORTED


def test_too_many_bodies_and_abi_size(B):
    w = uniform_fluid((4, 4, 4))
    cfg, sig, bodies = _cfg(B, w)
    rc, _, _ = B.pf_lbm_init(cfg, 17, bodies, w.rho0.reshape(-1), None, 0, 0, 0)
    assert rc == B.PF_LBM_EINVAL
    cfg.struct_size = 8
    rc, _, _ = B.pf_lbm_init(cfg, 0, bodies, w.rho0.reshape(-1), None, 0, 0, 0)
    assert rc == B.PF_LBM_EINVAL and "struct_size" in B.pf_lbm_last_error(None)


def test_small_workspace_rejected(B):
    """A workspace below the queried size is refused before any device work (the pointer is
    never dereferenced on this path)."""
    w = uniform_fluid((4, 4, 4))
    cfg, sig, bodies = _cfg(B, w)
    rc, _, need = B.pf_lbm_init(cfg, 0, bodies, w.rho0.reshape(-1), None, 0, 0, 0)
    assert rc == 0 and need > 0
    rc, _, _ = B.pf_lbm_init(cfg, 0, bodies, w.rho0.reshape(-1), None, 256, need - 1, 0)
    assert rc == B.PF_LBM_ENOMEM


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1902_10432_amd import binding
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(binding.LibraryMissing):
        binding.load_library()


def test_mlp_header_symbols_exported(B):
    from paper_1902_10432_amd import surrogate
    hdr = open(os.path.join(ROOT, "include", "pf_mlp.h")).read()
    declared = set(re.findall(r"\b(pf_mlp_[a-z_]+)\s*\(", hdr))
    lib = C.CDLL(B.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(surrogate.MLP_EXPORTED)


@pytest.mark.parametrize("field,value", [("n_in", 0), ("n_in", 17), ("hidden", 24), ("hidden", 528),
                                         ("layers", 0), ("layers", 9), ("max_batch", 0), ("max_batch", 65537)])
def test_mlp_invalid_configs_rejected(B, field, value):
    from paper_1902_10432_amd import surrogate as S
    lib = S._load()
    cfg = S.PfMlpConfig(C.sizeof(S.PfMlpConfig), 4, 128, 4, 1024)
    need = C.c_size_t(0)
    h = C.c_void_p()
    assert lib.pf_mlp_init(C.byref(cfg), 0, None, 0, None, C.byref(h), C.byref(need)) == B.PF_LBM_OK
    # parameters + gradients + two Adam moments in FP32 and two BF16 weight copies
    n_par = 4 * 128 + 128 + 3 * (128 * 128 + 128) + 128 + 1
    n_w = 4 * 128 + 3 * 128 * 128 + 128
    assert need.value >= 16 * n_par + 4 * n_w + 1024 * 128 * (4 + 2) * 4
    setattr(cfg, field, value)
    rc = lib.pf_mlp_init(C.byref(cfg), 0, None, 0, None, C.byref(h), C.byref(need))
    assert rc == B.PF_LBM_EINVAL
    assert lib.pf_mlp_last_error(None)


def test_dem_header_symbols_exported(B):
    from paper_1902_10432_amd import surrogate
    hdr = open(os.path.join(ROOT, "include", "pf_dem.h")).read()
    declared = set(re.findall(r"\b(pf_dem_[a-z_]+)\s*\(", hdr))
    lib = C.CDLL(B.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(surrogate.DEM_EXPORTED)


_NORM = {"in_shift": [0.0] * 4, "in_scale": [1.0] * 4, "out_shift": 0.0, "out_scale": 1.0}


@pytest.mark.parametrize("field,value", [("n", 1), ("n", 16385), ("max_neighbours", 0), ("max_neighbours", 65),
                                         ("max_pairs", 0), ("dt", 0.0), ("density", -1.0), ("k_n", -1.0),
                                         ("theta", 2.0), ("liquid_fraction", 1.0), ("gap_min", -0.1),
                                         ("gap_max", 0.0)])
def test_dem_invalid_configs_rejected(B, field, value):
    from paper_1902_10432_amd import surrogate as S
    lib = S._load_dem()
    cfg = S.dem_config(100, 50.0, 1.0, 1.0, 1.0, 0.1, 0.5, 0.1, 0.0, 2.0, _NORM)
    need = C.c_size_t(0)
    h = C.c_void_p()
    assert lib.pf_dem_init(C.byref(cfg), None, None, None, None, None, 0, None, C.byref(h), C.byref(need)) == 0
    assert need.value >= 100 * (8 + 3 * 24 + 4 * 32) + 8192 * (8 + 32 + 8 + 16 + 4)
    setattr(cfg, field, value)
    rc = lib.pf_dem_init(C.byref(cfg), None, None, None, None, None, 0, None, C.byref(h), C.byref(need))
    assert rc == B.PF_LBM_EINVAL
    assert lib.pf_dem_last_error(None)
