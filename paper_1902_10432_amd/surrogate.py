"""The learned pairwise bridge-force surrogate: a thin wrapper of the pf_mlp C ABI (argument
marshalling only; the network runs in the library's BF16-MFMA kernels)."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import binding as B

MLP_EXPORTED = ("pf_mlp_init", "pf_mlp_num_params", "pf_mlp_set_params", "pf_mlp_get_params", "pf_mlp_forward",
                "pf_mlp_gradients", "pf_mlp_train_step", "pf_mlp_destroy", "pf_mlp_last_error")


class PfMlpConfig(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n_in", C.c_int32), ("hidden", C.c_int32), ("layers", C.c_int32),
                ("max_batch", C.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = B.load_library()
        vp, dp, fp = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_float)
        lib.pf_mlp_init.restype = C.c_int
        lib.pf_mlp_init.argtypes = [C.POINTER(PfMlpConfig), C.c_uint64, vp, C.c_size_t, vp, C.POINTER(vp),
                                    C.POINTER(C.c_size_t)]
        lib.pf_mlp_num_params.restype = C.c_int32
        lib.pf_mlp_num_params.argtypes = [vp]
        lib.pf_mlp_set_params.restype = C.c_int
        lib.pf_mlp_set_params.argtypes = [vp, fp]
        lib.pf_mlp_get_params.restype = C.c_int
        lib.pf_mlp_get_params.argtypes = [vp, fp]
        lib.pf_mlp_forward.restype = C.c_int
        lib.pf_mlp_forward.argtypes = [vp, vp, C.c_int32, vp]
        lib.pf_mlp_gradients.restype = C.c_int
        lib.pf_mlp_gradients.argtypes = [vp, vp, vp, C.c_int32, fp, dp]
        lib.pf_mlp_train_step.restype = C.c_int
        lib.pf_mlp_train_step.argtypes = [vp, vp, vp, C.c_int32, C.c_float, dp]
        lib.pf_mlp_destroy.restype = None
        lib.pf_mlp_destroy.argtypes = [vp]
        lib.pf_mlp_last_error.restype = C.c_char_p
        lib.pf_mlp_last_error.argtypes = [vp]
        _lib = lib
    return _lib


class SurrogateError(RuntimeError):
    pass


class Surrogate:
    """MLP n_in -> hidden x layers -> 1 on one GPU stream; inputs/targets are torch tensors on the
    device, already normalised."""

    def __init__(self, n_in=4, hidden=128, layers=4, max_batch=8192, seed=0, device="cuda", stream=None):
        lib = _load()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        cfg = PfMlpConfig(C.sizeof(PfMlpConfig), n_in, hidden, layers, max_batch)
        need = C.c_size_t(0)
        h = C.c_void_p()
        self._check_init(lib.pf_mlp_init(C.byref(cfg), seed, None, 0, None, C.byref(h), C.byref(need)))
        self.workspace = torch.empty(need.value, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        self._check_init(lib.pf_mlp_init(C.byref(cfg), seed, C.c_void_p(self.workspace.data_ptr()), need.value,
                                         C.c_void_p(self.stream.cuda_stream), C.byref(h), C.byref(need)))
        self._h = h
        self.cfg = (n_in, hidden, layers, max_batch)
        self.n_params = lib.pf_mlp_num_params(h)

    @staticmethod
    def _check_init(rc):
        if rc != B.PF_LBM_OK:
            raise SurrogateError(f"pf_mlp_init {rc}: {_load().pf_mlp_last_error(None).decode()}")

    def _check(self, rc):
        if rc != B.PF_LBM_OK:
            raise SurrogateError(f"pf_mlp {rc}: {_load().pf_mlp_last_error(self._h).decode()}")

    def params(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        self._check(_load().pf_mlp_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def set_params(self, p: np.ndarray) -> None:
        a = np.ascontiguousarray(p, dtype=np.float32)
        self._check(_load().pf_mlp_set_params(self._h, a.ctypes.data_as(C.POINTER(C.c_float))))

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        x = x.to(self.device, torch.float32).contiguous()
        y = torch.empty(x.shape[0], dtype=torch.float32, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(_load().pf_mlp_forward(self._h, C.c_void_p(x.data_ptr()), x.shape[0], C.c_void_p(y.data_ptr())))
        self.stream.synchronize()
        return y

    def gradients(self, x: torch.Tensor, t: torch.Tensor):
        x = x.to(self.device, torch.float32).contiguous()
        t = t.to(self.device, torch.float32).contiguous()
        g = np.empty(self.n_params, dtype=np.float32)
        loss = C.c_double(0.0)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(_load().pf_mlp_gradients(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), x.shape[0],
                                             g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss)))
        return loss.value, g

    def train_step(self, x: torch.Tensor, t: torch.Tensor, lr: float, want_loss: bool = False):
        """One Adam step on device tensors x [n][n_in], t [n] (FP32, contiguous)."""
        loss = C.c_double(0.0)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(_load().pf_mlp_train_step(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), x.shape[0],
                                              float(lr), C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:  # the binding may already be torn down at interpreter shutdown
                _load().pf_mlp_destroy(h)
            except Exception:
                pass
            self._h = None


DEM_EXPORTED = ("pf_dem_init", "pf_dem_evaluate", "pf_dem_step", "pf_dem_state", "pf_dem_pairs",
                "pf_dem_set_overrides", "pf_dem_destroy", "pf_dem_last_error")


class PfDemConfig(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n", C.c_int32), ("max_neighbours", C.c_int32),
                ("max_pairs", C.c_int32), ("box", C.c_double), ("dt", C.c_double), ("density", C.c_double),
                ("k_n", C.c_double), ("gamma_n", C.c_double), ("theta", C.c_double),
                ("liquid_fraction", C.c_double), ("gap_min", C.c_double), ("gap_max", C.c_double),
                ("in_shift", C.c_float * 4), ("in_scale", C.c_float * 4), ("out_shift", C.c_float),
                ("out_scale", C.c_float)]


def _load_dem():
    lib = _load()
    if not getattr(lib, "_dem_ready", False):
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
        lib.pf_dem_init.restype = C.c_int
        lib.pf_dem_init.argtypes = [C.POINTER(PfDemConfig), dp, dp, dp, vp, vp, C.c_size_t, vp, C.POINTER(vp),
                                    C.POINTER(C.c_size_t)]
        lib.pf_dem_evaluate.restype = C.c_int
        lib.pf_dem_evaluate.argtypes = [vp]
        lib.pf_dem_step.restype = C.c_int
        lib.pf_dem_step.argtypes = [vp, C.c_int32]
        lib.pf_dem_state.restype = C.c_int
        lib.pf_dem_state.argtypes = [vp, dp, dp, dp]
        lib.pf_dem_pairs.restype = C.c_int
        lib.pf_dem_pairs.argtypes = [vp, C.c_int32, ip, dp, dp, ip]
        lib.pf_dem_set_overrides.restype = C.c_int
        lib.pf_dem_set_overrides.argtypes = [vp, C.c_int32, ip, dp]
        lib.pf_dem_destroy.restype = None
        lib.pf_dem_destroy.argtypes = [vp]
        lib.pf_dem_last_error.restype = C.c_char_p
        lib.pf_dem_last_error.argtypes = [vp]
        lib._dem_ready = True
    return lib


def dem_config(n, box, dt, density, k_n, gamma_n, theta, liquid_fraction, gap_min, gap_max, norm,
               max_neighbours=32, max_pairs=8192) -> PfDemConfig:
    """norm: dict with in_shift[4], in_scale[4], out_shift, out_scale (network normalisation)."""
    cfg = PfDemConfig()
    cfg.struct_size = C.sizeof(PfDemConfig)
    cfg.n, cfg.max_neighbours, cfg.max_pairs = int(n), int(max_neighbours), int(max_pairs)
    cfg.box, cfg.dt, cfg.density, cfg.k_n, cfg.gamma_n = float(box), float(dt), float(density), float(k_n), float(gamma_n)
    cfg.theta, cfg.liquid_fraction, cfg.gap_min, cfg.gap_max = float(theta), float(liquid_fraction), float(gap_min), float(gap_max)
    for k in range(4):
        cfg.in_shift[k] = float(norm["in_shift"][k])
        cfg.in_scale[k] = float(norm["in_scale"][k])
    cfg.out_shift, cfg.out_scale = float(norm["out_shift"]), float(norm["out_scale"])
    return cfg


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class SphereRun:
    """Many-sphere rigid-body run with surrogate bridge forces (pf_dem.h) on the network's stream."""

    def __init__(self, net: Surrogate, cfg: PfDemConfig, radii, x0, v0):
        lib = _load_dem()
        self.net, self.n = net, cfg.n
        self.max_pairs = cfg.max_pairs
        R = np.ascontiguousarray(radii, dtype=np.float64)
        x = np.ascontiguousarray(x0, dtype=np.float64).reshape(-1)
        v = np.ascontiguousarray(v0, dtype=np.float64).reshape(-1)
        assert R.size == cfg.n and x.size == 3 * cfg.n and v.size == 3 * cfg.n
        need = C.c_size_t(0)
        h = C.c_void_p()
        strm = C.c_void_p(net.stream.cuda_stream)
        self._chk0(lib.pf_dem_init(C.byref(cfg), _dptr(R), _dptr(x), _dptr(v), net._h, None, 0, strm, C.byref(h),
                                   C.byref(need)))
        self.workspace = torch.empty(need.value, dtype=torch.uint8, device=net.device)
        torch.cuda.synchronize(net.device)
        self._chk0(lib.pf_dem_init(C.byref(cfg), _dptr(R), _dptr(x), _dptr(v), net._h,
                                   C.c_void_p(self.workspace.data_ptr()), need.value, strm, C.byref(h), C.byref(need)))
        self._h = h

    @staticmethod
    def _chk0(rc):
        if rc != B.PF_LBM_OK:
            raise SurrogateError(f"pf_dem_init {rc}: {_load_dem().pf_dem_last_error(None).decode()}")

    def _chk(self, rc):
        if rc != B.PF_LBM_OK:
            raise SurrogateError(f"pf_dem {rc}: {_load_dem().pf_dem_last_error(self._h).decode()}")

    def evaluate(self):
        self._chk(_load_dem().pf_dem_evaluate(self._h))

    def step(self, n=1):
        self._chk(_load_dem().pf_dem_step(self._h, int(n)))

    def state(self):
        x, v, f = (np.empty((self.n, 3)) for _ in range(3))
        self._chk(_load_dem().pf_dem_state(self._h, _dptr(x), _dptr(v), _dptr(f)))
        return {"x": x, "v": v, "F": f}

    def pairs(self):
        cnt = C.c_int32(0)
        ij = np.empty((self.max_pairs, 2), dtype=np.int32)
        feat = np.empty((self.max_pairs, 4))
        force = np.empty(self.max_pairs)
        self._chk(_load_dem().pf_dem_pairs(self._h, self.max_pairs, ij.ctypes.data_as(C.POINTER(C.c_int32)),
                                           _dptr(feat), _dptr(force), C.byref(cnt)))
        k = min(cnt.value, self.max_pairs)
        return {"ij": ij[:k].copy(), "features": feat[:k].copy(), "force": force[:k].copy()}

    def set_overrides(self, ij, force):
        ij = np.ascontiguousarray(ij, dtype=np.int32).reshape(-1, 2)
        force = np.ascontiguousarray(force, dtype=np.float64).reshape(-1)
        self._chk(_load_dem().pf_dem_set_overrides(self._h, len(force), ij.ctypes.data_as(C.POINTER(C.c_int32)),
                                                   _dptr(force)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:  # the binding may already be torn down at interpreter shutdown
                _load_dem().pf_dem_destroy(h)
            except Exception:
                pass
            self._h = None
