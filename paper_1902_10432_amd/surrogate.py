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
            _load().pf_mlp_destroy(h)
            self._h = None
