"""A handle-owning wrapper over the C-ABI: PyTorch allocates the device workspace and the output
tensors and supplies the stream; the library does every step of the method on the GPU."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import binding as B

_FIELD = {"rho": B.PF_LBM_FIELD_RHO, "jx": B.PF_LBM_FIELD_JX, "jy": B.PF_LBM_FIELD_JY, "jz": B.PF_LBM_FIELD_JZ,
          "solid": B.PF_LBM_FIELD_SOLID, "owner": B.PF_LBM_FIELD_OWNER, "psi": B.PF_LBM_FIELD_PSI}


class PfLbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pf_lbm error {code}: {msg}")
        self.code = code


def make_config(params: dict, n_bodies: int, precision: str):
    """pf_lbm_config from a parameter dict (keys of pflbm_inputs.default_params)."""
    cfg = B.PfLbmConfig()
    cfg.struct_size = C.sizeof(B.PfLbmConfig)
    cfg.nx, cfg.ny, cfg.nz = int(params["nx"]), int(params["ny"]), int(params["nz"])
    cfg.lattice = int(params.get("lattice", B.PF_LBM_D3Q19))
    cfg.precision = {"fp64": B.PF_LBM_FP64, "fp32": B.PF_LBM_FP32, "fp16": B.PF_LBM_FP16_STORE}[precision]
    cfg.flags = ((B.PF_LBM_KINETICS if params["kinetics"] else 0) | (B.PF_LBM_MOTION if params["motion"] else 0)
                 | (B.PF_LBM_REPULSION if params["repulsion"] else 0))
    cfg.tau, cfg.G, cfg.rho0 = params["tau"], params["G"], params["rho0"]
    cfg.solid_threshold = params["solid_threshold"]
    cfg.mobility, cfg.eta = params["mobility"], params["eta"]
    sig = np.ascontiguousarray(np.asarray(params["sigma"], dtype=np.float64)[: n_bodies + 1, : n_bodies + 1])
    cfg.sigma = sig.ctypes.data_as(C.POINTER(C.c_double))
    cfg.r_c, cfg.n_exp, cfg.e0 = params["rc"], params["nexp"], params["e0"]
    cfg.R_A = params["RA"]
    for d in range(3):
        cfg.fext[d] = float(params["fext"][d])
    cfg.phi_floor = float(params["phi_floor"])
    return cfg, sig


def make_bodies(bodies: list):
    arr = (B.PfLbmBody * max(len(bodies), 1))()
    for i, b in enumerate(bodies):
        arr[i].mass_density = float(b["mass_density"])
        arr[i].wetting_rho = float(b["wetting_rho"])
        for d in range(3):
            arr[i].v[d] = float(b["v"][d])
            arr[i].w[d] = float(b["w"][d])
        arr[i].fixed = int(b.get("fixed", 0))
    return arr


class Simulation:
    """One simulation on one GPU.  ``params``/``bodies``/``rho0``/``phi0`` as produced by
    :mod:`pflbm_inputs`; ``precision`` 'fp64' or 'fp32'."""

    def __init__(self, params: dict, bodies: list, rho0: np.ndarray, phi0: np.ndarray, precision: str = "fp32",
                 device: str = "cuda", stream: torch.cuda.Stream | None = None):
        self.nb = len(bodies)
        self.shape = tuple(int(v) for v in (params["nz"], params["ny"], params["nx"]))
        self.device = torch.device(device)
        # a stream of its own (default priority): the library captures its step into a HIP graph
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        cfg, sig = make_config(params, self.nb, precision)
        barr = make_bodies(bodies)
        r = np.ascontiguousarray(rho0, dtype=np.float64).reshape(-1)
        p = np.ascontiguousarray(phi0, dtype=np.float64).reshape(-1) if self.nb else None
        rc, _, need = B.pf_lbm_init(cfg, self.nb, barr, r, p, 0, 0, 0)
        if rc != B.PF_LBM_OK:
            raise PfLbmError(rc, B.pf_lbm_last_error(None))
        self.workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        self.ws_bytes = need
        rc, h, _ = B.pf_lbm_init(cfg, self.nb, barr, r, p, self.workspace.data_ptr(), need, self.stream.cuda_stream)
        if rc != B.PF_LBM_OK:
            raise PfLbmError(rc, B.pf_lbm_last_error(None))
        self._h = h
        self._keep = (cfg, sig, barr)

    def close(self):
        if getattr(self, "_h", None):
            B.pf_lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        # at interpreter shutdown the binding module may already be torn down; the process
        # releases the handle with it
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != B.PF_LBM_OK:
            raise PfLbmError(rc, B.pf_lbm_last_error(self._h))

    def step(self, n: int = 1) -> None:
        self._check(B.pf_lbm_step(self._h, n))

    def bodies(self) -> dict:
        rc, F, T, X, V, W = B.pf_lbm_forces(self._h, self.nb)
        self._check(rc)
        return {"F": F, "T": T, "X": X, "V": V, "W": W}

    def field(self, name, dtype=torch.float64) -> torch.Tensor:
        which = B.PF_LBM_FIELD_PHI + int(name[3:]) if isinstance(name, str) and name.startswith("phi") else _FIELD[name]
        out = torch.empty(self.shape, dtype=dtype, device=self.device)
        dt = B.PF_LBM_DST_F64 if dtype == torch.float64 else B.PF_LBM_DST_F32
        self._check(B.pf_lbm_fields(self._h, which, out.data_ptr(), dt))
        self.stream.synchronize()  # the output is written on the library's stream
        return out

    def rho(self) -> np.ndarray:
        return self.field("rho").cpu().numpy()

    def mom(self) -> np.ndarray:
        return np.stack([self.field(k).cpu().numpy() for k in ("jx", "jy", "jz")])

    def phi(self) -> np.ndarray:
        if self.nb == 0:
            return np.zeros((0,) + self.shape)
        return np.stack([self.field(f"phi{a}").cpu().numpy() for a in range(self.nb)])

    def mask(self):
        return (self.field("solid").cpu().numpy().astype(np.int32), self.field("owner").cpu().numpy().astype(np.int32))

    def timing(self, enable: bool):
        rc, out = B.pf_lbm_timing(self._h, 1 if enable else 0)
        self._check(rc)
        return {"steps": int(out[0]), "kernel_ms": out[1], "step_ms": out[2]}

    def force_history(self, max_steps: int = 8192) -> np.ndarray:
        """[n, n_bodies, 6] FP64 force (x, y, z) and torque of the last n steps, oldest first."""
        rc, out = B.pf_lbm_force_history(self._h, max_steps, self.nb)
        self._check(rc)
        return out

    def autotune(self, steps_per_candidate: int = 10) -> dict:
        """Pick the fastest result-invariant launch shapes (advances the simulation)."""
        rc, out = B.pf_lbm_autotune(self._h, steps_per_candidate)
        self._check(rc)
        return {"tile_rows": int(out[0]), "chunk_planes": int(out[1]), "ms_per_step": out[2]}

    def set_tile(self, rows: int, planes: int) -> None:
        """Tile shape of the fluid pass: 64 x rows nodes, z-chunks of planes planes."""
        self._check(B.load_library().pf_lbm_set_tile(self._h, int(rows), int(planes)))

    def set_event_capacity(self, entries: int) -> None:
        """Entries of the per-step conversion event list in use; beyond them a step's conversion
        passes scan the whole phase-field box (same results)."""
        self._check(B.load_library().pf_lbm_set_event_capacity(self._h, int(entries)))

    def diag(self) -> dict:
        rc, out = B.pf_lbm_diagnostics(self._h)
        self._check(rc)
        return {"step": int(out[0]), "n_f2s": int(out[1]), "n_s2f": int(out[2]), "n_lost": int(out[3])}


def step_batch(sims, n_steps: int) -> None:
    """Advance independent simulations (each on its own stream) together: their launches
    interleave so that the kernels of different instances overlap on the GPU."""
    rc = B.pf_lbm_step_batch([s._h for s in sims], n_steps)
    if rc != B.PF_LBM_OK:
        errs = [B.pf_lbm_last_error(s._h) for s in sims]
        raise PfLbmError(rc, "; ".join(e for e in errs if e) or B.pf_lbm_last_error(None))


class Batch:
    """Independent simulations stepped as one captured HIP graph (pf_lbm_batch_*): graph_steps
    steps of every instance per replay.  The simulations must stay alive while the batch is
    used."""

    def __init__(self, sims, graph_steps: int = 2):
        self.sims = list(sims)
        rc, h = B.pf_lbm_batch_create([s._h for s in self.sims], graph_steps)
        if rc != B.PF_LBM_OK:
            raise PfLbmError(rc, B.pf_lbm_last_error(None))
        self._h = h

    def step(self, n: int) -> None:
        rc = B.pf_lbm_batch_step(self._h, n)
        if rc != B.PF_LBM_OK:
            raise PfLbmError(rc, B.pf_lbm_batch_last_error(self._h))

    def close(self):
        if getattr(self, "_h", None):
            B.pf_lbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
