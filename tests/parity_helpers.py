"""Element-by-element comparison of a GPU simulation (through the C-ABI) with the FP64 oracle.

Every output of the step is asserted:
* fields: relative L2 of density and of each phase field, and the per-node maximum of the
  absolute difference (density over its largest value, phase fields as they are, both in [0, 2));
  momentum density as the L2 of the difference over the L2 of the density (a velocity error in
  lattice units, meaningful also where the fluid is nearly at rest); solid mask and owner exact;
* bodies: force F, torque T, position X, velocity V and angular velocity W.  Each is measured
  against the size that a force error of the bar would reach in the steps taken:
    sF = max(|F_oracle|, force_scale)          sT = max(|T_oracle|, sF * lever)
    sV = max(|V_oracle|, steps * sF / M_min)   sX = steps * sV
    sW = max(|W_oracle|, steps * |I^-1|_max * sT)
  so a relative error e in every step's force and torque keeps each of them below e.
"""
import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def errors(sim, ref, steps, force_scale=0.0, lever=1.0, ref_fields=None):
    """All comparison figures (dict).  ref_fields: a dict of the oracle's outputs taken earlier
    (keys rho, mom, phi, mask, bodies, consts) instead of the live oracle object."""
    if ref_fields is None:
        ref_fields = snapshot(ref)
    r = ref_fields
    out = {}
    rho_g = sim.rho()
    out["rho"] = rel_l2(rho_g, r["rho"])
    out["rho_node"] = float(np.abs(rho_g - r["rho"]).max() / max(np.abs(r["rho"]).max(), 1e-300))
    out["mom"] = float(np.linalg.norm(sim.mom() - r["mom"]) / max(np.linalg.norm(r["rho"]), 1e-300))
    if sim.nb:
        phi_g = sim.phi()
        out["phi"] = rel_l2(phi_g, r["phi"])
        out["phi_node"] = float(np.abs(phi_g - r["phi"]).max())
        sg, so = sim.mask(), r["mask"]
        out["mask_mismatch"] = int((sg[0] != so[0]).sum() + (sg[1] != so[1]).sum())
        bg, bo, c = sim.bodies(), r["bodies"], r["consts"]
        sF = max(np.abs(bo["F"]).max(), force_scale, 1e-300)
        sT = max(np.abs(bo["T"]).max(), sF * lever)
        sV = max(np.abs(bo["V"]).max(), steps * sF / float(np.min(c["M"])))
        sX = steps * sV
        sW = max(np.abs(bo["W"]).max(), steps * float(np.abs(c["Iinv"]).max()) * sT, 1e-300)
        for k, s in (("F", sF), ("T", sT), ("V", sV), ("X", sX), ("W", sW)):
            out[k] = float(np.abs(bg[k] - bo[k]).max() / s)
    log("  " + ", ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in out.items()))
    return out


def snapshot(ref):
    """The oracle's outputs, copied (the oracle object can then be released)."""
    snap = {"rho": ref.rho(), "mom": ref.mom()}
    if ref.nb:
        snap.update(phi=ref.phi(), mask=ref.mask(), bodies=ref.bodies(), consts=ref.body_consts())
    return snap


def check(out, tol_field, tol_force, tol_node, tol_phi=None, tol_mom=None):
    """Assert the figures of errors() against the bars."""
    tol_phi = tol_field if tol_phi is None else tol_phi
    tol_mom = tol_field if tol_mom is None else tol_mom
    assert out["rho"] < tol_field, out
    assert out["rho_node"] < tol_node, out
    assert out["mom"] < tol_mom, out
    if "phi" in out:
        assert out["phi"] < tol_phi, out
        assert out["phi_node"] < tol_node, out
        assert out["mask_mismatch"] == 0, out
        for k in ("F", "T", "V", "X", "W"):
            assert out[k] < tol_force, (k, out)


def compare(sim, ref, steps, tol_field, tol_force, tol_node, force_scale=0.0, lever=1.0, tol_phi=None,
            tol_mom=None):
    out = errors(sim, ref, steps, force_scale=force_scale, lever=lever)
    check(out, tol_field, tol_force, tol_node, tol_phi=tol_phi, tol_mom=tol_mom)
    return out
