"""The learned pairwise bridge-force surrogate end to end: training data from the two-sphere bridge
sweep, training on the GPU with the library's own network kernels, and deployment in a many-sphere
rigid-body run whose sampled bridges are re-solved with the full PF-LBM step as error judge and
fallback.

Protocol of a field solve of one bridge (the same for training data and for the judge): two
spheres held fixed at the bridge's gap, the liquid a tanh-smoothed cylinder of the bridge's volume
(Sec. 2.2), the vapour started at BRIDGE_VAPOUR, `steps` PF-LBM steps, and the capillary force
taken as the mean over the last `window` steps of the attraction (F_0 - F_1) . e_x / 2 (an even
number of steps, so the period-2 oscillation of the populations averages out).
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from pflbm_inputs import BRIDGE_VAPOUR, SPHERE_DENSITY, bridge_pair, bridge_sweep_params, random_packing

from .simulation import Simulation, step_batch
from .surrogate import SphereRun, Surrogate, dem_config

GAP_MIN, GAP_MAX = 2.0, 8.0   # surface-gap range of the bridge sweep (lattice units)
MARGIN = 16                   # box length along the axis: 2 (r1 + r2) + gap + MARGIN


def features(r1, r2, gap, v_l, theta_rad):
    """Network features of bridges: (max(gap, GAP_MIN) / R*, R_min / R_max, V_L / R*^3, theta),
    R* = 2 r1 r2 / (r1 + r2); returns (features [k][4], R* [k])."""
    r1, r2, gap, v_l = (np.asarray(a, dtype=np.float64).reshape(-1) for a in (r1, r2, gap, v_l))
    rs = 2.0 * r1 * r2 / (r1 + r2)
    f = np.stack([np.maximum(gap, GAP_MIN) / rs, np.minimum(r1, r2) / np.maximum(r1, r2), v_l / rs ** 3,
                  np.broadcast_to(np.asarray(theta_rad, dtype=np.float64), rs.shape)], axis=1)
    return f, rs


def resolve(cases, steps: int = 2000, window: int = 1000, precision: str = "fp32", vapour: float = BRIDGE_VAPOUR):
    """Field solves of bridges (dicts of bridge_pair's arguments), all instances stepped together;
    returns (attraction per case, workload metadata, timing)."""
    assert steps % 2 == 0 and window % 2 == 0 and 0 < window <= steps
    t0 = time.perf_counter()
    sims, metas = [], []
    for q in cases:
        w = bridge_pair(q["shape"], q["r1"], q["r2"], q["gap"], q["liquid_fraction"], q["theta_deg"],
                        rho_v_init=vapour)
        for b in w.bodies:
            b["fixed"] = 1
        sims.append(Simulation(w.params, w.bodies, w.rho0, w.phi0, precision=precision))
        metas.append(w.meta)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if steps > window:
        step_batch(sims, steps - window)
    step_batch(sims, window)
    F = []
    for s in sims:
        h = s.force_history(window)
        F.append(0.5 * float((h[:, 0, 0] - h[:, 1, 0]).mean()))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    cells = sum(int(np.prod(q["shape"])) for q in cases) * steps
    del sims
    return np.array(F), metas, {"setup_s": t1 - t0, "solve_s": t2 - t1, "cell_updates": cells}


def training_set(n: int = 64, seeds=(0,), steps: int = 2000, window: int = 1000, log=print, **sweep):
    """Features and targets F / R* of the bridge sweep (bridge_sweep_params), solved by the field
    method; the liquid volume feature is the volume actually placed."""
    X, y, stats = [], [], []
    for sd in seeds:
        cases = bridge_sweep_params(n, sd, **sweep)
        F, metas, st = resolve(cases, steps, window)
        f, rs = features([q["r1"] for q in cases], [q["r2"] for q in cases], [q["gap"] for q in cases],
                         [m["liquid_volume"] for m in metas], np.radians([q["theta_deg"] for q in cases]))
        X.append(f)
        y.append(F / rs)
        stats.append(st)
        log(f"sweep seed {sd}: {len(cases)} bridges, {st['cell_updates'] / st['solve_s'] / 1e6:.0f} MLUPS, "
            f"setup {st['setup_s']:.1f} s")
    return np.concatenate(X), np.concatenate(y), stats


def normalisation(X, y):
    mu, sd = X.mean(axis=0), X.std(axis=0)
    sd = np.where(sd > 1e-12, sd, 1.0)
    ys = float(y.std()) or 1.0
    return {"in_shift": mu.tolist(), "in_scale": (1.0 / sd).tolist(), "out_shift": float(y.mean()), "out_scale": ys}


def _inputs(X, norm):
    return ((X - np.asarray(norm["in_shift"], dtype=np.float32).astype(np.float64))
            * np.asarray(norm["in_scale"], dtype=np.float32).astype(np.float64)).astype(np.float32)


def predict(net: Surrogate, X, norm):
    """De-normalised network output f (force / R*) for feature rows X."""
    y = net.forward(torch.from_numpy(_inputs(X, norm)).to(net.device)).cpu().numpy().astype(np.float64)
    return y * float(np.float32(norm["out_scale"])) + float(np.float32(norm["out_shift"]))


def train(X, y, norm, hidden: int = 128, layers: int = 4, steps: int = 600, lr: float = 5e-4, seed: int = 0,
          val_fraction: float = 0.2, check_every: int = 10, log=print):
    """Full-batch Adam on the GPU (pf_mlp_train_step) with a cosine learning-rate decay to lr / 20;
    a seeded split holds out val_fraction of the bridges, and the parameters with the lowest
    validation error are kept (early stopping: with a few hundred bridges, some of which break
    at gaps the scale-free inputs cannot tell apart, longer training fits that noise).  Returns
    (network, report)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = rng.permutation(len(y))
    nval = int(round(val_fraction * len(y)))
    val, tr = perm[:nval], perm[nval:]
    dev = torch.device("cuda")
    net = Surrogate(4, hidden, layers, max_batch=max(len(y), 8192), seed=seed)
    xt = torch.from_numpy(_inputs(X[tr], norm)).to(dev)
    yt = torch.from_numpy(((y[tr] - norm["out_shift"]) / norm["out_scale"]).astype(np.float32)).to(dev)
    first = net.train_step(xt, yt, lr, want_loss=True)
    best = (math.inf, net.params())
    t0 = time.perf_counter()
    for s in range(1, steps):
        a = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * s / steps)))
        net.train_step(xt, yt, a)
        if nval and (s % check_every == 0 or s == steps - 1):
            e = float(np.sqrt(np.mean((predict(net, X[val], norm) - y[val]) ** 2)))
            if e < best[0]:
                best = (e, net.params())
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    if nval:
        net.set_params(best[1])
    last = float(net.gradients(xt, yt)[0])
    rms = lambda idx: float(np.sqrt(np.mean(y[idx] ** 2))) if len(idx) else float("nan")  # noqa: E731
    err = lambda idx: float(np.sqrt(np.mean((predict(net, X[idx], norm) - y[idx]) ** 2))) if len(idx) else float("nan")  # noqa: E731
    const = float(np.sqrt(np.mean((y[val] - y[tr].mean()) ** 2))) if nval else float("nan")
    rep = {"samples": len(y), "train": len(tr), "validation": nval, "loss_first": first, "loss_final": last,
           "train_rmse": err(tr), "val_rmse": err(val), "val_rms": rms(val), "val_rmse_constant": const,
           "train_seconds": t_train, "steps": steps}
    log(f"trained {steps} steps in {t_train:.2f} s: loss {first:.3e} -> {last:.3e}, "
        f"validation RMSE {rep['val_rmse']:.3e} (constant predictor {const:.3e}, RMS {rep['val_rms']:.3e})")
    return net, rep


def deploy(net: Surrogate, norm, n: int = 1000, radius_unit: float = 15.0, liquid_fraction: float = 0.03,
           theta_deg: float = 30.0, steps: int = 1000, judge_every: int = 100, judge_pairs: int = 32,
           judge_box: int = 96, judge_steps: int = 2000, judge_window: int = 1000, dt: float = 5.0,
           density: float = SPHERE_DENSITY, k_n: float = 5.0, gamma_n: float = 270.0, fallback_tol: float = 0.25,
           seed: int = 0, train_data=None, refine_steps: int = 0, refine_lr: float = 2e-4, log=print):
    """Rigid-body run of n spheres (radii U[0.8, 1.2] radius_unit, seeded random packing) with
    network bridge forces.  Every judge_every steps, judge_pairs bridges (seeded choice among
    those whose pair fits the judge box) are re-solved by the field method; their errors are
    recorded, and bridges whose network force is off by more than fallback_tol of
    max(|F_field|, RMS of the judged field forces) take the field force (override) until the next
    judgement.  With train_data = (X, y) and refine_steps > 0 the judged bridges also join the
    training set and the network takes refine_steps Adam steps on the whole set after each
    judgement, so each judgement measures the error on bridges the network has not seen."""
    x0, radii, L = random_packing(n, 0.8 * radius_unit, 1.2 * radius_unit, seed=seed)
    theta = math.radians(theta_deg)
    cfg = dem_config(n, L, dt, density, k_n, gamma_n, theta, liquid_fraction, GAP_MIN, GAP_MAX, norm,
                     max_neighbours=32, max_pairs=8192)
    run = SphereRun(net, cfg, radii, x0, np.zeros_like(x0))
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    rounds = []
    t_steps = 0.0
    refine = train_data is not None and refine_steps > 0
    if refine:
        Xr, yr = np.asarray(train_data[0], dtype=np.float64), np.asarray(train_data[1], dtype=np.float64)
    for s0 in range(0, steps, judge_every):
        torch.cuda.synchronize()
        t = time.perf_counter()
        run.step(judge_every)
        torch.cuda.synchronize()
        t_steps += time.perf_counter() - t
        run.set_overrides(np.zeros((0, 2)), np.zeros(0))
        t = time.perf_counter()
        run.evaluate()
        torch.cuda.synchronize()
        t_eval = time.perf_counter() - t
        pr = run.pairs()
        ij, feat, Fs = pr["ij"], pr["features"], pr["force"]
        if len(ij) == 0:
            rounds.append({"step": s0 + judge_every, "bridges": 0})
            continue
        gaps = feat[:, 0] * (2.0 * radii[ij[:, 0]] * radii[ij[:, 1]] / (radii[ij[:, 0]] + radii[ij[:, 1]]))
        fits = np.nonzero(2 * (radii[ij[:, 0]] + radii[ij[:, 1]]) + gaps + MARGIN <= judge_box)[0]
        pick = np.sort(rng.choice(fits, min(judge_pairs, len(fits)), replace=False))
        cases = [{"shape": (judge_box,) * 3, "r1": float(radii[ij[k, 0]]), "r2": float(radii[ij[k, 1]]),
                  "gap": float(gaps[k]), "liquid_fraction": liquid_fraction, "theta_deg": theta_deg} for k in pick]
        Fp, _, st = resolve(cases, judge_steps, judge_window)
        d = Fs[pick] - Fp
        scale = max(float(np.sqrt(np.mean(Fp ** 2))), 1e-12)
        bad = np.abs(d) > fallback_tol * np.maximum(np.abs(Fp), scale)
        run.set_overrides(ij[pick][bad], Fp[bad])
        t_refine = 0.0
        if refine:
            # the judged bridges join the training set (F / R*), then a short refinement
            rs = 2.0 * radii[ij[pick, 0]] * radii[ij[pick, 1]] / (radii[ij[pick, 0]] + radii[ij[pick, 1]])
            Xr = np.concatenate([Xr, feat[pick]])
            yr = np.concatenate([yr, Fp / rs])
            dev = net.device
            xt = torch.from_numpy(_inputs(Xr, norm)).to(dev)
            yt = torch.from_numpy(((yr - norm["out_shift"]) / norm["out_scale"]).astype(np.float32)).to(dev)
            t = time.perf_counter()
            for _ in range(refine_steps):
                net.train_step(xt, yt, refine_lr)
            torch.cuda.synchronize()
            t_refine = time.perf_counter() - t
        x = run.state()["x"]
        rec = {"step": s0 + judge_every, "bridges": int(len(ij)), "judged": int(len(pick)),
               "rmse": float(np.sqrt(np.mean(d ** 2))), "rms_field": scale, "mae": float(np.abs(d).mean()),
               "fallbacks": int(bad.sum()), "surrogate_eval_s": t_eval, "field_solve_s": st["solve_s"],
               "field_setup_s": st["setup_s"], "field_mlups": st["cell_updates"] / st["solve_s"] / 1e6,
               "mean_coordination": 2.0 * len(ij) / n, "x_finite": bool(np.isfinite(x).all()),
               "refine_s": t_refine}
        rounds.append(rec)
        log(f"step {rec['step']}: {rec['bridges']} bridges, judged {rec['judged']}: RMSE {rec['rmse']:.3e} "
            f"(field RMS {scale:.3e}), {rec['fallbacks']} fallbacks; network {t_eval * 1e3:.2f} ms for all "
            f"bridges, field {st['solve_s']:.2f} s for {len(pick)}")
    judged = [r for r in rounds if r.get("judged")]
    per_pair_net = float(np.mean([r["surrogate_eval_s"] / r["bridges"] for r in judged]))
    per_pair_field = float(np.mean([r["field_solve_s"] / r["judged"] for r in judged]))
    half = len(judged) // 2
    rel = [r["rmse"] / r["rms_field"] for r in judged]
    summary = {"spheres": n, "box": L, "radius_unit": radius_unit, "liquid_fraction": liquid_fraction,
               "refine_steps": refine_steps if refine else 0,
               "rel_rmse_first_half": float(np.mean(rel[:half])) if half else float("nan"),
               "rel_rmse_second_half": float(np.mean(rel[half:])) if judged else float("nan"),
               "theta_deg": theta_deg, "steps": steps, "dt": dt, "step_seconds": t_steps,
               "rmse": float(np.sqrt(np.mean([r["rmse"] ** 2 for r in judged]))),
               "rms_field": float(np.sqrt(np.mean([r["rms_field"] ** 2 for r in judged]))),
               "fallbacks": int(sum(r["fallbacks"] for r in judged)),
               "judged": int(sum(r["judged"] for r in judged)),
               "seconds_per_bridge_network": per_pair_net, "seconds_per_bridge_field": per_pair_field,
               "speedup_per_bridge": per_pair_field / per_pair_net, "rounds": rounds}
    return summary
