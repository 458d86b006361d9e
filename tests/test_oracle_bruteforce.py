"""Brute-force pin of the whole oracle step on a tiny grid.

An independent, literal re-implementation of one coupled step in Python/NumPy, written from the
paper's equations in a different form from the oracle: push streaming link by link (the
population that would enter a solid node comes back to its own node, Sec. 3.2.2), the Guo term
in its vector form (Sec. 3.2.1), the equilibrium in its cs-form, repulsion over all pairs of solid
nodes (Sec. 3.1.2), advection sweeps with array rolls (Sec. 3.1.1), the multi-phase-field
kinetics summed over all active phase triples (Sec. 3.3), node conversion pushed from each
converted node (Sec. 3.2.2), and body mass, centre and inertia recomputed from the initial phase
fields.  8 x 7 x 9 cells, one moving and rotating body next to a fixed one (inside the repulsion
range), strong density contrasts, fast kinetics: after three steps every population, phase
value, mask entry and body quantity must agree with the oracle to round-off.
"""
import math

import numpy as np
import pytest

from pflbm_inputs import default_params

CS2 = 1.0 / 3.0
PI = math.pi


def d3q19():
    """Rest, the 6 face and the 12 edge neighbours (c_s^2 = 1/3)."""
    c = [(0, 0, 0)]
    for ax in range(3):
        for s in (1, -1):
            v = [0, 0, 0]
            v[ax] = s
            c.append(tuple(v))
    for a, b in ((0, 1), (0, 2), (1, 2)):
        for sa in (1, -1):
            for sb in (1, -1):
                v = [0, 0, 0]
                v[a], v[b] = sa, sb
                c.append(tuple(v))
    c = np.array(c, dtype=np.int64)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    opp = np.array([int(np.where((c == -ci).all(axis=1))[0][0]) for ci in c])
    return c, w, opp


def d3q27():
    """Every c in {-1, 0, 1}^3, with the tensor-product weights w(c) = w1(c_x) w1(c_y) w1(c_z),
    w1(0) = 2/3, w1(+-1) = 1/6 (which gives 8/27, 2/27, 1/54, 1/216 by shell)."""
    c19, _, _ = d3q19()
    corners = [(a, b, d) for a in (1, -1) for b in (1, -1) for d in (1, -1)]
    c = np.concatenate([c19, np.array(corners, dtype=np.int64)])
    w1 = {0: 2.0 / 3.0, 1: 1.0 / 6.0, -1: 1.0 / 6.0}
    w = np.array([w1[int(a)] * w1[int(b)] * w1[int(d)] for a, b, d in c])
    opp = np.array([int(np.where((c == -ci).all(axis=1))[0][0]) for ci in c])
    return c, w, opp


def mimg(d, L):
    return d - L * np.floor(d / L + 0.5)


class Brute:
    def __init__(self, p, bodies, rho0, phi0):
        self.p = p
        self.floor = p["phi_floor"]  # resolution of "phi > 0" (Sec. 3.3)
        self.nz, self.ny, self.nx = rho0.shape
        self.n = np.array([self.nx, self.ny, self.nz])
        self.c, self.w, self.opp = d3q27() if p.get("lattice", 19) == 27 else d3q19()
        self.q = len(self.w)
        self.nb = len(bodies)
        self.phi = phi0.copy()
        self.rho_s = np.array([b["mass_density"] for b in bodies])
        self.wet = np.array([b["wetting_rho"] for b in bodies])
        self.fixed = np.array([b.get("fixed", 0) for b in bodies])
        self.V = np.array([b["v"] for b in bodies], dtype=float)
        self.W = np.array([b["w"] for b in bodies], dtype=float)
        # bodies lie inside the box: plain centroid and inertia of the phase field
        z, y, x = np.meshgrid(np.arange(self.nz), np.arange(self.ny), np.arange(self.nx), indexing="ij")
        self.pos = np.stack([x, y, z], axis=-1).astype(float)          # [nz, ny, nx, 3] as (x, y, z)
        self.M = np.zeros(self.nb)
        self.X = np.zeros((self.nb, 3))
        self.Iinv = np.zeros((self.nb, 3, 3))
        self.Vref = np.zeros(self.nb)
        for b in range(self.nb):
            ph = phi0[b]
            vol = ph.sum()
            self.Vref[b] = vol
            self.M[b] = self.rho_s[b] * vol
            self.X[b] = (ph[..., None] * self.pos).reshape(-1, 3).sum(0) / vol
            r = self.pos - self.X[b]
            I = np.zeros((3, 3))
            for i in range(3):
                for j in range(3):
                    I[i, j] = (self.rho_s[b] * ph * ((i == j) * (r ** 2).sum(-1) - r[..., i] * r[..., j])).sum()
            self.Iinv[b] = np.linalg.inv(I)
        self.solid, self.owner = self.classify()
        self.f = np.zeros(rho0.shape + (self.q,))
        for idx in np.ndindex(rho0.shape):
            if not self.solid[idx]:
                self.f[idx] = self.feq(rho0[idx], np.zeros(3))
        self.n_f2s = self.n_s2f = 0

    # -- helpers ---------------------------------------------------------------------------
    def feq(self, rho, u):
        cu = self.c @ u
        return self.w * rho * (1 + cu / CS2 + cu ** 2 / (2 * CS2 ** 2) - (u @ u) / (2 * CS2))

    def wrap(self, x, y, z):
        return (z % self.nz, y % self.ny, x % self.nx)

    def classify(self):
        s = self.phi.sum(0)
        solid = (1.0 - s) < self.p["solid_threshold"]
        owner = np.where(solid, np.argmax(self.phi, axis=0), -1)
        return solid, owner

    def body_vel(self, b, pt):
        r = mimg(np.asarray(pt, float) - self.X[b], self.n.astype(float))
        return self.V[b] + np.cross(self.W[b], r)

    def lever(self, b, pt):
        return mimg(np.asarray(pt, float) - self.X[b], self.n.astype(float))

    # -- one step --------------------------------------------------------------------------
    def step(self):
        p = self.p
        G, tau = p["G"], p["tau"]
        F = np.zeros((self.nb, 3))
        T = np.zeros((self.nb, 3))
        rho = self.f.sum(-1) * (~self.solid)
        psi = np.where(self.solid, 1 - np.exp(-self.wet[np.maximum(self.owner, 0)] / p["rho0"]),
                       1 - np.exp(-rho / p["rho0"]))
        # pseudopotential force on fluid nodes, reaction on bodies at the link midpoint
        frc = np.zeros(rho.shape + (3,))
        for (z, y, x) in np.ndindex(rho.shape):
            if self.solid[z, y, x]:
                continue
            acc = np.zeros(3)
            for i in range(1, self.q):
                n = self.wrap(x + self.c[i, 0], y + self.c[i, 1], z + self.c[i, 2])
                acc += self.w[i] * psi[n] * self.c[i]
                if self.solid[n]:
                    b = self.owner[n]
                    fb = G * psi[z, y, x] * self.w[i] * psi[n] * self.c[i]
                    F[b] += fb
                    T[b] += np.cross(self.lever(b, (x + 0.5 * self.c[i, 0], y + 0.5 * self.c[i, 1], z + 0.5 * self.c[i, 2])), fb)
            frc[z, y, x] = -G * psi[z, y, x] * acc + np.asarray(p["fext"], float)
        # collision (Guo: (1 - 1/2tau) w_i [(c - v)/cs2 + (c.v) c / cs4] . F)
        fs = np.zeros_like(self.f)
        for idx in np.ndindex(rho.shape):
            if self.solid[idx]:
                continue
            f = self.f[idx]
            r = rho[idx]
            v = (self.c.T @ f + 0.5 * frc[idx]) / r if r > 1e-300 else np.zeros(3)
            guo = (1 - 0.5 / tau) * self.w * (((self.c - v) / CS2 + np.outer(self.c @ v, np.ones(3)) * self.c / CS2 ** 2) @ frc[idx])
            fs[idx] = f - (f - self.feq(r, v)) / tau + guo
        # push streaming, half-way bounce-back from moving walls, mass correction
        fn = np.zeros_like(self.f)
        for (z, y, x) in np.ndindex(rho.shape):
            if self.solid[z, y, x]:
                continue
            fn[z, y, x, 0] += fs[z, y, x, 0]
            for i in range(1, self.q):
                d = self.wrap(x + self.c[i, 0], y + self.c[i, 1], z + self.c[i, 2])
                if not self.solid[d]:
                    fn[d + (i,)] += fs[z, y, x, i]
                    continue
                b = self.owner[d]
                mid = (x + 0.5 * self.c[i, 0], y + 0.5 * self.c[i, 1], z + 0.5 * self.c[i, 2])
                o = self.opp[i]
                g = 2 * rho[z, y, x] * self.w[o] * (self.c[o] @ self.body_vel(b, mid)) / CS2
                back = fs[z, y, x, i] + g
                fn[z, y, x, o] += back
                fn[z, y, x, 0] -= g
                dm = self.c[i] * fs[z, y, x, i] - self.c[o] * back   # momentum handed to the body
                F[b] += dm
                T[b] += np.cross(self.lever(b, mid), dm)
        self.f = fn
        # repulsion over all pairs of solid nodes of different bodies
        if p["repulsion"] and self.nb > 1:
            cells = [idx for idx in np.ndindex(rho.shape) if self.solid[idx]]
            for a_i, ip in enumerate(cells):
                for iq in cells[a_i + 1:]:
                    b1, b2 = self.owner[ip], self.owner[iq]
                    if b1 == b2:
                        continue
                    P = np.array([ip[2], ip[1], ip[0]], float)
                    Q = np.array([iq[2], iq[1], iq[0]], float)
                    d = mimg(P - Q, self.n.astype(float))
                    r = np.linalg.norm(d)
                    if not (0 < r < p["rc"]):
                        continue
                    fp = p["e0"] * (p["nexp"] / p["rc"]) * abs((r - p["rc"]) / p["rc"]) ** (p["nexp"] - 1) * d / r
                    F[b1] += fp
                    T[b1] += np.cross(self.lever(b1, P), fp)
                    F[b2] -= fp
                    T[b2] += np.cross(self.lever(b2, Q), -fp)
        self.F, self.T = F, T
        # rigid bodies, semi-implicit Euler
        if p["motion"]:
            for b in range(self.nb):
                if self.fixed[b]:
                    continue
                self.V[b] += F[b] / self.M[b]
                self.X[b] += self.V[b]
                self.W[b] += self.Iinv[b] @ T[b]
        # volume terms from the phase fields before advection
        h = np.zeros(self.nb + 1)
        for a in range(self.nb):
            cnt = ((self.phi[a] > self.floor) & (self.phi[a] < 1)).sum()
            h[a + 1] = (4 * p["eta"] / PI ** 2) * (self.Vref[a] - self.phi[a].sum()) / cnt if cnt else 0.0
        # advection: split conservative sweeps along x, y, z with MC-limited fluxes
        for a in range(self.nb):
            ph = self.phi[a]
            for ax, arr_ax in ((0, 2), (1, 1), (2, 0)):
                u = np.zeros(ph.shape)
                for idx in np.ndindex(ph.shape):
                    u[idx] = self.body_vel(a, self.pos[idx] * (np.arange(3) != ax))[ax]
                m1, p1, p2 = (np.roll(ph, k, axis=arr_ax) for k in (1, -1, -2))
                def slope(dl, dr):
                    m = np.minimum(np.minimum(2 * abs(dl), 2 * abs(dr)), 0.5 * abs(dl + dr))
                    return np.where(dl * dr <= 0, 0.0, np.sign(dl) * m)
                up = u * (ph + 0.5 * (1 - u) * slope(ph - m1, p1 - ph))
                dn = u * (p1 - 0.5 * (1 + u) * slope(p1 - ph, p2 - p1))
                flux = np.where(u >= 0, up, dn)                 # face i + 1/2
                ph = ph - (flux - np.roll(flux, 1, axis=arr_ax))
            self.phi[a] = ph
        # kinetics
        if p["kinetics"]:
            allp = np.concatenate([(1 - self.phi.sum(0))[None], self.phi])
            sig = np.asarray(p["sigma"], float)
            mu = PI ** 2 / p["eta"] ** 2
            new = self.phi.copy()
            for idx in np.ndindex(rho.shape):
                z, y, x = idx
                nbrs = [self.wrap(x + dx, y + dy, z + dz) for dx, dy, dz in
                        ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))]
                act = [q for q in range(self.nb + 1) if allp[q][idx] > self.floor or any(allp[q][n] > self.floor for n in nbrs)]
                I = {q: sum(allp[q][n] for n in nbrs) - 6 * allp[q][idx] + mu * allp[q][idx] for q in act}
                if len(act) < 2:
                    continue
                for a in act:
                    if a == 0:
                        continue
                    rate = 0.0
                    for b in act:
                        if b == a:
                            continue
                        t = sig[a, b] * (I[a] - I[b]) + PI ** 2 / (4 * p["eta"]) * (h[a] - h[b])
                        t += sum((sig[b, g] - sig[a, g]) * I[g] for g in act if g not in (a, b))
                        rate += p["mobility"] / len(act) * t
                    new[a - 1][idx] += rate
            new = np.where(new < self.floor, 0.0, np.minimum(new, 1.0))
            s = new.sum(0)
            self.phi = np.where(s > 1, new / np.where(s > 1, s, 1), new)
        # reclassification and node conversion, pushed from each converted node
        old_solid = self.solid
        self.solid, self.owner = self.classify()
        add = np.zeros_like(self.f)
        for idx in np.ndindex(rho.shape):
            if old_solid[idx] and not self.solid[idx]:
                self.f[idx] = 0.0
                self.n_s2f += 1
        for (z, y, x) in np.ndindex(rho.shape):
            if old_solid[z, y, x] or not self.solid[z, y, x]:
                continue
            self.n_f2s += 1
            f = self.f[z, y, x]
            r = f.sum()
            u = self.c.T @ f / r if r > 1e-300 else np.zeros(3)
            share = self.feq(r, u)
            for R in (p["RA"], math.sqrt(2), math.sqrt(3)):
                if R < p["RA"]:
                    continue
                nbr = [self.wrap(x + dx, y + dy, z + dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                       if 0 < math.sqrt(dx * dx + dy * dy + dz * dz) <= R + 1e-9]
                nbr = [n for n in nbr if not self.solid[n]]
                if nbr:
                    for n in nbr:
                        add[n] += share / len(nbr)
                    break
        self.f = np.where(self.solid[..., None], 0.0, self.f + add)


def _inputs():
    shape = (9, 7, 8)
    rng = np.random.default_rng(5)
    z, y, x = np.meshgrid(*(np.arange(s) for s in shape), indexing="ij")
    phi = np.zeros((2,) + shape)
    for b, (cx, cy, cz, R) in enumerate(((3.2, 3.1, 4.3, 2.2), (6.0, 3.4, 4.6, 1.4))):
        d = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) - R
        phi[b] = 0.5 * (1 - np.tanh(2 * d / 2.0))
    phi[phi < 1e-2] = 0.0
    s = phi.sum(0)
    phi = np.where(s > 1, phi / np.where(s > 1, s, 1), phi)
    rho = 0.3 + 1.5 * rng.random(shape)
    p = default_params(shape[2], shape[1], shape[0], 2, mobility=0.01, e0=0.3)
    bodies = [dict(mass_density=2.0, wetting_rho=1.2, v=[0.3, -0.2, -0.15], w=[0.01, 0.02, -0.015], fixed=0),
              dict(mass_density=3.0, wetting_rho=0.6, v=[0, 0, 0], w=[0, 0, 0], fixed=1)]
    return p, bodies, rho, phi


@pytest.mark.parametrize("lattice", [19, 27])
def test_whole_step_matches_brute_force(oracle_mod, lattice):
    p, bodies, rho, phi = _inputs()
    p["lattice"] = lattice
    bf = Brute(p, bodies, rho, phi)
    o = oracle_mod.Oracle(p, bodies, rho, phi)
    c_or, _ = o.lattice()
    perm = [int(np.where((bf.c == ci).all(axis=1))[0][0]) for ci in c_or]   # oracle index -> brute index
    assert bf.solid.sum() > 0 and (bf.owner == 1).sum() > 0
    for step in range(3):
        bf.step()
        o.step(1)
        ob = o.bodies()
        for key, mine in (("F", bf.F), ("T", bf.T), ("X", bf.X), ("V", bf.V), ("W", bf.W)):
            scale = max(np.abs(mine).max(), 1e-12)
            assert np.abs(ob[key] - mine).max() < 1e-11 * scale + 1e-15, (step, key, ob[key], mine)
        np.testing.assert_allclose(o.phi(), bf.phi, rtol=0, atol=1e-13)
        solid, owner = o.mask()
        assert np.array_equal(solid.astype(bool), bf.solid)
        assert np.array_equal(np.where(solid > 0, owner, -1), bf.owner)
        np.testing.assert_allclose(o.populations()[..., :], bf.f[..., perm], rtol=0, atol=1e-13)
    d = o.diag()
    assert (d["n_f2s"], d["n_s2f"]) == (bf.n_f2s, bf.n_s2f)
    assert bf.n_f2s > 0 and bf.n_s2f > 0, "the case must exercise both kinds of node conversion"
    assert np.abs(bf.F[0] - 0).max() > 0 and np.abs(ob["F"]).max() > 0
