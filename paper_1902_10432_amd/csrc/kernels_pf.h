// Phase-field and solid-coupling kernels of the step, all restricted to the box that holds the
// support of every phase field (plus a 3-cell margin): split MC-limited advection with the
// rigid-body update, the multi-phase-field kinetics, reclassification, node conversion and the
// upkeep of the cell words.
#pragma once

#include "device_common.h"
#include "kernels_lbm.h"

namespace pfl {

// monotonized-central slope (van Leer 1977)
template <typename T>
__device__ __forceinline__ T mc_slope(T dl, T dr) {
    if (dl * dr <= T(0)) return T(0);
    const T a = fabs(dl), b = fabs(dr), c = T(0.5) * fabs(dl + dr);
    T m = T(2) * a;
    if (T(2) * b < m) m = T(2) * b;
    if (c < m) m = c;
    return dl > T(0) ? m : -m;
}

// flux through face i+1/2 from the four values i-1, i, i+1, i+2 for velocity u (|u| <= 1):
// u [phi_up +- (1 - |u|) s_up / 2] with the upwind cell's MC slope (second-order, TVD)
template <typename T>
__device__ __forceinline__ T mc_flux(T u, T am1, T a0, T a1, T a2) {
    if (u >= T(0)) return u * (a0 + T(0.5) * (T(1) - u) * mc_slope(a0 - am1, a1 - a0));
    return u * (a1 - T(0.5) * (T(1) + u) * mc_slope(a1 - a0, a2 - a1));
}

// Sum K values of per-block partials part[k * nblk + j] into out[k] with the whole block:
// wave w takes k = w, w + 4, ...; fixed order (deterministic).
__device__ __forceinline__ void block_totals(const double *part, int nblk, int K, double *out) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int k = wave; k < K; k += 4) {
        const double s = wave_sum_array(part + (long long)k * nblk, nblk);
        if (lane == 0) out[k] = s;
    }
    __syncthreads();
}

// One directional sweep (axis AX) of d phi_a/dt = -u_B . grad phi_a in conservative form for
// every body a: phi_i -= F_{i+1/2} - F_{i-1/2}.  The rigid velocity component along the sweep
// does not vary along the sweep line, so the update is exactly conservative.  The bodies' motion
// is that of the rigid-body update of this step (the next table).  The sweep visits the tiles of
// the box, one per block, and on each only the bodies active there (tact, pair form); elsewhere
// its update is the identity.
template <typename T, int AX, int NBMAX>
__global__ __launch_bounds__(256) void k_advect(Prm<T> p, int parity, StepState *st, const BodyDev *__restrict__ next,
                                                const double *__restrict__ src, double *__restrict__ dst,
                                                const uint32_t *__restrict__ tact) {
    __shared__ double lb[PF_LBM_MAX_BODIES][9];  // X, V, W of each body for this sweep
    const int tid = threadIdx.x;
    const int nbod = p.nb;
    // the box words are read first so that their latency overlaps the body-table reads
    int32_t box[6];
    for (int d = 0; d < 6; ++d) box[d] = st->box[parity][d];
    if (tid < nbod)
        for (int d = 0; d < 3; ++d) {
            lb[tid][d] = next[tid].X[d];
            lb[tid][3 + d] = next[tid].V[d];
            lb[tid][6 + d] = next[tid].W[d];
        }
    __syncthreads();
    const TileIter<T> ti(box, p);
    const int n[3] = {p.nx, p.ny, p.nz};
    const long long Np = p.Np;
    const int step = AX == 0 ? 1 : (AX == 1 ? p.nx : p.nx * p.ny);
    const int L = n[AX];
    constexpr int A1 = (AX + 1) % 3, A2 = (AX + 2) % 3;
    const uint32_t pm = pair_mask(nbod);
    uint32_t cfl = 0;
    const int bid = xcd_block(blockIdx.x, gridDim.x);
    for (int tk = bid; tk < ti.total; tk += gridDim.x) {
        int tc[3];
        const int tl = ti.tile(tk, tc);
        uint32_t am = pairs_to_bodies(tact[tl] & pm);  // bodies active on the tile (uniform)
        if (!am) continue;
        int u[3], c[3];
        const bool ok = ti.node(tc, tid, c, u);
        // threads off the grid or the box address node 0 and discard what they load
        const int idx = ok ? c[0] + p.nx * (c[1] + p.ny * c[2]) : 0;
        const int i = ok ? c[AX] : 0;
        // flat indices of the five cells i-2..i+2 along the axis (periodic); cells outside the
        // box hold no phase (the support stays 3 cells inside it through the step) and are not
        // read, so the intermediate buffers need no clearing outside the box
        int off[5];
        bool in[5];
#pragma unroll
        for (int s = -2; s <= 2; ++s) {
            off[s + 2] = idx + (wrap2(i + s, L) - i) * step;
            in[s + 2] = ok && ti.inside(AX, u[AX] + s);
        }
        // the stencils of up to four active phases first, loaded unconditionally (the wrapped
        // indices lie in the grid; values outside the box are masked), so that one memory latency
        // covers the group
        constexpr int G = NBMAX < 4 ? NBMAX : 4;
        while (am) {
            int ag[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                ag[g] = am ? __ffs(am) - 1 : -1;
                am &= am ? am - 1u : 0u;
            }
            double sv[G][5];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const double *s0 = src + (long long)(ag[g] >= 0 ? ag[g] : ag[0]) * Np;
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    const double t = s0[off[q]];
                    sv[g][q] = in[q] ? t : 0.0;
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int a = ag[g];
                if (a < 0) break;
                if (!ok) continue;
                // velocity component along AX at this sweep line
                const double r1 = mimg_r((double)c[A1] - lb[a][A1], n[A1], p.inv_n[A1]);
                const double r2 = mimg_r((double)c[A2] - lb[a][A2], n[A2], p.inv_n[A2]);
                const double uu = lb[a][3 + AX] + (lb[a][6 + A1] * r2 - lb[a][6 + A2] * r1);
                const double vm2 = sv[g][0], vm1 = sv[g][1], v0 = sv[g][2], v1 = sv[g][3], v2 = sv[g][4];
                const double Fp = mc_flux(uu, vm1, v0, v1, v2);
                const double Fm = mc_flux(uu, vm2, vm1, v0, v1);
                dst[(long long)a * Np + idx] = v0 - (Fp - Fm);
                if (fabs(uu) > 1.0 && (vm2 != 0.0 || vm1 != 0.0 || v0 != 0.0 || v1 != 0.0 || v2 != 0.0)) cfl = 1;
            }
        }
    }
    if (cfl) atomicOr(&st->err, 2u);  // rare: only when the input breaks the CFL bound
}

// Multi-phase-field kinetics at one node (Sec. 3.3), explicit Euler: v[a] are the advected solid
// phases at the node, nbv(e, a) the value of phase a at face neighbour e (0..5); phase 0 = fluid
// = 1 - sum of solids.  For nodes where at least two phases are active (above floor_, the
// resolution of "phi > 0", at the node or a face neighbour):
//   dphi_a/dt = sum_{b active, b != a} (M/N) ( sigma_ab (I_a - I_b)
//               + sum_{g active, g != a, b} (sigma_bg - sigma_ag) I_g + pi^2/(4 eta) (h_a - h_b) ),
// I = lap(phi) + (pi^2/eta^2) phi with the 7-point Laplacian, h_fluid = 0 and h_a the volume
// driving term (evaluated from the phase fields at time t, the level the explicit step starts
// from, before the advection sweeps); then each solid phase is clipped to [0, 1] (values below
// floor_ to 0) and the solids are rescaled if their sum exceeds 1.  sg: (NBMAX+1)^2 interface
// energies, hh: driving terms with hh[0] = 0.
template <int NBMAX, typename NbrF>
__device__ __forceinline__ void kinetics_node(const double *v, NbrF nbv, int nbod, const double *sg, const double *hh,
                                              double mu, double vterm, double M, double floor_, double *out) {
    using T = double;
    constexpr int NP = NBMAX + 1;
    T v0[NP];
    T sum0 = T(0);
#pragma unroll
    for (int a = 0; a < NBMAX; ++a) {
        v0[a + 1] = v[a];
        sum0 += v[a];
    }
    v0[0] = T(1) - sum0;
    T lap[NP];
    bool on[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        lap[q] = T(-6) * v0[q];
        on[q] = v0[q] > floor_;
    }
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        T s = T(0);
#pragma unroll
        for (int a = 0; a < NBMAX; ++a) {
            const T w = nbv(e, a);
            s += w;
            lap[a + 1] += w;
            on[a + 1] = on[a + 1] || w > floor_;
        }
        const T vf = T(1) - s;
        lap[0] += vf;
        on[0] = on[0] || vf > floor_;
    }
    int na = 0;
    T I[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        if (q > nbod) on[q] = false;
        I[q] = lap[q] + mu * v0[q];
        na += on[q] ? 1 : 0;
    }
    T tot = T(0);
#pragma unroll
    for (int a = 1; a < NP; ++a) {
        T nv = v0[a];
        if (na >= 2 && on[a]) {
            T rate = T(0);
#pragma unroll
            for (int b = 0; b < NP; ++b) {
                if (b == a || !on[b]) continue;
                T t = sg[a * NP + b] * (I[a] - I[b]);
#pragma unroll
                for (int g = 0; g < NP; ++g) {
                    if (g == a || g == b || !on[g]) continue;
                    t += (sg[b * NP + g] - sg[a * NP + g]) * I[g];
                }
                t += vterm * (hh[a] - hh[b]);
                rate += (M / T(na)) * t;
            }
            nv = v0[a] + rate;
        }
        nv = nv < floor_ ? T(0) : (nv > T(1) ? T(1) : nv);
        out[a - 1] = nv;
        tot += nv;
    }
    if (tot > T(1)) {
#pragma unroll
        for (int a = 0; a < NBMAX; ++a) out[a] /= tot;
    }
}

// Reclassification of the nodes of a phase update and the per-block results the next step
// publishes (publish_step_state): support bounds (unwrapped coordinates), conversion counts,
// per-body solid radius, sum of phi and count of interface nodes phi_floor < phi < 1.
template <int NBMAX>
struct ClassAcc {
    int lo[3], hi[3];
    uint32_t f2s, s2f;
    float rad[NBMAX];
    double vol[NBMAX];
    uint32_t icnt[NBMAX];

    __device__ __forceinline__ ClassAcc() {
        for (int d = 0; d < 3; ++d) {
            lo[d] = INT32_MAX;
            hi[d] = INT32_MIN;
        }
        f2s = s2f = 0;
#pragma unroll
        for (int a = 0; a < NBMAX; ++a) {
            rad[a] = 0.0f;
            vol[a] = 0.0;
            icnt[a] = 0u;
        }
    }

    // Solid iff the fluid fraction 1 - sum phi is below the threshold, owner = argmax phi (lowest
    // index on ties; Sec. 3.2.2).  Updates the cell word (marks a change of side) and returns the
    // event-list entry + 1 of a node that changed side (bit 31: it became solid), else 0.
    // old: the node's cell word, read by the caller ahead of the phase loads
    template <typename PT>
    __device__ __forceinline__ uint32_t node(const Prm<PT> &p, const BodyDev *__restrict__ bodies,
                                             cell_t *__restrict__ mask, int idx, const int *u, const int *c,
                                             const double *out, cell_t old) {
        const int nbod = p.nb;
        double sum = 0.0, best = -1.0;
        int arg = 0;
#pragma unroll
        for (int a = 0; a < NBMAX; ++a) {
            if (a >= nbod) break;
            sum += out[a];
            if (out[a] > best) {
                best = out[a];
                arg = a;
            }
            vol[a] += out[a];
            icnt[a] += (out[a] > p.phi_floor && out[a] < 1.0) ? 1u : 0u;
        }
        const bool solid = nbod > 0 && (1.0 - sum) < p.threshold;
        uint32_t event = 0;
        cell_t m = (old & C_NBMASK) | (solid ? solid_word(arg) : 0u);
        if (solid && !(old & C_SOLID)) {
            m |= C_F2S;
            ++f2s;
            event = ((uint32_t)idx | 0x80000000u) + 1u;
        }
        if (!solid && (old & C_SOLID)) {
            m |= C_S2F;
            ++s2f;
            event = (uint32_t)idx + 1u;
        }
        if (m != old) mask[idx] = m;
        if (solid) {
            // distance of this solid node from its body's centre (bounds the repulsion search)
            const BodyDev &B = bodies[arg];
            const double rx = mimg_r(c[0] - B.X[0], p.nx, p.inv_n[0]), ry = mimg_r(c[1] - B.X[1], p.ny, p.inv_n[1]),
                         rz = mimg_r(c[2] - B.X[2], p.nz, p.inv_n[2]);
            const float r = (float)sqrt(rx * rx + ry * ry + rz * rz) + 1e-3f;
#pragma unroll
            for (int a = 0; a < NBMAX; ++a)
                if (a == arg) rad[a] = fmaxf(rad[a], r);
        }
        if (sum > 0.0)
            for (int d = 0; d < 3; ++d) {
                lo[d] = min(lo[d], u[d]);
                hi[d] = max(hi[d], u[d]);
            }
        return event;
    }

    // whole block (256 threads, uniform call): cpart[blockIdx.x] and the conversion counters
    __device__ void finish(int nbod, StepState *st, ClassifyPart *cpart) {
        __shared__ int32_t sb[4][6];
        __shared__ uint32_t sc[4][2];
        __shared__ float sr[4][NBMAX];
        __shared__ double sv[4][NBMAX];
        __shared__ uint32_t si[4][NBMAX];
        const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
        for (int d = 0; d < 3; ++d) {
            const int l = wave_min(lo[d]), h = wave_max(hi[d]);
            if (lane == 0) {
                sb[wave][d] = l;
                sb[wave][3 + d] = h;
            }
        }
        const uint32_t a2 = (uint32_t)wave_sum((int)f2s), b2 = (uint32_t)wave_sum((int)s2f);
        if (lane == 0) {
            sc[wave][0] = a2;
            sc[wave][1] = b2;
        }
#pragma unroll
        for (int a = 0; a < NBMAX; ++a) {
            if (a >= nbod) break;
            float r = rad[a];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) r = fmaxf(r, __shfl_xor(r, off, 64));
            const double v = wave_sum(vol[a]);
            const int ic = wave_sum((int)icnt[a]);
            if (lane == 0) {
                sr[wave][a] = r;
                sv[wave][a] = v;
                si[wave][a] = (uint32_t)ic;
            }
        }
        __syncthreads();
        if (tid == 0) {
            ClassifyPart cp;
            for (int d = 0; d < 3; ++d) {
                cp.lo[d] = min(min(sb[0][d], sb[1][d]), min(sb[2][d], sb[3][d]));
                cp.hi[d] = max(max(sb[0][3 + d], sb[1][3 + d]), max(sb[2][3 + d], sb[3][3 + d]));
            }
            cp.f2s = sc[0][0] + sc[1][0] + sc[2][0] + sc[3][0];
            cp.s2f = sc[0][1] + sc[1][1] + sc[2][1] + sc[3][1];
            for (int b = 0; b < PF_LBM_MAX_BODIES; ++b) {
                const bool on = b < nbod;
                cp.srad[b] = on ? fmaxf(fmaxf(sr[0][b], sr[1][b]), fmaxf(sr[2][b], sr[3][b])) : 0.0f;
                cp.vol[b] = on ? ((sv[0][b] + sv[1][b]) + sv[2][b]) + sv[3][b] : 0.0;
                cp.icnt[b] = on ? si[0][b] + si[1][b] + si[2][b] + si[3][b] : 0u;
            }
            cpart[blockIdx.x] = cp;
            if (cp.f2s + cp.s2f) {  // rare: nodes of this block changed side
                atomicAdd(&st->n_f2s, (unsigned long long)cp.f2s);
                atomicAdd(&st->n_s2f, (unsigned long long)cp.s2f);
            }
        }
    }
};

// Append event-list entries (entry + 1, 0 = none) of a wave: one atomic per wave that saw a node
// change side (rare).  Called by every lane.
__device__ __forceinline__ void append_events(StepState *st, uint32_t *evlist, uint32_t evcap, uint32_t event) {
    const int lane = threadIdx.x & 63;
    const unsigned long long bal = __ballot(event != 0);
    if (!bal) return;
    uint32_t slot0 = 0;
    if (lane == 0) slot0 = atomicAdd(&st->n_events, (uint32_t)__popcll(bal));
    slot0 = __shfl(slot0, 0, 64);
    if (event) {
        const uint32_t slot = slot0 + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
        if (slot < evcap) evlist[slot] = event - 1u;
    }
}

// Phase update after the advection sweeps, one tile of the box per block and one node per thread,
// on the tiles where some body is active: kinetics (kinetics_node; without kinetics the phases
// pass unchanged), reclassification with the event list, per-block partials, and the tile's new
// state word.  Bodies inactive on the tile hold their tile constant at every node the stencil
// reaches, so their values are taken from the state word instead of memory.  On a tile where
// no body is active nothing changes; the bodies that fill it (phi = 1) add its node count to
// their volume sums.  Face neighbours outside the box hold no phase and are not read.
template <typename PT, int NBMAX>
__global__ __launch_bounds__(256) void k_phase_update(Prm<PT> p, int parity, StepState *st,
                                                      const BodyDev *__restrict__ bodies,
                                                      const double *__restrict__ sigma, const double *__restrict__ src,
                                                      double *__restrict__ dst, cell_t *__restrict__ mask,
                                                      ClassifyPart *__restrict__ cpart, uint32_t *__restrict__ evlist,
                                                      uint32_t evcap, const uint32_t *__restrict__ tact,
                                                      uint4 *__restrict__ tstate) {
    constexpr int NP = NBMAX + 1;
    __shared__ double sg[NP * NP];
    __shared__ double hh[NP];
    const int tid = threadIdx.x;
    const int nbod = p.nb, np1 = nbod + 1;
    // the box words are read first so that their latency overlaps the table reads
    int32_t box[6];
    for (int d = 0; d < 6; ++d) box[d] = st->box[parity][d];
    for (int k = tid; k < NP * NP; k += 256) {
        const int r = k / NP, c = k % NP;
        sg[k] = (r < np1 && c < np1) ? sigma[r * np1 + c] : 0.0;
    }
    if (tid < NP) hh[tid] = (tid == 0 || tid > nbod) ? 0.0 : bodies[tid - 1].h;
    __syncthreads();
    const TileIter<PT> ti(box, p);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const long long Np = p.Np;
    const bool kin = (p.flags & PF_LBM_KINETICS) != 0;
    const double PI = 3.14159265358979323846;
    const double mu = PI * PI / (p.eta * p.eta), vterm = PI * PI / (4.0 * p.eta), M = p.mobility;
    const uint32_t pm = pair_mask(nbod);
    const int wave = tid >> 6, lane = tid & 63;
    ClassAcc<NBMAX> acc;
    const int bid = xcd_block(blockIdx.x, gridDim.x);
    for (int tk = bid; tk < ti.total; tk += gridDim.x) {
        int tc[3];
        const int tl = ti.tile(tk, tc);
        const uint32_t act = tact[tl] & pm;  // uniform
        const uint4 sw = tstate[tl];
        const uint32_t s0 = (sw.x | sw.y) | (sw.z | sw.w);
        if (!act) {
            if (tid == 0) {
                const int cnt = min(TLX, nx - tc[0] * TLX) * min(TLY, ny - tc[1] * TLY) * min(TLZ, nz - tc[2] * TLZ);
#pragma unroll
                for (int a = 0; a < NBMAX; ++a)
                    if (a < nbod && ((s0 >> (2 * a)) & 3u) == 1u) acc.vol[a] += (double)cnt;
            }
            continue;
        }
        uint32_t event = 0, bits = 0;
        int u[3], c[3];
        const bool ok = ti.node(tc, tid, c, u);
        if (ok) {
            const int idx = c[0] + nx * (c[1] + ny * c[2]);
            const cell_t old = mask[idx];  // issued with the phase loads
            double v[NBMAX], out[NBMAX], cst[NBMAX];
            bool on[NBMAX];
#pragma unroll
            for (int a = 0; a < NBMAX; ++a) {
                on[a] = a < nbod && ((act >> (2 * a)) & 1u);
                cst[a] = (a < nbod && ((s0 >> (2 * a)) & 3u) == 1u) ? 1.0 : 0.0;
                v[a] = on[a] ? src[(long long)a * Np + idx] : cst[a];
                out[a] = v[a];
            }
            if (kin) {
                const Nbr nb(c[0], c[1], c[2], nx, ny, nz);
                const int offs[6] = {nb.xp, nb.xm, nb.yp, nb.ym, nb.zp, nb.zm};
                const bool ins[6] = {ti.inside(0, u[0] + 1), ti.inside(0, u[0] - 1), ti.inside(1, u[1] + 1),
                                     ti.inside(1, u[1] - 1), ti.inside(2, u[2] + 1), ti.inside(2, u[2] - 1)};
                kinetics_node<NBMAX>(
                    v,
                    [&](int e, int a) {
                        return on[a] ? (ins[e] ? src[(long long)a * Np + idx + offs[e]] : 0.0) : cst[a];
                    },
                    nbod, sg, hh, mu, vterm, M, p.phi_floor, out);
            }
            // every body is written: a body inactive here keeps its constant, except where the
            // final rescale of the solids moves it by rounding (its state word then shows it)
#pragma unroll
            for (int a = 0; a < NBMAX; ++a)
                if (a < nbod) {
                    dst[(long long)a * Np + idx] = out[a];
                    bits |= (out[a] != 0.0 ? 1u : 0u) << (2 * a);
                    bits |= (out[a] != 1.0 ? 2u : 0u) << (2 * a);
                }
            event = acc.node(p, bodies, mask, idx, u, c, out, old);
        } else if (c[0] < nx && c[1] < ny && c[2] < nz) {
            bits = pm << 1;  // a node of the tile outside the box: every phase is 0 there
        }
        append_events(st, evlist, evcap, event);
        // the state word of this wave's layer of the tile from the new phases
        bits = wave_or(bits);
        if (lane == 0) ((uint32_t *)tstate)[4 * tl + wave] = bits;
        // one tile's loads at a time: letting the next tile's loads move up doubles the registers
        asm volatile("" ::: "memory");
    }
    acc.finish(nbod, st, cpart);
}

// The rigid-body update of Sec. 3.1.1 (one block): the force partials of this step (momentum
// exchange, pseudopotential reaction, repulsion) summed in a fixed order, and the bodies advanced
// from the current table with dt = 1: V += F/M, X += V, omega += I^-1 T, published with F and T in
// the next table, which the later kernels of the step read.  hist: ring of hcap steps of per-body
// force and torque, [step][body][6].
__device__ __forceinline__ void rigid_body_update(int flags, int nbod, StepState *st, const BodyDev *__restrict__ cur,
                                                  BodyDev *__restrict__ next, const double *__restrict__ fpart,
                                                  int fblk, double *__restrict__ hist, int hcap) {
    __shared__ double tot[PF_LBM_MAX_BODIES * 6];
    const int tid = threadIdx.x;
    block_totals(fpart, fblk, nbod * 6, tot);
    if (tid < nbod) {
        const BodyDev &B = cur[tid];
        const double *F = &tot[tid * 6], *Tq = &tot[tid * 6 + 3];
        BodyDev Bn = B;
        bool finite = true;
        const bool move = (flags & PF_LBM_MOTION) && !B.fixed;
        for (int d = 0; d < 3; ++d) Bn.V[d] = move ? B.V[d] + F[d] / B.M : B.V[d];
        for (int d = 0; d < 3; ++d) Bn.X[d] = move ? B.X[d] + Bn.V[d] : B.X[d];
        for (int d = 0; d < 3; ++d)
            Bn.W[d] = move ? B.W[d] + (B.Iinv[3 * d + 0] * Tq[0] + B.Iinv[3 * d + 1] * Tq[1] + B.Iinv[3 * d + 2] * Tq[2])
                           : B.W[d];
        for (int d = 0; d < 3; ++d) {
            Bn.F[d] = F[d];
            Bn.T[d] = Tq[d];
            finite = finite && isfinite(F[d]) && isfinite(Tq[d]) && isfinite(Bn.X[d]) && isfinite(Bn.V[d]) &&
                     isfinite(Bn.W[d]);
        }
        next[tid] = Bn;
        if (!finite) atomicOr(&st->err, 1u);
        if (hist) {
            double *hrow = hist + ((long long)((st->step_no - 1u) % (uint32_t)hcap) * nbod + tid) * 6;
            for (int d = 0; d < 3; ++d) {
                hrow[d] = F[d];
                hrow[3 + d] = Tq[d];
            }
        }
    }
}

// After the force scan: the last block runs the rigid-body update; the others the activity of
// the tiles of this step's box (one thread per tile, see TileIter): hot where the tile or a tile
// within p.trad tiles is mixed or differs from it (thot[parity]); active where hot now or at the
// previous step (tact).  States of tiles outside the box are those of their last visit (zero
// phases unless the support was there), which can only add activity.  tstate: four words per
// tile (one per z-layer of it), ORed.
template <typename T>
__global__ __launch_bounds__(256) void k_tile_activity(Prm<T> p, int parity, StepState *st,
                                                       const uint4 *__restrict__ tstate, uint32_t *__restrict__ thot,
                                                       uint32_t *__restrict__ tact, const BodyDev *__restrict__ cur,
                                                       BodyDev *__restrict__ next, const double *__restrict__ fpart,
                                                       int fblk, double *__restrict__ hist, int hcap) {
    if (blockIdx.x == gridDim.x - 1) {
        rigid_body_update(p.flags, p.nb, st, cur, next, fpart, fblk, hist, hcap);
        return;
    }
    const int nblk = gridDim.x - 1;
    auto word = [&](int t) {
        const uint4 w = tstate[t];
        return (w.x | w.y) | (w.z | w.w);
    };
    const TileIter<T> ti(st->box[parity], p);
    const uint32_t pm = pair_mask(p.nb);
    const int ntl = p.tn[0] * p.tn[1] * p.tn[2];
    // neighbour tile coordinate t + d (|d| <= 2) wrapped into [0, n) (n may be 1 or 2)
    auto wrapt = [](int t, int n) {
        t += t < 0 ? n : 0;
        t += t < 0 ? n : 0;
        t -= t >= n ? n : 0;
        t -= t >= n ? n : 0;
        return t;
    };
    const bool near = p.trad[0] == 1 && p.trad[1] == 1 && p.trad[2] == 1;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < ti.total; k += nblk * 256) {
        int tc[3];
        const int tl = ti.tile(k, tc);
        uint32_t dif = 0;
        if (near) {
            // the 27 words in one round of loads
            int xs[3], ys[3], zs[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                xs[d] = wrapt(tc[0] + d - 1, p.tn[0]);
                ys[d] = p.tn[0] * wrapt(tc[1] + d - 1, p.tn[1]);
                zs[d] = p.tn[0] * p.tn[1] * wrapt(tc[2] + d - 1, p.tn[2]);
            }
            uint32_t w[27];
#pragma unroll
            for (int j = 0; j < 27; ++j) w[j] = word(xs[j % 3] + ys[(j / 3) % 3] + zs[j / 9]);
            const uint32_t s0 = w[13];
#pragma unroll
            for (int j = 0; j < 27; ++j) dif |= (w[j] ^ s0) | (w[j] & (w[j] >> 1) & PAIR_LO);
        } else {
            const uint32_t s0 = word(tl);
            for (int dz = -p.trad[2]; dz <= p.trad[2]; ++dz) {
                const int z = wrapt(tc[2] + dz, p.tn[2]);
                for (int dy = -p.trad[1]; dy <= p.trad[1]; ++dy) {
                    const int y = wrapt(tc[1] + dy, p.tn[1]);
                    for (int dx = -p.trad[0]; dx <= p.trad[0]; ++dx) {
                        const uint32_t s = word(wrapt(tc[0] + dx, p.tn[0]) + p.tn[0] * (y + p.tn[1] * z));
                        dif |= (s ^ s0) | (s & (s >> 1) & PAIR_LO);
                    }
                }
            }
        }
        const uint32_t hot = (dif | (dif >> 1)) & pm;
        thot[(long long)parity * ntl + tl] = hot;
        tact[tl] = hot | (thot[(long long)(parity ^ 1) * ntl + tl] & pm);
    }
}

// State words of every tile from the phase fields (initialisation), and both steps' hot masks set
// (every body active on every tile of the first two steps' boxes).  One tile per block.
template <typename T>
__global__ __launch_bounds__(256) void k_tile_init(Prm<T> p, const double *__restrict__ phi, uint32_t *__restrict__ tstate,
                                                   uint32_t *__restrict__ thot) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ntl = p.tn[0] * p.tn[1] * p.tn[2];
    const uint32_t pm = pair_mask(p.nb);
    for (int tl = blockIdx.x; tl < ntl; tl += gridDim.x) {
        const int tc[3] = {tl % p.tn[0], (tl / p.tn[0]) % p.tn[1], tl / (p.tn[0] * p.tn[1])};
        const int c[3] = {tc[0] * TLX + (tid & 7), tc[1] * TLY + ((tid >> 3) & 7), tc[2] * TLZ + (tid >> 6)};
        uint32_t bits = 0;
        if (c[0] < p.nx && c[1] < p.ny && c[2] < p.nz) {
            const long long idx = c[0] + (long long)p.nx * (c[1] + (long long)p.ny * c[2]);
            for (int a = 0; a < p.nb; ++a) {
                const double v = phi[(long long)a * p.Np + idx];
                bits |= (v != 0.0 ? 1u : 0u) << (2 * a);
                bits |= (v != 1.0 ? 2u : 0u) << (2 * a);
            }
        }
        bits = wave_or(bits);
        if (lane == 0) tstate[4 * tl + wave] = bits;
        if (tid == 0) {
            thot[tl] = pm;
            thot[ntl + tl] = pm;
        }
    }
}

// Classification of the initial phase fields (Sec. 3.2.2): solid iff the fluid fraction
// 1 - sum phi is below the threshold, owner = argmax phi (lowest index on ties).  Each block
// writes to cpart[block] its support bounds (unwrapped coordinates), per-body solid radius, sum
// of phi and count of interface nodes phi_floor < phi < 1, which the first step publishes.  (During
// the run the phase-update kernel classifies.)
template <typename PT>
__global__ __launch_bounds__(256) void k_classify_init(Prm<PT> p, int parity, const StepState *st,
                                                       const BodyDev *__restrict__ bodies,
                                                       const double *__restrict__ phi, cell_t *__restrict__ mask,
                                                       ClassifyPart *cpart) {
    using T = double;
    __shared__ int32_t sb[4][6];
    __shared__ uint32_t sc[4][2];
    __shared__ float sr[4][PF_LBM_MAX_BODIES];
    __shared__ double sv[4][PF_LBM_MAX_BODIES];
    __shared__ uint32_t si[4][PF_LBM_MAX_BODIES];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const BoxIter it(st->box[parity], p.nx, p.ny, p.nz);
    const int nx = p.nx, ny = p.ny, nz = p.nz, nbod = p.nb;
    const long long Np = p.Np;
    int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    uint32_t f2s = 0, s2f = 0;
    float rad[PF_LBM_MAX_BODIES];
    for (int b = 0; b < PF_LBM_MAX_BODIES; ++b) rad[b] = 0.0f;
    // per-body sums accumulate in this wave's LDS slots, in iteration order
    for (int k = tid; k < 4 * PF_LBM_MAX_BODIES; k += 256) {
        (&sv[0][0])[k] = 0.0;
        (&si[0][0])[k] = 0u;
    }
    __syncthreads();
    for (int base = blockIdx.x * 256; base < it.vol; base += gridDim.x * 256) {
        const int k = base + tid;
        const bool valid = k < it.vol;
        int u[3] = {0, 0, 0}, c[3] = {0, 0, 0};
        int idx = 0;
        if (valid) {
            it.cell(k, u, c);
            idx = c[0] + nx * (c[1] + ny * c[2]);
        }
        T sum = T(0), best = T(-1);
        int arg = 0;
        for (int a = 0; a < nbod; ++a) {
            const T v = valid ? phi[(long long)a * Np + idx] : T(0);
            sum += v;
            if (v > best) {
                best = v;
                arg = a;
            }
            const double vs = wave_sum(v);
            const int ic = wave_sum((v > p.phi_floor && v < 1.0) ? 1 : 0);
            if (lane == 0) {
                sv[wave][a] += vs;
                si[wave][a] += (uint32_t)ic;
            }
        }
        if (!valid) continue;
        const bool solid = nbod > 0 && (T(1) - sum) < (T)p.threshold;
        mask[idx] = solid ? solid_word(arg) : 0u;
        if (solid) {
            // distance of this solid node from its body's centre (bounds the repulsion search)
            const BodyDev &B = bodies[arg];
            const double rx = mimg_r(c[0] - B.X[0], nx, p.inv_n[0]), ry = mimg_r(c[1] - B.X[1], ny, p.inv_n[1]),
                         rz = mimg_r(c[2] - B.X[2], nz, p.inv_n[2]);
            const float r = (float)sqrt(rx * rx + ry * ry + rz * rz) + 1e-3f;
            for (int b = 0; b < PF_LBM_MAX_BODIES; ++b)
                if (b == arg) rad[b] = fmaxf(rad[b], r);
        }
        if (sum > T(0)) {
            for (int d = 0; d < 3; ++d) {
                lo[d] = min(lo[d], u[d]);
                hi[d] = max(hi[d], u[d]);
            }
        }
    }
    for (int d = 0; d < 3; ++d) {
        const int l = wave_min(lo[d]), h = wave_max(hi[d]);
        if (lane == 0) {
            sb[wave][d] = l;
            sb[wave][3 + d] = h;
        }
    }
    const uint32_t a2 = (uint32_t)wave_sum((int)f2s), b2 = (uint32_t)wave_sum((int)s2f);
    if (lane == 0) {
        sc[wave][0] = a2;
        sc[wave][1] = b2;
    }
    for (int b = 0; b < nbod; ++b) {
        float r = rad[b];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) r = fmaxf(r, __shfl_xor(r, off, 64));
        if (lane == 0) sr[wave][b] = r;
    }
    __syncthreads();
    if (tid == 0) {
        ClassifyPart cp;
        for (int d = 0; d < 3; ++d) {
            cp.lo[d] = min(min(sb[0][d], sb[1][d]), min(sb[2][d], sb[3][d]));
            cp.hi[d] = max(max(sb[0][3 + d], sb[1][3 + d]), max(sb[2][3 + d], sb[3][3 + d]));
        }
        cp.f2s = sc[0][0] + sc[1][0] + sc[2][0] + sc[3][0];
        cp.s2f = sc[0][1] + sc[1][1] + sc[2][1] + sc[3][1];
        for (int b = 0; b < PF_LBM_MAX_BODIES; ++b) {
            const bool on = b < nbod;
            cp.srad[b] = on ? fmaxf(fmaxf(sr[0][b], sr[1][b]), fmaxf(sr[2][b], sr[3][b])) : 0.0f;
            cp.vol[b] = on ? ((sv[0][b] + sv[1][b]) + sv[2][b]) + sv[3][b] : 0.0;
            cp.icnt[b] = on ? si[0][b] + si[1][b] + si[2][b] + si[3][b] : 0u;
        }
        cpart[blockIdx.x] = cp;
    }
}

// Equilibrium of (rho, u) in direction i (Sec. 3.2.1)
template <typename T, int I, class L>
__device__ __forceinline__ T feq_dir(T rho, T ux, T uy, T uz) {
    const T cu = T(Dir<I, L>::x) * ux + T(Dir<I, L>::y) * uy + T(Dir<I, L>::z) * uz;
    const T uu = ux * ux + uy * uy + uz * uz;
    return Dir<I, L>::template w<T>() * rho * (T(1) + T(3) * cu + T(4.5) * cu * cu - T(1.5) * uu);
}

// The 3x3x3 neighbourhood of a node, its 27 cell words loaded in one round and kept as bit sets
// (bit k for offset k = (dz + 1) 9 + (dy + 1) 3 + (dx + 1); 13 is the node itself), for the
// conversion tests of the gather kernel, which otherwise wait for memory once per neighbour.
struct Nbhd {
    uint32_t f2s_bits = 0, fluid_bits = 0;  // "became solid" mark; not solid
    cell_t centre;
    int x, y, z, nx, ny, nz;
    __device__ __forceinline__ Nbhd(const cell_t *mask, int x_, int y_, int z_, int nx_, int ny_, int nz_)
        : x(x_), y(y_), z(z_), nx(nx_), ny(ny_), nz(nz_) {
        cell_t w[27];
#pragma unroll
        for (int k = 0; k < 27; ++k) w[k] = mask[index(k)];
#pragma unroll
        for (int k = 0; k < 27; ++k) {
            if (w[k] & C_F2S) f2s_bits |= 1u << k;
            if (!(w[k] & C_SOLID)) fluid_bits |= 1u << k;
        }
        centre = w[13];
    }
    __device__ __forceinline__ uint32_t index(int k) const {
        return (uint32_t)(wrapi(x + k % 3 - 1, nx) + nx * (wrapi(y + (k / 3) % 3 - 1, ny) + ny * wrapi(z + k / 9 - 1, nz)));
    }
    // does any of the 26 neighbours with a cell index below `below` carry the "became solid" mark
    // (below = 0xFFFFFFFF: any neighbour)
    __device__ __forceinline__ bool f2s(uint32_t below) const {
        for (uint32_t b = f2s_bits & ~(1u << 13); b; b &= b - 1)
            if (index(__ffs(b) - 1) < below) return true;
        return false;
    }
    // N_F of the centre node that became solid (Sec. 3.2.2): the fluid nodes within R_A, widened
    // to sqrt 2 and then sqrt 3 while it is empty; returns its size (0 if empty) and squared radius
    __device__ __forceinline__ int conversion_radius(double RA, double &r2sel) const {
        const double radii2[3] = {RA * RA, 2.0, 3.0};
        for (int t = 0; t < 3; ++t) {
            if (t > 0 && radii2[t] <= RA * RA + 1e-9) continue;
            uint32_t within = 0;
#pragma unroll
            for (int k = 0; k < 27; ++k) {
                const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
                const int d2 = dx * dx + dy * dy + dz * dz;
                if (d2 > 0 && !(d2 > radii2[t] + 1e-9)) within |= 1u << k;
            }
            const int c = __popc(fluid_bits & within);
            if (c > 0) {
                r2sel = radii2[t];
                return c;
            }
        }
        r2sel = 0.0;
        return 0;
    }
};

// Node conversion at one fluid node r (Sec. 3.2.2): the node gathers, from each neighbour that
// just became solid and whose neighbourhood N_F contains it, f_eq(rho_n, u_n) / |N_F| with
// rho_n, u_n = j_n / rho_n of the converted node's populations; a node that just became fluid
// starts from empty populations.  Sources are only read here (k_post empties them).
// psi: the pseudopotential of this step (reference density of the FP16 form)
template <typename S, class L>
__device__ void gather_receiver(const Prm<ArT<S>> &p, const cell_t *__restrict__ mask, S *f,
                                const ArT<S> *__restrict__ psi, int x, int y, int z, int idx, cell_t m,
                                const Nbhd &nr) {
    using T = ArT<S>;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const long long Np = p.Np;
    constexpr bool H = sizeof(S) == 2;
    const T rr = H ? ref_density(psi[idx], p.rho0) : T(0);
    T acc[L::Q];
    sfor<L::Q>([&](auto I) {
        acc[I] = (m & C_S2F) ? T(0)
                             : pop_get<S>(f[(long long)I * Np + idx], Dir<decltype(I)::value, L>::template w<T>(), rr);
    });
    // sources in increasing offset order; the loop runs per lane over its own sources only (a loop
    // over all 26 offsets would run, in a wave, over the union of its lanes' sources)
    for (uint32_t srcs = nr.f2s_bits & ~(1u << 13); srcs; srcs &= srcs - 1) {
        const int k = __ffs(srcs) - 1;
        const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
        const int d2 = dx * dx + dy * dy + dz * dz;
        const int sx = wrapi(x + dx, nx), sy = wrapi(y + dy, ny), sz = wrapi(z + dz, nz);
        const int n = sx + nx * (sy + ny * sz);
        double r2;
        const int cnt = Nbhd(mask, sx, sy, sz, nx, ny, nz).conversion_radius(p.R_A, r2);
        if (cnt == 0 || d2 > r2 + 1e-9) continue;
        T fs[L::Q];
        const T rn = H ? ref_density(psi[n], p.rho0) : T(0);
        sfor<L::Q>([&](auto I) {
            fs[I] = pop_get<S>(f[(long long)I * Np + n], Dir<decltype(I)::value, L>::template w<T>(), rn);
        });
        T rho = T(0), jx = T(0), jy = T(0), jz = T(0);
        sfor<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            rho += fs[i];
            jx += T(Dir<i, L>::x) * fs[i];
            jy += T(Dir<i, L>::y) * fs[i];
            jz += T(Dir<i, L>::z) * fs[i];
        });
        T vx = T(0), vy = T(0), vz = T(0);
        if (rho > T(0)) {
            vx = jx / rho;
            vy = jy / rho;
            vz = jz / rho;
        }
        const T inv = T(1) / T(cnt);
        sfor<L::Q>([&](auto I) { acc[I] += feq_dir<T, decltype(I)::value, L>(rho, vx, vy, vz) * inv; });
    }
    sfor<L::Q>([&](auto I) {
        f[(long long)I * Np + idx] = pop_put<S>(acc[I], Dir<decltype(I)::value, L>::template w<T>(), rr);
    });
}


// Node conversion, receiving side, after the reclassification of the step.  Usual case: no node
// changed side and the kernel returns at once.  Otherwise the event list drives it: work item
// (event e, neighbour d) handles the fluid node r = e + d when e is the converted node of lowest
// index among r's neighbours (so each receiver is handled once, in a fixed order of its sources),
// and a node that became fluid with no converted neighbour is emptied.  When the list overflowed,
// the whole box is scanned instead.
template <typename S, class L>
__global__ __launch_bounds__(256) void k_convert_gather(Prm<ArT<S>> p, int parity, StepState *st,
                                                        const cell_t *__restrict__ mask, S *f,
                                                        const ArT<S> *__restrict__ psi,
                                                        const uint32_t *__restrict__ evlist, uint32_t evcap) {
    using T = ArT<S>;
    const uint32_t nev = st->n_events;
    if (!nev) return;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const long long Np = p.Np;
    const int gtid = blockIdx.x * 256 + threadIdx.x, gstride = gridDim.x * 256;
    // nodes that became solid with no fluid node in reach of R_A, sqrt 2 or sqrt 3: their content
    // has no receiver and is lost (counted)
    unsigned long long lost = 0;
    if (nev > evcap) {
        const BoxIter it(st->box[parity], nx, ny, nz);
        for (int k = gtid; k < it.vol; k += gstride) {
            int u[3], c[3];
            it.cell(k, u, c);
            const int idx = c[0] + nx * (c[1] + ny * c[2]);
            const cell_t m = mask[idx];
            if (m & C_F2S) {
                double r2;
                if (Nbhd(mask, c[0], c[1], c[2], nx, ny, nz).conversion_radius(p.R_A, r2) == 0) ++lost;
            }
            if (m & C_SOLID) continue;
            const Nbhd nr(mask, c[0], c[1], c[2], nx, ny, nz);
            if (!(m & C_S2F) && !nr.f2s(0xFFFFFFFFu)) continue;
            gather_receiver<S, L>(p, mask, f, psi, c[0], c[1], c[2], idx, m, nr);
        }
        if (lost) atomicAdd(&st->n_lost, lost);  // rare
        return;
    }
    for (int j = gtid; j < (int)nev * 27; j += gstride) {
        const uint32_t ent = evlist[j / 27];
        const int d = j % 27;  // 13 = the event node itself
        const uint32_t e = ent & 0x7FFFFFFFu;
        const int ex = (int)(e % (uint32_t)nx), ey = (int)((e / (uint32_t)nx) % (uint32_t)ny), ez = (int)(e / ((uint32_t)nx * ny));
        if (d == 13) {
            const Nbhd ne(mask, ex, ey, ez, nx, ny, nz);
            double r2;
            if ((ent & 0x80000000u) && ne.conversion_radius(p.R_A, r2) == 0) ++lost;
            // a node that became fluid with no converted neighbour starts empty
            if ((ne.centre & C_S2F) && !ne.f2s(0xFFFFFFFFu)) {
                const T re = sizeof(S) == 2 ? ref_density(psi[e], p.rho0) : T(0);
                sfor<L::Q>([&](auto I) {
                    f[(long long)I * Np + e] = pop_put<S>(T(0), Dir<decltype(I)::value, L>::template w<T>(), re);
                });
            }
            continue;
        }
        if (!(ent & 0x80000000u)) continue;  // only nodes that became solid hand on mass
        const int rx = wrapi(ex + d % 3 - 1, nx), ry = wrapi(ey + (d / 3) % 3 - 1, ny), rz = wrapi(ez + d / 9 - 1, nz);
        const int r = rx + nx * (ry + ny * rz);
        const Nbhd nr(mask, rx, ry, rz, nx, ny, nz);
        const cell_t m = nr.centre;
        if (m & C_SOLID) continue;
        if (nr.f2s(e)) continue;  // a lower-index source handles r
        gather_receiver<S, L>(p, mask, f, psi, rx, ry, rz, r, m, nr);
    }
    if (lost) atomicAdd(&st->n_lost, lost);  // rare
}

// Upkeep of the cell words at one node: node conversion, source side (Sec. 3.2.2) -- a node that
// became solid is emptied (its content was handed on, or counted as lost, by k_convert_gather)
// -- then the neighbour bits (bit i: the node in direction i is solid) are recomputed and the
// event bits cleared.  Only solid bits of neighbours are read,
// which this pass never changes, so repeated visits of one node write the same word.
// empty: 0 never, 1 when the word carries the "became solid" mark (one visit per node), 2 always
// (the caller knows the node became solid).
template <typename S, class L>
__device__ __forceinline__ void refresh_node(const Prm<ArT<S>> &p, cell_t *mask, uint32_t *nbw, S *f, const ArT<S> *psi,
                                             int x, int y, int z, uint32_t idx, int empty) {
    using T = ArT<S>;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    // runtime loops: events are rare, and the kernels that run this keep few registers
    const cell_t m = mask[idx];
    if (empty == 2 || (empty == 1 && (m & C_F2S))) {
        const T rr = sizeof(S) == 2 ? ref_density(psi[idx], p.rho0) : T(0);
#pragma unroll 1
        for (int i = 0; i < L::Q; ++i) {
            const int c2 = kCX[i] * kCX[i] + kCY[i] * kCY[i] + kCZ[i] * kCZ[i];
            f[(long long)i * p.Np + idx] = pop_put<S>(T(0), T(L::wshell[c2]), rr);
        }
    }
    uint32_t bits = 0;
    {
        // the neighbours' words in rounds of nine loads (one latency per round, few registers)
        const Nbr nb(x, y, z, nx, ny, nz);
#pragma unroll 1
        for (int i0 = 1; i0 < L::Q; i0 += 9) {
            cell_t w[9];
#pragma unroll
            for (int j = 0; j < 9; ++j) {
                const int i = i0 + j < L::Q ? i0 + j : 0;  // direction 0: the node itself, ignored
                w[j] = mask[(int)idx + nb.off_rt(i)];
            }
#pragma unroll
            for (int j = 0; j < 9; ++j)
                if (i0 + j < L::Q && (w[j] & C_SOLID)) bits |= 1u << (i0 + j);
        }
    }
    // D3Q19: the bits in the cell word; D3Q27: in the neighbour-bit word
    const cell_t mn = (m & ~(C_F2S | C_S2F | C_NBMASK)) | (L::kBits ? bits : 0u);
    if (mn != m) mask[idx] = mn;
    if constexpr (!L::kBits)
        if (nbw[idx] != bits) nbw[idx] = bits;
}

// Closing work of a step's node conversions, run after the conversion gather: with full != 0
// (initialisation) or an overflowed event list, every node of the box is refreshed; otherwise
// only the nodes whose words can have changed: each event node (emptied if it became solid) and
// the Q - 1 nodes that have it as a neighbour.  Threads gtid (of gstride) take the work in turn.
template <typename S, class L>
__device__ __forceinline__ void post_events(const Prm<ArT<S>> &p, const int32_t *box, uint32_t nev,
                                            cell_t *mask, uint32_t *nbw, S *f, const ArT<S> *psi,
                                            const uint32_t *evlist, uint32_t evcap, int full, int gtid,
                                            int gstride) {
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    if (full || nev > evcap) {
        const BoxIter it(box, nx, ny, nz);
        for (int k = gtid; k < it.vol; k += gstride) {
            int u[3], c[3];
            it.cell(k, u, c);
            refresh_node<S, L>(p, mask, nbw, f, psi, c[0], c[1], c[2], (uint32_t)(c[0] + nx * (c[1] + ny * c[2])),
                               full ? 0 : 1);
        }
    } else {
        // the event node and the Q - 1 nodes whose bit for it may change
        constexpr int NR = L::Q;
        for (int j = gtid; j < (int)nev * NR; j += gstride) {
            const uint32_t ent = evlist[j / NR];
            const int i = j % NR;
            const uint32_t e = ent & 0x7FFFFFFFu;
            const int ex = (int)(e % (uint32_t)nx), ey = (int)((e / (uint32_t)nx) % (uint32_t)ny), ez = (int)(e / ((uint32_t)nx * ny));
            // node whose neighbour in direction i is e
            const int x = wrapi(ex - kCX[i], nx), y = wrapi(ey - kCY[i], ny), z = wrapi(ez - kCZ[i], nz);
            refresh_node<S, L>(p, mask, nbw, f, psi, x, y, z, (uint32_t)(x + nx * (y + ny * z)),
                               (i == 0 && (ent & 0x80000000u)) ? 2 : 0);
        }
    }
}

// Every box node refreshed (initialisation: neighbour bits of the first cell words).
template <typename S, class L>
__global__ __launch_bounds__(256) void k_post(Prm<ArT<S>> p, int parity, StepState *st, cell_t *__restrict__ mask,
                                              uint32_t *nbw, S *f, const ArT<S> *__restrict__ psi) {
    post_events<S, L>(p, st->box[parity], 0u, mask, nbw, f, psi, nullptr, 0u, 1, blockIdx.x * 256 + threadIdx.x,
                      gridDim.x * 256);
}

// Closing work of a step's node conversions, launched after the conversion gather (post_events
// on the step's event list and box): nodes that became solid are emptied (their content was
// handed on by the gather) and the neighbour bits around every event are refreshed, before the
// next step's fluid pass reads them.  Usual case: no node changed side and every thread returns
// at once.  psi: the pseudopotential of this step (reference density of the FP16 form).
template <typename S, class L>
__global__ __launch_bounds__(256) void k_close_events(Prm<ArT<S>> p, int parity, StepState *st, S *f, cell_t *mask,
                                                      uint32_t *nbw, const ArT<S> *__restrict__ psi,
                                                      const uint32_t *__restrict__ evlist, uint32_t evcap) {
    const uint32_t nev = st->n_events;
    if (!nev) return;
    post_events<S, L>(p, st->box[parity], nev, mask, nbw, f, psi, evlist, evcap, 0, blockIdx.x * 256 + threadIdx.x,
                      gridDim.x * 256);
}

// ---- initialisation and read-out helpers ------------------------------------------------------

// phase fields from the FP64 host copy, into both buffers
template <typename T>
__global__ void k_init_phi(Prm<T> p, const double *__restrict__ src, double *__restrict__ a, double *__restrict__ b) {
    const long long total = (long long)p.nb * p.N;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < total; k += (long long)gridDim.x * 256) {
        const long long ph = k / p.N, c = k % p.N;
        const double v = src[k];
        a[ph * p.Np + c] = v;
        b[ph * p.Np + c] = v;
    }
}

// fluid at rest: f = f_eq(rho, 0) = w_i rho on fluid nodes, 0 on solid nodes
// fluid at rest: f = f_eq(rho, 0) = w_i rho on fluid nodes, 0 on solid nodes; psi_init gets the
// pseudopotential of these populations (the reference of the FP16 form for the first step)
template <typename S, class L>
__global__ void k_init_f(Prm<ArT<S>> p, const double *__restrict__ rho, const cell_t *__restrict__ mask,
                         const BodyDev *__restrict__ bodies, ArT<S> *__restrict__ psi_init, S *__restrict__ fa) {
    using T = ArT<S>;
    for (int idx = blockIdx.x * 256 + threadIdx.x; idx < p.N; idx += gridDim.x * 256) {
        const cell_t m = mask[idx];
        const bool solid = (m & C_SOLID) != 0;
        const T r = solid ? T(0) : (T)rho[idx];
        const T ps = solid ? (T)bodies[owner_of(m)].psi_s : -expm1(-r * p.inv_rho0);
        psi_init[idx] = ps;
        const T rr = sizeof(S) == 2 ? ref_density(ps, p.rho0) : T(0);
        sfor<L::Q>([&](auto I) {
            constexpr T w = Dir<decltype(I)::value, L>::template w<T>();
            fa[(long long)I * p.Np + idx] = pop_put<S>(w * r, w, rr);
        });
    }
}

template <typename T>
__global__ void k_zero_mask(Prm<T> p, cell_t *mask) {
    for (int idx = blockIdx.x * 256 + threadIdx.x; idx < p.N; idx += gridDim.x * 256) mask[idx] = 0;
}

template <typename S, typename D, class L>
__global__ void k_fields(Prm<ArT<S>> p, int which, const S *__restrict__ f, const cell_t *__restrict__ mask,
                         const ArT<S> *__restrict__ psi, const double *__restrict__ phi, D *__restrict__ dst) {
    using T = ArT<S>;
    for (int idx = blockIdx.x * 256 + threadIdx.x; idx < p.N; idx += gridDim.x * 256) {
        const cell_t m = mask[idx];
        double out = 0.0;
        if (which >= 16) {
            out = phi[(long long)(which - 16) * p.Np + idx];
        } else if (which == 4) {
            out = (m & C_SOLID) ? 1.0 : 0.0;
        } else if (which == 5) {
            out = (m & C_SOLID) ? (double)owner_of(m) : -1.0;
        } else if (which == 6) {
            out = (double)psi[idx];
        } else if (!(m & C_SOLID)) {
            const T rr = sizeof(S) == 2 ? ref_density(psi[idx], p.rho0) : T(0);
            double s = 0.0;
            sfor<L::Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                const double c = which == 0 ? 1.0 : (which == 1 ? Dir<i, L>::x : (which == 2 ? Dir<i, L>::y : Dir<i, L>::z));
                s += c * (double)pop_get<S>(f[(long long)i * p.Np + idx], Dir<i, L>::template w<T>(), rr);
            });
            out = s;
        }
        dst[idx] = (D)out;
    }
}

}  // namespace pfl
