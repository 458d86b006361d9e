// Phase-field and solid-coupling kernels of the step, all restricted to the box that holds the
// support of every phase field (plus a 3-cell margin): split MC-limited advection, the
// multi-phase-field kinetics, reclassification, node conversion and solid-solid repulsion.
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

// One directional sweep (axis AX) of d phi_a/dt = -u_B . grad phi_a in conservative form for
// every body a: phi_i -= F_{i+1/2} - F_{i-1/2}.  The rigid velocity component along the sweep
// does not vary along the sweep line, so the update is exactly conservative.  The last sweep
// (AX = 2) also sums phi_a and counts its interface nodes 0 < phi_a < 1 for the volume term;
// the last block turns them into h_a = (4 eta/pi^2)(V_ref - V)/|interface| (Sec. 3.3).
template <typename T, int AX>
__global__ __launch_bounds__(256) void k_advect(Prm<T> p, int parity, StepState *st, BodyDev *bodies,
                                                const T *__restrict__ src, T *__restrict__ dst, double *vpart) {
    __shared__ double red[4][PF_LBM_MAX_BODIES][2];
    __shared__ uint32_t ticket;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int nbod = p.nb;
    if (AX == 2) {
        for (int k = tid; k < 4 * PF_LBM_MAX_BODIES * 2; k += 256) (&red[0][0][0])[k] = 0.0;
        __syncthreads();
    }
    const int32_t *bx = st->box[parity];
    const long long vol = box_volume(bx);
    const int n[3] = {p.nx, p.ny, p.nz};
    const long long Np = p.Np;
    const long long stride = (long long)gridDim.x * 256;
    uint32_t cfl = 0;
    for (long long base = (long long)blockIdx.x * 256; base < vol; base += stride) {
        const long long k = base + tid;
        const bool valid = k < vol;
        int c[3] = {0, 0, 0}, idx = 0, step = 1, L = n[AX];
        if (valid) {
            int u3[3];
            box_cell(bx, k, u3[0], u3[1], u3[2]);
            for (int d = 0; d < 3; ++d) c[d] = wrapi(u3[d], n[d]);
            idx = c[0] + p.nx * (c[1] + p.ny * c[2]);
            step = AX == 0 ? 1 : (AX == 1 ? p.nx : p.nx * p.ny);
        }
        const int i = c[AX];
        // flat indices of the five cells i-2..i+2 along the axis (periodic)
        int off[5];
#pragma unroll
        for (int s = -2; s <= 2; ++s) off[s + 2] = idx + (wrapi(i + s, L) - i) * step;
        for (int a = 0; a < nbod; ++a) {
            double vsum = 0.0, cnt = 0.0;
            if (valid) {
                const BodyDev &B = bodies[a];
                // velocity component along AX at this sweep line
                const double r1 = mimg((double)c[(AX + 1) % 3] - B.X[(AX + 1) % 3], n[(AX + 1) % 3]);
                const double r2 = mimg((double)c[(AX + 2) % 3] - B.X[(AX + 2) % 3], n[(AX + 2) % 3]);
                const double ud = B.V[AX] + (B.W[(AX + 1) % 3] * r2 - B.W[(AX + 2) % 3] * r1);
                const T u = (T)ud;
                const T *s0 = src + (long long)a * Np;
                const T vm2 = s0[off[0]], vm1 = s0[off[1]], v0 = s0[off[2]], v1 = s0[off[3]], v2 = s0[off[4]];
                const T Fp = mc_flux(u, vm1, v0, v1, v2);
                const T Fm = mc_flux(u, vm2, vm1, v0, v1);
                const T nv = v0 - (Fp - Fm);
                dst[(long long)a * Np + idx] = nv;
                if (fabs(ud) > 1.0 && (vm2 != T(0) || vm1 != T(0) || v0 != T(0) || v1 != T(0) || v2 != T(0))) cfl = 1;
                vsum = (double)nv;
                cnt = (nv > T(0) && nv < T(1)) ? 1.0 : 0.0;
            }
            if (AX == 2) {
                const double s = wave_sum(vsum), q = wave_sum(cnt);
                if (lane == 0) {
                    red[wave][a][0] += s;
                    red[wave][a][1] += q;
                }
            }
        }
    }
    if (cfl) atomicOr(&st->err, 2u);
    if (AX != 2) return;
    __syncthreads();
    for (int k = tid; k < nbod * 2; k += 256) {
        const int a = k / 2, c = k % 2;
        vpart[((long long)blockIdx.x * nbod + a) * 2 + c] = ((red[0][a][c] + red[1][a][c]) + red[2][a][c]) + red[3][a][c];
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) ticket = atomicAdd(&st->done[1], 1u);
    __syncthreads();
    if (ticket != gridDim.x - 1) return;
    __threadfence();
    if (tid < nbod) {
        double v = 0.0, q = 0.0;
        for (int j = 0; j < (int)gridDim.x; ++j) {
            v += vpart[((long long)j * nbod + tid) * 2];
            q += vpart[((long long)j * nbod + tid) * 2 + 1];
        }
        const double PI = 3.14159265358979323846;
        bodies[tid].h = q > 0.0 ? (4.0 * p.eta / (PI * PI)) * (bodies[tid].Vref - v) / q : 0.0;
    }
    if (tid == 0) st->done[1] = 0;
}

// Multi-phase-field kinetics (Sec. 3.3), explicit Euler, for nodes where at least two phases are
// active (present at the node or a face neighbour; phase 0 = fluid = 1 - sum of solids):
//   dphi_a/dt = sum_{b active, b != a} (M/N) ( sigma_ab (I_a - I_b)
//               + sum_{g active, g != a, b} (sigma_bg - sigma_ag) I_g + pi^2/(4 eta) (h_a - h_b) ),
//   I = lap(phi) + (pi^2/eta^2) phi with the 7-point Laplacian, h_fluid = 0.
// Then each solid phase is clipped to [0, 1] and the solids are rescaled if their sum exceeds 1.
// Without kinetics the kernel copies the advected fields.  src -> dst over the box.
template <typename T, int NBMAX>
__global__ __launch_bounds__(256) void k_kinetics(Prm<T> p, int parity, const StepState *st,
                                                  const BodyDev *__restrict__ bodies, const double *__restrict__ sigma,
                                                  const T *__restrict__ src, T *__restrict__ dst) {
    constexpr int NP = NBMAX + 1;
    __shared__ double sg[NP * NP];
    __shared__ double hh[NP];
    const int nbod = p.nb, np1 = nbod + 1;
    for (int k = threadIdx.x; k < np1 * np1; k += 256) sg[(k / np1) * NP + (k % np1)] = sigma[k];
    if (threadIdx.x < np1) hh[threadIdx.x] = threadIdx.x == 0 ? 0.0 : bodies[threadIdx.x - 1].h;
    __syncthreads();
    const int32_t *bx = st->box[parity];
    const long long vol = box_volume(bx);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const long long Np = p.Np;
    const bool kin = (p.flags & 1) != 0;
    const T PI = T(3.14159265358979323846);
    const T mu = PI * PI / (T)(p.eta * p.eta);
    const T vterm = PI * PI / (T)(4.0 * p.eta);
    const T M = (T)p.mobility;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < vol; k += (long long)gridDim.x * 256) {
        int ux, uy, uz;
        box_cell(bx, k, ux, uy, uz);
        const int x = wrapi(ux, nx), y = wrapi(uy, ny), z = wrapi(uz, nz);
        const int idx = x + nx * (y + ny * z);
        T v0[NP];
#pragma unroll
        for (int a = 0; a < NBMAX; ++a) v0[a + 1] = a < nbod ? src[(long long)a * Np + idx] : T(0);
        if (!kin) {
#pragma unroll
            for (int a = 0; a < NBMAX; ++a)
                if (a < nbod) dst[(long long)a * Np + idx] = v0[a + 1];
            continue;
        }
        const Nbr nb(x, y, z, nx, ny, nz);
        const int offs[6] = {nb.xp, nb.xm, nb.yp, nb.ym, nb.zp, nb.zm};
        T sum0 = T(0);
#pragma unroll
        for (int a = 0; a < NBMAX; ++a) sum0 += v0[a + 1];
        v0[0] = T(1) - sum0;
        T lap[NP];
        bool on[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            lap[q] = T(-6) * v0[q];
            on[q] = v0[q] > T(0);
        }
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            T s = T(0);
#pragma unroll
            for (int a = 0; a < NBMAX; ++a) {
                const T v = a < nbod ? src[(long long)a * Np + idx + offs[e]] : T(0);
                s += v;
                lap[a + 1] += v;
                on[a + 1] = on[a + 1] || v > T(0);
            }
            const T vf = T(1) - s;
            lap[0] += vf;
            on[0] = on[0] || vf > T(0);
        }
        int na = 0;
        T I[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            if (q > nbod) on[q] = false;
            I[q] = lap[q] + mu * v0[q];
            na += on[q] ? 1 : 0;
        }
        T out[NP];
        T tot = T(0);
#pragma unroll
        for (int a = 1; a < NP; ++a) {
            T nv = v0[a];
            if (na >= 2 && on[a]) {
                T rate = T(0);
#pragma unroll
                for (int b = 0; b < NP; ++b) {
                    if (b == a || !on[b]) continue;
                    T t = (T)sg[a * NP + b] * (I[a] - I[b]);
#pragma unroll
                    for (int g = 0; g < NP; ++g) {
                        if (g == a || g == b || !on[g]) continue;
                        t += ((T)sg[b * NP + g] - (T)sg[a * NP + g]) * I[g];
                    }
                    t += vterm * (T)(hh[a] - hh[b]);
                    rate += (M / T(na)) * t;
                }
                nv = v0[a] + rate;
            }
            nv = nv < T(0) ? T(0) : (nv > T(1) ? T(1) : nv);
            out[a] = nv;
            tot += nv;
        }
        if (tot > T(1)) {
#pragma unroll
            for (int a = 1; a < NP; ++a) out[a] /= tot;
        }
#pragma unroll
        for (int a = 0; a < NBMAX; ++a)
            if (a < nbod) dst[(long long)a * Np + idx] = out[a + 1];
    }
}

// Reclassification (Sec. 3.2.2): solid iff the fluid fraction 1 - sum phi is below the
// threshold, owner = argmax phi (lowest index on ties).  Marks the nodes that changed side,
// copies the final phase fields into the second buffer, and accumulates the bounding box of
// the support (unwrapped coordinates) with integer atomics.
template <typename T>
__global__ __launch_bounds__(256) void k_classify(Prm<T> p, int parity, StepState *st, const T *__restrict__ phi,
                                                  T *__restrict__ phi_copy, uint8_t *__restrict__ mask, int init) {
    const int32_t *bx = st->box[parity];
    const long long vol = box_volume(bx);
    const int nx = p.nx, ny = p.ny, nz = p.nz, nbod = p.nb;
    const long long Np = p.Np;
    int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    unsigned long long f2s = 0, s2f = 0;
    const long long stride = (long long)gridDim.x * 256;
    for (long long base = (long long)blockIdx.x * 256; base < vol; base += stride) {
        const long long k = base + threadIdx.x;
        if (k < vol) {
            int u[3];
            box_cell(bx, k, u[0], u[1], u[2]);
            const int x = wrapi(u[0], nx), y = wrapi(u[1], ny), z = wrapi(u[2], nz);
            const int idx = x + nx * (y + ny * z);
            T sum = T(0), best = T(-1);
            int arg = 0;
            for (int a = 0; a < nbod; ++a) {
                const T v = phi[(long long)a * Np + idx];
                if (phi_copy) phi_copy[(long long)a * Np + idx] = v;
                sum += v;
                if (v > best) {
                    best = v;
                    arg = a;
                }
            }
            const bool solid = nbod > 0 && (T(1) - sum) < (T)p.threshold;
            const uint8_t old = mask[idx];
            uint8_t m = solid ? (uint8_t)(M_SOLID | arg) : (uint8_t)0;
            if (!init) {
                if (solid && !(old & M_SOLID)) {
                    m |= M_F2S;
                    ++f2s;
                }
                if (!solid && (old & M_SOLID)) {
                    m |= M_S2F;
                    ++s2f;
                }
            }
            mask[idx] = m;
            if (sum > T(0)) {
                for (int d = 0; d < 3; ++d) {
                    lo[d] = min(lo[d], u[d]);
                    hi[d] = max(hi[d], u[d]);
                }
            }
        }
    }
    for (int d = 0; d < 3; ++d) {
        const int l = wave_min(lo[d]), h = wave_max(hi[d]);
        if ((threadIdx.x & 63) == 0 && l <= h) {
            atomicMin(&st->tight[d], l);
            atomicMax(&st->tight[3 + d], h);
        }
    }
    const unsigned long long a = wave_sum(f2s), b = wave_sum(s2f);
    if ((threadIdx.x & 63) == 0) {
        if (a) atomicAdd(&st->n_f2s, a);
        if (b) atomicAdd(&st->n_s2f, b);
    }
}

// Equilibrium of (rho, u) in direction i (Sec. 3.2.1)
template <typename T, int I>
__device__ __forceinline__ T feq_dir(T rho, T ux, T uy, T uz) {
    const T cu = T(Dir<I>::x) * ux + T(Dir<I>::y) * uy + T(Dir<I>::z) * uz;
    const T uu = ux * ux + uy * uy + uz * uz;
    return Dir<I>::template w<T>() * rho * (T(1) + T(3) * cu + T(4.5) * cu * cu - T(1.5) * uu);
}

// number of fluid nodes (current mask) within squared radius r2 of node (x, y, z), over the 26
// neighbours
__device__ __forceinline__ int fluid_count(const uint8_t *mask, int x, int y, int z, int nx, int ny, int nz, double r2) {
    int cnt = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int d2 = dx * dx + dy * dy + dz * dz;
                if (d2 == 0 || d2 > r2 + 1e-9) continue;
                const int n = wrapi(x + dx, nx) + nx * (wrapi(y + dy, ny) + ny * wrapi(z + dz, nz));
                if (!(mask[n] & M_SOLID)) ++cnt;
            }
    return cnt;
}

// the neighbourhood N_F(x_n) of a node that became solid: fluid nodes within R_A, widened to
// sqrt(2) and then sqrt(3) while it is empty.  Returns its squared radius and size (0 if empty).
__device__ __forceinline__ int conversion_radius(const uint8_t *mask, int x, int y, int z, int nx, int ny, int nz,
                                                 double RA, double &r2sel) {
    const double radii2[3] = {RA * RA, 2.0, 3.0};
    for (int t = 0; t < 3; ++t) {
        if (t > 0 && radii2[t] <= RA * RA + 1e-9) continue;
        const int c = fluid_count(mask, x, y, z, nx, ny, nz, radii2[t]);
        if (c > 0) {
            r2sel = radii2[t];
            return c;
        }
    }
    r2sel = 0.0;
    return 0;
}

// Node conversion, receiving side (Sec. 3.2.2): every fluid node gathers, from each neighbour
// that just became solid and whose neighbourhood N_F contains it, f_eq(rho_n, u_n) / |N_F| with
// rho_n, u_n = j_n / rho_n of the converted node's populations.  A node that just became fluid
// starts from empty populations.  Sources are only read here and emptied by k_convert_finish.
template <typename T>
__global__ __launch_bounds__(256) void k_convert_gather(Prm<T> p, int parity, const StepState *st,
                                                        const uint8_t *__restrict__ mask, T *f) {
    const int32_t *bx = st->box[parity];
    const long long vol = box_volume(bx);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const long long Np = p.Np;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < vol; k += (long long)gridDim.x * 256) {
        int ux, uy, uz;
        box_cell(bx, k, ux, uy, uz);
        const int x = wrapi(ux, nx), y = wrapi(uy, ny), z = wrapi(uz, nz);
        const int idx = x + nx * (y + ny * z);
        const uint8_t m = mask[idx];
        if (m & M_SOLID) continue;
        bool any = (m & M_S2F) != 0;
        for (int dz = -1; dz <= 1 && !any; ++dz)
            for (int dy = -1; dy <= 1 && !any; ++dy)
                for (int dx = -1; dx <= 1 && !any; ++dx) {
                    if (!dx && !dy && !dz) continue;
                    const int n = wrapi(x + dx, nx) + nx * (wrapi(y + dy, ny) + ny * wrapi(z + dz, nz));
                    if (mask[n] & M_F2S) any = true;
                }
        if (!any) continue;
        T acc[19];
        sfor<19>([&](auto I) { acc[I] = (m & M_S2F) ? T(0) : f[(long long)I * Np + idx]; });
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int d2 = dx * dx + dy * dy + dz * dz;
                    if (d2 == 0) continue;
                    const int sx = wrapi(x + dx, nx), sy = wrapi(y + dy, ny), sz = wrapi(z + dz, nz);
                    const int n = sx + nx * (sy + ny * sz);
                    if (!(mask[n] & M_F2S)) continue;
                    double r2;
                    const int cnt = conversion_radius(mask, sx, sy, sz, nx, ny, nz, p.R_A, r2);
                    if (cnt == 0 || d2 > r2 + 1e-9) continue;
                    T fs[19];
                    sfor<19>([&](auto I) { fs[I] = f[(long long)I * Np + n]; });
                    T rho = T(0), jx = T(0), jy = T(0), jz = T(0);
                    sfor<19>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        rho += fs[i];
                        jx += T(Dir<i>::x) * fs[i];
                        jy += T(Dir<i>::y) * fs[i];
                        jz += T(Dir<i>::z) * fs[i];
                    });
                    T vx = T(0), vy = T(0), vz = T(0);
                    if (rho > T(0)) {
                        vx = jx / rho;
                        vy = jy / rho;
                        vz = jz / rho;
                    }
                    const T inv = T(1) / T(cnt);
                    sfor<19>([&](auto I) { acc[I] += feq_dir<T, decltype(I)::value>(rho, vx, vy, vz) * inv; });
                }
        sfor<19>([&](auto I) { f[(long long)I * Np + idx] = acc[I]; });
    }
}

// Node conversion, source side: empty the populations of nodes that became solid, count those
// whose neighbourhood held no fluid node, clear the event bits; the last block turns the support
// bounds into the next step's box (3-cell margin, whole axis once it would wrap onto itself)
// and resets the accumulators.
template <typename T>
__global__ __launch_bounds__(256) void k_convert_finish(Prm<T> p, int parity, StepState *st, uint8_t *__restrict__ mask,
                                                        T *f) {
    __shared__ uint32_t ticket;
    const int32_t *bx = st->box[parity];
    const long long vol = box_volume(bx);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const long long Np = p.Np;
    unsigned long long lost = 0;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < vol; k += (long long)gridDim.x * 256) {
        int ux, uy, uz;
        box_cell(bx, k, ux, uy, uz);
        const int x = wrapi(ux, nx), y = wrapi(uy, ny), z = wrapi(uz, nz);
        const int idx = x + nx * (y + ny * z);
        const uint8_t m = mask[idx];
        if (!(m & (M_F2S | M_S2F))) continue;
        if (m & M_F2S) {
            double r2;
            if (conversion_radius(mask, x, y, z, nx, ny, nz, p.R_A, r2) == 0) ++lost;
            sfor<19>([&](auto I) { f[(long long)I * Np + idx] = T(0); });
        }
        mask[idx] = m & (uint8_t)~(M_F2S | M_S2F);
    }
    if (lost) atomicAdd(&st->n_lost, lost);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) ticket = atomicAdd(&st->done[2], 1u);
    __syncthreads();
    if (ticket != gridDim.x - 1 || threadIdx.x != 0) return;
    __threadfence();
    const int n[3] = {nx, ny, nz};
    int32_t *nbx = st->box[parity ^ 1];
    volatile int32_t *tg = st->tight;
    bool empty = false;
    for (int d = 0; d < 3; ++d) empty = empty || tg[d] > tg[3 + d];
    for (int d = 0; d < 3; ++d) {
        int lo = tg[d] - 3, hi = tg[3 + d] + 3;
        if (hi - lo + 1 >= n[d]) {
            lo = 0;
            hi = n[d] - 1;
        }
        nbx[d] = empty ? 0 : lo;
        nbx[3 + d] = empty ? -1 : hi;
        tg[d] = INT32_MAX;
        tg[3 + d] = INT32_MIN;
    }
    st->done[2] = 0;
}

// Solid-solid repulsion (Sec. 3.1.2) between solid nodes p of body b1 and q of body b2 > b1
// with |p - q| < r_c (minimum image): f = e0 (n/r_c) (p - q)/|p - q| |(|p - q| - r_c)/r_c|^(n-1)
// on b1 at p, -f on b2 at q; torques about the centres.  Same per-wave, per-body LDS
// accumulation and block partials as k_body_forces (summed by its last block).
template <typename T>
__global__ __launch_bounds__(256) void k_repulsion(Prm<T> p, int parity, const StepState *st,
                                                   const uint8_t *__restrict__ mask, const BodyDev *__restrict__ bodies,
                                                   double *part) {
    __shared__ double acc[4][PF_LBM_MAX_BODIES][6];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int nbod = p.nb;
    for (int k = tid; k < 4 * PF_LBM_MAX_BODIES * 6; k += 256) (&acc[0][0][0])[k] = 0.0;
    __syncthreads();
    const int32_t *bx = st->box[parity];
    const long long vol = box_volume(bx);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const double rc = p.r_c, ne = p.n_exp, e0 = p.e0;
    const int R = (int)ceil(rc);
    const long long stride = (long long)gridDim.x * 256;
    for (long long base = (long long)blockIdx.x * 256; base < vol; base += stride) {
        const long long k = base + tid;
        uint32_t touched = 0;
        int x = 0, y = 0, z = 0, b1 = -1;
        if (k < vol) {
            int ux, uy, uz;
            box_cell(bx, k, ux, uy, uz);
            x = wrapi(ux, nx);
            y = wrapi(uy, ny);
            z = wrapi(uz, nz);
            const uint8_t m = mask[x + nx * (y + ny * z)];
            if (m & M_SOLID) {
                b1 = m & M_OWNER;
                for (int dz = -R; dz <= R; ++dz)
                    for (int dy = -R; dy <= R; ++dy)
                        for (int dx = -R; dx <= R; ++dx) {
                            const int d2 = dx * dx + dy * dy + dz * dz;
                            if (d2 == 0 || !((double)d2 < rc * rc)) continue;
                            const uint8_t mq = mask[wrapi(x + dx, nx) + nx * (wrapi(y + dy, ny) + ny * wrapi(z + dz, nz))];
                            if ((mq & M_SOLID) && (int)(mq & M_OWNER) > b1) touched |= (1u << b1) | (1u << (mq & M_OWNER));
                        }
            }
        }
        uint32_t wt = wave_or(touched);
        while (wt) {
            const int b = __ffs(wt) - 1;
            wt &= wt - 1;
            double v[6] = {0, 0, 0, 0, 0, 0};
            if (touched & (1u << b)) {
                for (int dz = -R; dz <= R; ++dz)
                    for (int dy = -R; dy <= R; ++dy)
                        for (int dx = -R; dx <= R; ++dx) {
                            const int d2 = dx * dx + dy * dy + dz * dz;
                            if (d2 == 0 || !((double)d2 < rc * rc)) continue;
                            const uint8_t mq = mask[wrapi(x + dx, nx) + nx * (wrapi(y + dy, ny) + ny * wrapi(z + dz, nz))];
                            if (!(mq & M_SOLID)) continue;
                            const int b2 = mq & M_OWNER;
                            if (b2 <= b1 || (b != b1 && b != b2)) continue;
                            const double r = sqrt((double)d2);
                            const double mag = e0 * (ne / rc) * pow(fabs((r - rc) / rc), ne - 1.0);
                            // force on b1 at p, directed from q to p
                            double fx = -dx / r * mag, fy = -dy / r * mag, fz = -dz / r * mag;
                            double ax = x, ay = y, az = z;
                            if (b == b2) {
                                fx = -fx;
                                fy = -fy;
                                fz = -fz;
                                ax = x + dx;
                                ay = y + dy;
                                az = z + dz;
                            }
                            const BodyDev &B = bodies[b];
                            const double rx = mimg(ax - B.X[0], nx), ry = mimg(ay - B.X[1], ny), rz = mimg(az - B.X[2], nz);
                            v[0] += fx;
                            v[1] += fy;
                            v[2] += fz;
                            v[3] += ry * fz - rz * fy;
                            v[4] += rz * fx - rx * fz;
                            v[5] += rx * fy - ry * fx;
                        }
            }
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const double s = wave_sum(v[c]);
                if (lane == 0) acc[wave][b][c] += s;
            }
        }
    }
    __syncthreads();
    for (int k = tid; k < nbod * 6; k += 256) {
        const int b = k / 6, c = k % 6;
        part[((long long)blockIdx.x * nbod + b) * 6 + c] = ((acc[0][b][c] + acc[1][b][c]) + acc[2][b][c]) + acc[3][b][c];
    }
}

// ---- initialisation and read-out helpers ------------------------------------------------------

// phase fields from the FP64 host copy, into both buffers
template <typename T>
__global__ void k_init_phi(Prm<T> p, const double *__restrict__ src, T *__restrict__ a, T *__restrict__ b) {
    const long long total = (long long)p.nb * p.N;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < total; k += (long long)gridDim.x * 256) {
        const long long ph = k / p.N, c = k % p.N;
        const T v = (T)src[k];
        a[ph * p.Np + c] = v;
        b[ph * p.Np + c] = v;
    }
}

// fluid at rest: f = f_eq(rho, 0) = w_i rho on fluid nodes, 0 on solid nodes
template <typename T>
__global__ void k_init_f(Prm<T> p, const double *__restrict__ rho, const uint8_t *__restrict__ mask, T *__restrict__ fa) {
    for (int idx = blockIdx.x * 256 + threadIdx.x; idx < p.N; idx += gridDim.x * 256) {
        const bool solid = (mask[idx] & M_SOLID) != 0;
        const T r = solid ? T(0) : (T)rho[idx];
        sfor<19>([&](auto I) { fa[(long long)I * p.Np + idx] = Dir<decltype(I)::value>::template w<T>() * r; });
    }
}

template <typename T>
__global__ void k_zero_mask(Prm<T> p, uint8_t *mask) {
    for (int idx = blockIdx.x * 256 + threadIdx.x; idx < p.N; idx += gridDim.x * 256) mask[idx] = 0;
}

template <typename T, typename D>
__global__ void k_fields(Prm<T> p, int which, const T *__restrict__ f, const uint8_t *__restrict__ mask,
                         const T *__restrict__ psi, const T *__restrict__ phi, D *__restrict__ dst) {
    for (int idx = blockIdx.x * 256 + threadIdx.x; idx < p.N; idx += gridDim.x * 256) {
        const uint8_t m = mask[idx];
        double out = 0.0;
        if (which >= 16) {
            out = (double)phi[(long long)(which - 16) * p.Np + idx];
        } else if (which == 4) {
            out = (m & M_SOLID) ? 1.0 : 0.0;
        } else if (which == 5) {
            out = (m & M_SOLID) ? (double)(m & M_OWNER) : -1.0;
        } else if (which == 6) {
            out = (double)psi[idx];
        } else if (!(m & M_SOLID)) {
            double s = 0.0;
            sfor<19>([&](auto I) {
                constexpr int i = decltype(I)::value;
                const double c = which == 0 ? 1.0 : (which == 1 ? Dir<i>::x : (which == 2 ? Dir<i>::y : Dir<i>::z));
                s += c * (double)f[(long long)i * p.Np + idx];
            });
            out = s;
        }
        dst[idx] = (D)out;
    }
}

}  // namespace pfl
