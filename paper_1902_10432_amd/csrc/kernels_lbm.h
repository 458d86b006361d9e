// Fluid kernels of the step: pseudopotential, fused force + Guo-BGK collision + push streaming
// with moving-wall bounce-back, and the per-body force/torque sums with the rigid-body update.
#pragma once

#include "device_common.h"

namespace pfl {

// Pseudopotential psi = 1 - exp(-rho/rho0) of every fluid node; a solid node carries the value
// of its body's wetting density (Sec. 3.2.3).  Dense, one thread per cell.
template <typename T>
__global__ __launch_bounds__(256) void k_psi(Prm<T> p, const T *__restrict__ f, const uint8_t *__restrict__ mask,
                                             const BodyDev *__restrict__ bodies, T *__restrict__ psi) {
    const int idx = xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (idx >= p.N) return;
    const uint8_t m = mask[idx];
    T out;
    if (m & M_SOLID) {
        out = (T)bodies[m & M_OWNER].psi_s;
    } else {
        T r = T(0);
        sfor<19>([&](auto I) { r += f[(long long)I * p.Np + idx]; });
        out = -expm1(-r * p.inv_rho0);
    }
    psi[idx] = out;
}

// periodic neighbour offsets of one cell (index deltas for +1 / -1 along each axis)
struct Nbr {
    int xp, xm, yp, ym, zp, zm;
    __device__ __forceinline__ Nbr(int x, int y, int z, int nx, int ny, int nz) {
        const int pl = nx * ny;
        xp = x == nx - 1 ? 1 - nx : 1;
        xm = x == 0 ? nx - 1 : -1;
        yp = y == ny - 1 ? (1 - ny) * nx : nx;
        ym = y == 0 ? (ny - 1) * nx : -nx;
        zp = z == nz - 1 ? (1 - nz) * pl : pl;
        zm = z == 0 ? (nz - 1) * pl : -pl;
    }
    template <int I>
    __device__ __forceinline__ int off() const {
        return (Dir<I>::x == 1 ? xp : (Dir<I>::x == -1 ? xm : 0)) + (Dir<I>::y == 1 ? yp : (Dir<I>::y == -1 ? ym : 0)) +
               (Dir<I>::z == 1 ? zp : (Dir<I>::z == -1 ? zm : 0));
    }
};

// Rigid-body velocity V + omega x (p - X) at point p (minimum image), Sec. 3.1.1.
__device__ __forceinline__ void wall_velocity(const BodyDev &B, double px, double py, double pz, double nx, double ny,
                                              double nz, double &ux, double &uy, double &uz) {
    const double rx = mimg(px - B.X[0], nx), ry = mimg(py - B.X[1], ny), rz = mimg(pz - B.X[2], nz);
    ux = B.V[0] + (B.W[1] * rz - B.W[2] * ry);
    uy = B.V[1] + (B.W[2] * rx - B.W[0] * rz);
    uz = B.V[2] + (B.W[0] * ry - B.W[1] * rx);
}

// One fluid node per thread: load its 19 post-stream populations, form the Shan-Chen/Benzi force
// from the 18 neighbour pseudopotentials (solid neighbours act with their wetting density),
// collide with BGK + Guo forcing at the half-force velocity, and push each post-collision
// population to its neighbour, or reflect it half-way into the node's own opposite slot with the
// moving-wall term when the neighbour is solid.  The wall terms are taken back from the rest
// population (Sec. 3.2.1, 3.2.2, 3.2.3).  Solid nodes are skipped and receive nothing.
template <typename T>
__global__ __launch_bounds__(256) void k_collide_stream(Prm<T> p, const T *__restrict__ fin, T *__restrict__ fout,
                                                        const T *__restrict__ psi, const uint8_t *__restrict__ mask,
                                                        const BodyDev *__restrict__ bodies) {
    const int idx = xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (idx >= p.N) return;
    if (mask[idx] & M_SOLID) return;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int x = idx % nx, yz = idx / nx, y = yz % ny, z = yz / ny;
    const Nbr nb(x, y, z, nx, ny, nz);
    const long long Np = p.Np;

    T f[19];
    sfor<19>([&](auto I) { f[I] = fin[(long long)I * Np + idx]; });
    T rho = T(0), jx = T(0), jy = T(0), jz = T(0);
    sfor<19>([&](auto I) {
        constexpr int i = decltype(I)::value;
        rho += f[i];
        if constexpr (Dir<i>::x == 1) jx += f[i];
        if constexpr (Dir<i>::x == -1) jx -= f[i];
        if constexpr (Dir<i>::y == 1) jy += f[i];
        if constexpr (Dir<i>::y == -1) jy -= f[i];
        if constexpr (Dir<i>::z == 1) jz += f[i];
        if constexpr (Dir<i>::z == -1) jz -= f[i];
    });

    // pseudopotential force and solid-neighbour map
    T sx = T(0), sy = T(0), sz = T(0);
    uint32_t solid_dirs = 0;
    uint8_t nbm[19];
    sfor<19>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (i > 0) {
            const int n = idx + nb.template off<i>();
            const T wp = Dir<i>::template w<T>() * psi[n];
            if constexpr (Dir<i>::x != 0) sx += T(Dir<i>::x) * wp;
            if constexpr (Dir<i>::y != 0) sy += T(Dir<i>::y) * wp;
            if constexpr (Dir<i>::z != 0) sz += T(Dir<i>::z) * wp;
            nbm[i] = mask[n];
            if (nbm[i] & M_SOLID) solid_dirs |= 1u << i;
        }
    });
    const T gp = -p.G * psi[idx];
    const T Fx = gp * sx + p.fext[0], Fy = gp * sy + p.fext[1], Fz = gp * sz + p.fext[2];

    // half-force velocity; an empty node has v = 0
    T ux = T(0), uy = T(0), uz = T(0);
    if (rho > T(0)) {
        const T inv = T(1) / rho;
        ux = (jx + T(0.5) * Fx) * inv;
        uy = (jy + T(0.5) * Fy) * inv;
        uz = (jz + T(0.5) * Fz) * inv;
    }
    const T uu = ux * ux + uy * uy + uz * uz;
    const T uF = ux * Fx + uy * Fy + uz * Fz;
    const T om = p.omega, guo = p.guo;

    // collision: f* = f - (f - f_eq)/tau + (1 - 1/(2 tau)) w [3 (c - v).F + 9 (c.v)(c.F)]
    sfor<19>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr T w = Dir<i>::template w<T>();
        const T cu = T(Dir<i>::x) * ux + T(Dir<i>::y) * uy + T(Dir<i>::z) * uz;
        const T cF = T(Dir<i>::x) * Fx + T(Dir<i>::y) * Fy + T(Dir<i>::z) * Fz;
        const T feq = w * rho * (T(1) + T(3) * cu + T(4.5) * cu * cu - T(1.5) * uu);
        const T Fi = guo * w * (T(3) * (cF - uF) + T(9) * cu * cF);
        f[i] = f[i] - om * (f[i] - feq) + Fi;
    });

    // streaming
    T drho = T(0);
    sfor<19>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (i > 0) {
            if (!(solid_dirs & (1u << i))) {
                fout[(long long)i * Np + idx + nb.template off<i>()] = f[i];
            } else {
                // reflected into direction opp(i) with g = -2 rho w_i (c_i . u_w) / c_s^2, u_w at
                // the link midpoint x + c_i / 2
                const BodyDev &B = bodies[nbm[i] & M_OWNER];
                double uwx, uwy, uwz;
                wall_velocity(B, x + 0.5 * Dir<i>::x, y + 0.5 * Dir<i>::y, z + 0.5 * Dir<i>::z, nx, ny, nz, uwx, uwy, uwz);
                const double cuw = Dir<i>::x * uwx + Dir<i>::y * uwy + Dir<i>::z * uwz;
                const T g = T(-6.0 * Dir<i>::template w<double>() * cuw) * rho;
                fout[(long long)Dir<i>::opp * Np + idx] = f[i] + g;
                drho += g;
            }
        }
    });
    fout[idx] = f[0] - drho;
}

// Per-body sums over the fluid nodes next to solid nodes (box-restricted):
//   momentum exchange  c_i (2 f*_i + g) for each link from a fluid node into body b, recovered
//   from the reflected population f_opp(i) = f*_i + g written by k_collide_stream;
//   pseudopotential reaction  +G psi(x) w_i psi(varrho_b) c_i (opposite of the fluid's share);
//   torques about X_b with the link midpoint as lever arm.
// Each wave reduces its contributions per touched body (64-lane shuffles) into LDS in a fixed
// order; blocks write FP64 partials; the last block to finish sums all partials (and the
// repulsion partials of the previous classification) in block order, stores F, T and advances
// the bodies: V += F/M, X += V, omega += I^-1 T (Sec. 3.1.1).  Deterministic, no float atomics.
template <typename T>
__global__ __launch_bounds__(256) void k_body_forces(Prm<T> p, int parity, StepState *st, const T *__restrict__ fin,
                                                     const T *__restrict__ fpost, const T *__restrict__ psi,
                                                     const uint8_t *__restrict__ mask, BodyDev *bodies,
                                                     double *part, const double *rep_part, int rep_blocks) {
    __shared__ double acc[4][PF_LBM_MAX_BODIES][6];
    __shared__ uint32_t ticket;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int nbod = p.nb;
    for (int k = tid; k < 4 * PF_LBM_MAX_BODIES * 6; k += 256) (&acc[0][0][0])[k] = 0.0;
    __syncthreads();
    const int32_t *bx = st->box[parity];
    const long long vol = box_volume(bx);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const long long Np = p.Np;
    const long long stride = (long long)gridDim.x * 256;
    for (long long base = (long long)blockIdx.x * 256; base < vol; base += stride) {
        const long long k = base + tid;
        uint32_t touched = 0;
        int x = 0, y = 0, z = 0, idx = 0;
        T rho = T(0), ps0 = T(0);
        if (k < vol) {
            int ux, uy, uz;
            box_cell(bx, k, ux, uy, uz);
            x = wrapi(ux, nx);
            y = wrapi(uy, ny);
            z = wrapi(uz, nz);
            idx = x + nx * (y + ny * z);
            if (!(mask[idx] & M_SOLID)) {
                const Nbr nb(x, y, z, nx, ny, nz);
                sfor<19>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    if constexpr (i > 0) {
                        const uint8_t mn = mask[idx + nb.template off<i>()];
                        if (mn & M_SOLID) touched |= 1u << (mn & M_OWNER);
                    }
                });
                if (touched) {
                    sfor<19>([&](auto I) { rho += fin[(long long)I * Np + idx]; });
                    ps0 = psi[idx];
                }
            }
        }
        uint32_t wt = wave_or(touched);
        while (wt) {
            const int b = __ffs(wt) - 1;
            wt &= wt - 1;
            double v[6] = {0, 0, 0, 0, 0, 0};
            if (touched & (1u << b)) {
                const Nbr nb(x, y, z, nx, ny, nz);
                const BodyDev &B = bodies[b];
                sfor<19>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    if constexpr (i > 0) {
                        const int n = idx + nb.template off<i>();
                        const uint8_t mn = mask[n];
                        if ((mn & M_SOLID) && (mn & M_OWNER) == b) {
                            const double px = x + 0.5 * Dir<i>::x, py = y + 0.5 * Dir<i>::y, pz = z + 0.5 * Dir<i>::z;
                            double uwx, uwy, uwz;
                            wall_velocity(B, px, py, pz, nx, ny, nz, uwx, uwy, uwz);
                            const double cuw = Dir<i>::x * uwx + Dir<i>::y * uwy + Dir<i>::z * uwz;
                            const T g = T(-6.0 * Dir<i>::template w<double>() * cuw) * rho;
                            const T fr = fpost[(long long)Dir<i>::opp * Np + idx];
                            // momentum to the body + pseudopotential reaction, both along c_i
                            const double s = (double)(T(2) * fr - g) +
                                             (double)(p.G * ps0 * Dir<i>::template w<T>() * psi[n]);
                            const double fx = s * Dir<i>::x, fy = s * Dir<i>::y, fz = s * Dir<i>::z;
                            const double rx = mimg(px - B.X[0], nx), ry = mimg(py - B.X[1], ny), rz = mimg(pz - B.X[2], nz);
                            v[0] += fx;
                            v[1] += fy;
                            v[2] += fz;
                            v[3] += ry * fz - rz * fy;
                            v[4] += rz * fx - rx * fz;
                            v[5] += rx * fy - ry * fx;
                        }
                    }
                });
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
    __threadfence();
    __syncthreads();
    if (tid == 0) ticket = atomicAdd(&st->done[0], 1u);
    __syncthreads();
    if (ticket != gridDim.x - 1) return;
    // ---- last block: fixed-order totals and the rigid-body update
    __threadfence();
    __shared__ double tot[PF_LBM_MAX_BODIES * 6];
    for (int k = tid; k < nbod * 6; k += 256) {
        double s = 0.0;
        for (int j = 0; j < (int)gridDim.x; ++j) s += part[(long long)j * nbod * 6 + k];
        for (int j = 0; j < rep_blocks; ++j) s += rep_part[(long long)j * nbod * 6 + k];
        tot[k] = s;
    }
    __syncthreads();
    if (tid < nbod) {
        BodyDev &B = bodies[tid];
        const double *F = &tot[tid * 6], *Tq = &tot[tid * 6 + 3];
        bool finite = true;
        for (int d = 0; d < 3; ++d) {
            B.F[d] = F[d];
            B.T[d] = Tq[d];
            finite = finite && isfinite(F[d]) && isfinite(Tq[d]);
        }
        if ((p.flags & 2) && !B.fixed) {
            for (int d = 0; d < 3; ++d) B.V[d] += F[d] / B.M;
            for (int d = 0; d < 3; ++d) B.X[d] += B.V[d];
            for (int d = 0; d < 3; ++d)
                B.W[d] += B.Iinv[3 * d + 0] * Tq[0] + B.Iinv[3 * d + 1] * Tq[1] + B.Iinv[3 * d + 2] * Tq[2];
        }
        for (int d = 0; d < 3; ++d) finite = finite && isfinite(B.V[d]) && isfinite(B.X[d]) && isfinite(B.W[d]);
        if (!finite) atomicOr(&st->err, 1u);
    }
    if (tid == 0) st->done[0] = 0;
}

}  // namespace pfl
