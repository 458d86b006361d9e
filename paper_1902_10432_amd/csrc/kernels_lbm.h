// Fluid kernels of the step: fused force + Guo-BGK collision + push streaming with moving-wall
// bounce-back, and the per-body force/torque sums (the pseudopotential pass, which also closes
// the previous step's node conversions, is in kernels_pf.h).
#pragma once

#include "device_common.h"

namespace pfl {

// periodic neighbour offsets of one cell as unsigned index deltas (the sum with the cell index
// wraps modulo 2^32 onto the neighbour's index, which lets loads use a scalar base + 32-bit
// offset)
struct NbrU {
    uint32_t xp, xm, yp, ym, zp, zm;
    // scale: bytes per element for byte offsets, 1 for element indices
    __device__ __forceinline__ NbrU(int x, int y, int z, int nx, int ny, int nz, int scale) {
        const int pl = nx * ny;
        xp = (uint32_t)((x == nx - 1 ? 1 - nx : 1) * scale);
        xm = (uint32_t)((x == 0 ? nx - 1 : -1) * scale);
        yp = (uint32_t)((y == ny - 1 ? (1 - ny) * nx : nx) * scale);
        ym = (uint32_t)((y == 0 ? (ny - 1) * nx : -nx) * scale);
        zp = (uint32_t)((z == nz - 1 ? (1 - nz) * pl : pl) * scale);
        zm = (uint32_t)((z == 0 ? (nz - 1) * pl : -pl) * scale);
    }
    template <int I>
    __device__ __forceinline__ uint32_t at(uint32_t idx) const {
        uint32_t o = idx;
        if constexpr (Dir<I>::x == 1) o += xp;
        if constexpr (Dir<I>::x == -1) o += xm;
        if constexpr (Dir<I>::y == 1) o += yp;
        if constexpr (Dir<I>::y == -1) o += ym;
        if constexpr (Dir<I>::z == 1) o += zp;
        if constexpr (Dir<I>::z == -1) o += zm;
        return o;
    }
};

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
    // the same for a direction known only at run time
    __device__ __forceinline__ int off_rt(int i) const {
        const int cx = kCX[i], cy = kCY[i], cz = kCZ[i];
        return (cx > 0 ? xp : (cx < 0 ? xm : 0)) + (cy > 0 ? yp : (cy < 0 ? ym : 0)) + (cz > 0 ? zp : (cz < 0 ? zm : 0));
    }
};

// Rigid-body velocity V + omega x (p - X) at point p (minimum image), Sec. 3.1.1.
template <typename T>
__device__ __forceinline__ void wall_velocity(const Prm<T> &p, const BodyDev &B, double px, double py, double pz,
                                              double &ux, double &uy, double &uz) {
    const double rx = mimg_r(px - B.X[0], p.nx, p.inv_n[0]), ry = mimg_r(py - B.X[1], p.ny, p.inv_n[1]),
                 rz = mimg_r(pz - B.X[2], p.nz, p.inv_n[2]);
    ux = B.V[0] + (B.W[1] * rz - B.W[2] * ry);
    uy = B.V[1] + (B.W[2] * rx - B.W[0] * rz);
    uz = B.V[2] + (B.W[0] * ry - B.W[1] * rx);
}

// reciprocal: correctly rounded in FP64 (parity with the FP64 oracle), hardware rcp in FP32
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// 3-D launch (64 x R threads per block, R = 1, 2 or 4, grid ceil(nx/64) x ceil(ny/R) x nz) with the
// flat block id remapped so that each XCD works on a contiguous range of planes.
__device__ __forceinline__ bool cell_of_block(int nx, int ny, int &x, int &y, int &z) {
    const int gx = gridDim.x, gy = gridDim.y;
    const int lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const int r = xcd_block(lin, gx * gy * gridDim.z);
    const int bz = r / (gx * gy), rem = r - bz * gx * gy, by = rem / gx, bxx = rem - by * gx;
    x = bxx * 64 + (int)threadIdx.x;
    y = by * (int)blockDim.y + (int)threadIdx.y;
    z = bz;
    return x < nx && y < ny;
}

// One fluid node per thread: load its 19 post-stream populations, form the Shan-Chen/Benzi force
// from the 18 neighbour pseudopotentials (solid neighbours act with their wetting density),
// collide with BGK + Guo forcing at the half-force velocity, and push each post-collision
// population to its neighbour, or reflect it half-way into the node's own opposite slot with the
// moving-wall term when the neighbour is solid.  The wall terms are taken back from the rest
// population (Sec. 3.2.1, 3.2.2, 3.2.3).  Solid nodes are skipped and receive nothing.
//
// With bodies, the first block also publishes the step's box, solid radii, volume terms and event
// flag from the previous reclassification (publish_step_state) before its own cells: that short
// reduction chain then hides behind the longest pass of the step instead of costing a launch.
//
// Arithmetic is organised by opposite pairs (c_opp = -c): with cu = c.v, cF = c.F,
//   f*_i = (1 - 1/tau) f_i + w (even + odd),  f*_opp = (1 - 1/tau) f_opp + w (even - odd),
//   even = rho/tau (1 - 3/2 v.v) - 3 g v.F + 9/2 rho/tau cu^2 + 9 g cu cF,  odd = 3 rho/tau cu + 3 g cF,
// g = 1 - 1/(2 tau), which is the BGK relaxation to the second-order equilibrium plus the Guo term.
template <typename S, class L>
__global__ __launch_bounds__(256) void k_collide_stream(Prm<ArT<S>> p, const S *__restrict__ fin, S *__restrict__ fout,
                                                        const ArT<S> *__restrict__ psi,
                                                        const ArT<S> *__restrict__ psi_prev,
                                                        const cell_t *__restrict__ mask,
                                                        BodyDev *bodies, int parity, StepState *st,
                                                        const ClassifyPart *__restrict__ cpart, int cblk,
                                                        const uint32_t *__restrict__ nbw) {
    using T = ArT<S>;
    if (cpart && (blockIdx.x | blockIdx.y | blockIdx.z) == 0)
        publish_step_state((int)threadIdx.y, (int)blockDim.y, parity, p.nx, p.ny, p.nz, p.nb, p.eta, st, bodies, cpart,
                           cblk);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    int x, y, z;
    if (!cell_of_block(nx, ny, x, y, z)) return;
    const uint32_t idx = (uint32_t)(x + nx * (y + ny * z));
    const cell_t w0 = mask[idx];
    if (w0 & C_SOLID) return;
    // bit i: the neighbour in direction i is solid (D3Q19: kept in the cell word; D3Q27: the
    // neighbour-bit word of the node)
    uint32_t solid_dirs;
    if constexpr (L::kBits)
        solid_dirs = w0 & C_NBMASK;
    else
        solid_dirs = nbw[idx];
    const uint32_t ib = idx * (uint32_t)sizeof(T);      // psi (arithmetic type)
    const uint32_t is = idx * (uint32_t)sizeof(S);      // populations (storage type)
    const NbrU nb(x, y, z, nx, ny, nz, (int)sizeof(T));
    const NbrU ns(x, y, z, nx, ny, nz, (int)sizeof(S));
    const long long Np = p.Np;
    constexpr bool H = sizeof(S) == 2;  // FP16 storage: deviations from w_i R

    T f[L::Q];
    {
        const T rin = H ? ref_density(psi_prev[idx], p.rho0) : T(0);  // reference of the inputs
        sfor<L::Q>([&](auto I) {
            f[I] = pop_get<S>(ldb_nt(fin + (long long)I * Np, is), Dir<decltype(I)::value, L>::template w<T>() * rin);
        });
    }
    // moments from pair sums and differences
    T rho = f[0], jx = T(0), jy = T(0), jz = T(0);
    sfor<(L::Q - 1) / 2>([&](auto K) {
        constexpr int i = 2 * decltype(K)::value + 1;  // i and i + 1 are opposite
        const T sp = f[i] + f[i + 1], dm = f[i] - f[i + 1];
        rho += sp;
        if constexpr (Dir<i, L>::x == 1) jx += dm;
        if constexpr (Dir<i, L>::x == -1) jx -= dm;
        if constexpr (Dir<i, L>::y == 1) jy += dm;
        if constexpr (Dir<i, L>::y == -1) jy -= dm;
        if constexpr (Dir<i, L>::z == 1) jz += dm;
        if constexpr (Dir<i, L>::z == -1) jz -= dm;
    });

    // pseudopotential force from pair differences of the neighbours' psi
    T s1x = T(0), s1y = T(0), s1z = T(0), s2x = T(0), s2y = T(0), s2z = T(0), s3x = T(0), s3y = T(0), s3z = T(0);
    T rdst[L::Q];  // FP16 form: reference density of each push destination
    sfor<(L::Q - 1) / 2>([&](auto K) {
        constexpr int i = 2 * decltype(K)::value + 1;
        const T pa = ldb(psi, nb.template at<i>(ib)), pb = ldb(psi, nb.template at<i + 1>(ib));
        if constexpr (H) {
            rdst[i] = ref_density(pa, p.rho0);
            rdst[i + 1] = ref_density(pb, p.rho0);
        }
        const T dp = pa - pb;
        if constexpr (Dir<i, L>::c2 == 1) {
            if constexpr (Dir<i, L>::x != 0) s1x += T(Dir<i, L>::x) * dp;
            if constexpr (Dir<i, L>::y != 0) s1y += T(Dir<i, L>::y) * dp;
            if constexpr (Dir<i, L>::z != 0) s1z += T(Dir<i, L>::z) * dp;
        } else if constexpr (Dir<i, L>::c2 == 2) {
            if constexpr (Dir<i, L>::x != 0) s2x += T(Dir<i, L>::x) * dp;
            if constexpr (Dir<i, L>::y != 0) s2y += T(Dir<i, L>::y) * dp;
            if constexpr (Dir<i, L>::z != 0) s2z += T(Dir<i, L>::z) * dp;
        } else {
            s3x += T(Dir<i, L>::x) * dp;
            s3y += T(Dir<i, L>::y) * dp;
            s3z += T(Dir<i, L>::z) * dp;
        }
    });
    const T psi0 = ldb(psi, ib);
    const T gp = -p.G * psi0;
    const T rown = H ? ref_density(psi0, p.rho0) : T(0);  // reference of this node's own slots
    const T w1 = T(L::wshell[1]), w2 = T(L::wshell[2]);
    T Fx = w1 * s1x + w2 * s2x, Fy = w1 * s1y + w2 * s2y, Fz = w1 * s1z + w2 * s2z;
    if constexpr (L::Q == 27) {
        const T w3 = T(L::wshell[3]);
        Fx += w3 * s3x;
        Fy += w3 * s3y;
        Fz += w3 * s3z;
    }
    Fx = gp * Fx + p.fext[0];
    Fy = gp * Fy + p.fext[1];
    Fz = gp * Fz + p.fext[2];

    // half-force velocity; an empty node has v = 0
    T ux = T(0), uy = T(0), uz = T(0);
    if (rho > T(0)) {
        const T inv = recip(rho);
        ux = (jx + T(0.5) * Fx) * inv;
        uy = (jy + T(0.5) * Fy) * inv;
        uz = (jz + T(0.5) * Fz) * inv;
    }
    const T om = p.omega, g = p.guo, omr = om * rho;
    const T A = omr * (T(1) - T(1.5) * (ux * ux + uy * uy + uz * uz)) - T(3) * g * (ux * Fx + uy * Fy + uz * Fz);
    const T B = T(3) * omr, C = T(4.5) * omr, D = T(3) * g, E = T(9) * g, keep = T(1) - om;
    f[0] = keep * f[0] + Dir<0, L>::template w<T>() * A;
    sfor<(L::Q - 1) / 2>([&](auto K) {
        constexpr int i = 2 * decltype(K)::value + 1;
        constexpr T w = Dir<i, L>::template w<T>();
        const T cu = T(Dir<i, L>::x) * ux + T(Dir<i, L>::y) * uy + T(Dir<i, L>::z) * uz;
        const T cF = T(Dir<i, L>::x) * Fx + T(Dir<i, L>::y) * Fy + T(Dir<i, L>::z) * Fz;
        const T even = A + cu * (C * cu + E * cF);
        const T odd = B * cu + D * cF;
        f[i] = keep * f[i] + w * (even + odd);
        f[i + 1] = keep * f[i + 1] + w * (even - odd);
    });

    // streaming
    if (!solid_dirs) {
        sfor<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (i > 0)
                stb(fout + (long long)i * Np, ns.template at<i>(is), pop_put<S>(f[i], Dir<i, L>::template w<T>() * rdst[i]));
        });
        stb(fout, is, pop_put<S>(f[0], Dir<0, L>::template w<T>() * rown));
        return;
    }
    const NbrU ne(x, y, z, nx, ny, nz, 1);
    T drho = T(0);
    if constexpr (L::kBits && sizeof(S) != 2) {
        // D3Q19, FP32 and FP64 populations: the owners of the solid neighbours come from one
        // round of gathers, then the reflections run body by body (wave-uniform loop) with the
        // body read once.  c_i . u_w at the link midpoint x + c_i/2 equals c_i . u_w(x), as
        // c_i . (omega x c_i) = 0, so the node's rigid velocity serves every link.  (Loads inside
        // per-link branches wait for memory once per link; this path keeps the interface waves
        // from trailing the pass.  The FP16-storage form keeps the per-link path: its encoded
        // reflections are sensitive to the rounding of the wall term.)
        uint32_t own[(L::Q + 7) / 8] = {};
        uint32_t touched = 0;
        sfor<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (i > 0) {
                const cell_t mw = ldb(mask, ne.template at<i>(idx) * 4u);
                if (!(solid_dirs & (1u << i))) {
                    stb(fout + (long long)i * Np, ns.template at<i>(is),
                        pop_put<S>(f[i], Dir<i, L>::template w<T>() * rdst[i]));
                } else {
                    const uint32_t o = (uint32_t)owner_of(mw);
                    own[i >> 3] |= o << (4 * (i & 7));
                    touched |= 1u << o;
                }
            }
        });
        for (int b = 0; b < p.nb; ++b) {
            if (!__ballot((touched >> b) & 1u)) continue;
            if (!((touched >> b) & 1u)) continue;
            const BodyDev &Bd = bodies[b];
            const double rx = mimg_r(x - Bd.X[0], nx, p.inv_n[0]), ry = mimg_r(y - Bd.X[1], ny, p.inv_n[1]),
                         rz = mimg_r(z - Bd.X[2], nz, p.inv_n[2]);
            const double u0x = Bd.V[0] + (Bd.W[1] * rz - Bd.W[2] * ry), u0y = Bd.V[1] + (Bd.W[2] * rx - Bd.W[0] * rz),
                         u0z = Bd.V[2] + (Bd.W[0] * ry - Bd.W[1] * rx);
            sfor<L::Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                if constexpr (i > 0) {
                    if ((solid_dirs & (1u << i)) && ((own[i >> 3] >> (4 * (i & 7))) & 15u) == (uint32_t)b) {
                        double cuw = 0.0;
                        if constexpr (Dir<i, L>::x != 0) cuw += Dir<i, L>::x * u0x;
                        if constexpr (Dir<i, L>::y != 0) cuw += Dir<i, L>::y * u0y;
                        if constexpr (Dir<i, L>::z != 0) cuw += Dir<i, L>::z * u0z;
                        const T gw = T(-6.0 * Dir<i, L>::template w<double>() * cuw) * rho;
                        stb(fout + (long long)Dir<i, L>::opp * Np, is,
                            pop_put<S>(f[i] + gw, Dir<i, L>::template w<T>() * rown));
                        drho += gw;
                    }
                }
            });
        }
    } else {
        sfor<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (i > 0) {
                if (!(solid_dirs & (1u << i))) {
                    stb(fout + (long long)i * Np, ns.template at<i>(is), pop_put<S>(f[i], Dir<i, L>::template w<T>() * rdst[i]));
                } else {
                    // reflected into direction opp(i) with g = -2 rho w_i (c_i . u_w) / c_s^2, u_w at
                    // the link midpoint x + c_i / 2
                    const BodyDev &Bd = bodies[owner_of(mask[ne.template at<i>(idx)])];
                    double uwx, uwy, uwz;
                    wall_velocity(p, Bd, x + 0.5 * Dir<i, L>::x, y + 0.5 * Dir<i, L>::y, z + 0.5 * Dir<i, L>::z, uwx, uwy, uwz);
                    const double cuw = Dir<i, L>::x * uwx + Dir<i, L>::y * uwy + Dir<i, L>::z * uwz;
                    const T gw = T(-6.0 * Dir<i, L>::template w<double>() * cuw) * rho;
                    stb(fout + (long long)Dir<i, L>::opp * Np, is, pop_put<S>(f[i] + gw, Dir<i, L>::template w<T>() * rown));
                    drho += gw;
                }
            }
        });
    }
    stb(fout, is, pop_put<S>(f[0] - drho, Dir<0, L>::template w<T>() * rown));
}

// Per-body force and torque sums of the step, one box node per thread (Sec. 3.1.1, 3.1.2, 3.2.2):
//  * fluid nodes next to solid nodes: momentum exchange c_i (2 f*_i + g) for each link into body
//    b, recovered from the reflected population f_opp(i) = f*_i + g written by k_collide_stream,
//    plus the pseudopotential reaction +G psi(x) w_i psi(varrho_b) c_i (opposite of the fluid's
//    share), with the link midpoint as lever arm;
//  * solid nodes (repulsion enabled): between a node p of body b1 and a node q of body b2 > b1
//    with |p - q| < r_c, f = e0 (n/r_c) (p - q)/|p - q| |(|p - q| - r_c)/r_c|^(n-1) on b1 at p
//    and -f on b2 at q; only nodes within r_c of a higher-index body's solid radius search.
// Torques are about the body centres X_b (minimum image).  Each wave reduces its contributions
// per touched body (64-lane shuffles) into LDS in a fixed order and every block writes FP64
// partials [body * 6 + component][block], summed by the first advection sweep (k_advect), which
// also advances the bodies.
// waves per block of the force scan (one block per CU), sized so that the gathered link values
// stay in registers: 12 in FP32, 8 in FP64
template <typename T, class L>
constexpr int force_waves() {
    return L::Q == 19 ? (sizeof(T) == 4 ? 12 : 8) : (sizeof(T) == 4 ? 8 : 4);
}

template <typename S, class L>
__global__ __launch_bounds__((64 * force_waves<ArT<S>, L>())) void k_body_forces(Prm<ArT<S>> p, int parity,
                                                     const StepState *st, const S *__restrict__ fin,
                                                     const S *__restrict__ fpost, const ArT<S> *__restrict__ psi,
                                                     const ArT<S> *__restrict__ psi_prev,
                                                     const cell_t *__restrict__ mask,
                                                     const BodyDev *__restrict__ bodies, double *part,
                                                     const uint32_t *__restrict__ nbw) {
    using T = ArT<S>;
    constexpr int W = force_waves<T, L>(), NT = 64 * W;
    __shared__ double acc[W][PF_LBM_MAX_BODIES][6];
    __shared__ double bt[W][PF_LBM_MAX_BODIES][9];  // X, V, W of every body
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int nbod = p.nb;
    // each wave clears and fills only its own row of the sums and reads its own copy of the body
    // motion (loaded here, off the dependent chain of the scan): no barrier before the scan
    for (int k = lane; k < PF_LBM_MAX_BODIES * 6; k += 64) (&acc[wave][0][0])[k] = 0.0;
    for (int k = lane; k < nbod * 9; k += 64) {
        const BodyDev &B = bodies[k / 9];
        const int c = k % 9;
        bt[wave][k / 9][c] = c < 3 ? B.X[c] : (c < 6 ? B.V[c - 3] : B.W[c - 6]);
    }
    __builtin_amdgcn_wave_barrier();
    const BoxIter it(st->box[parity], p.nx, p.ny, p.nz);
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const long long Np = p.Np;
    const bool rep = nbod > 1 && (p.flags & PF_LBM_REPULSION);
    const double rc = p.r_c;
    constexpr int RC = 16;  // repulsion offsets per round of loads
    for (int base = blockIdx.x * NT; base < it.vol; base += gridDim.x * NT) {
        const int k = base + tid;
        uint32_t touched = 0;
        int x = 0, y = 0, z = 0, idx = 0, b1 = -1;
        uint32_t nbits = 0;  // solid-neighbour bits of a fluid node
        bool fluid = false;
        T rho = T(0), ps0 = T(0);
        // per link i into a solid neighbour: its owner (4-bit fields) and the body-independent part
        // of the link force, a_i = 2 f_opp(i) + G psi(x) w_i psi(x + c_i)
        uint32_t own[(L::Q + 7) / 8] = {};
        T a[L::Q];
        if (k < it.vol) {
            int u[3], c[3];
            it.cell(k, u, c);
            x = c[0];
            y = c[1];
            z = c[2];
            idx = x + nx * (y + ny * z);
            const cell_t w0 = mask[idx];
            if (!(w0 & C_SOLID)) {
                fluid = true;
                uint32_t mo[L::Q];  // words of the neighbours
                const NbrU ne(x, y, z, nx, ny, nz, 1);
                if constexpr (L::kBits)
                    nbits = w0 & C_NBMASK;
                else
                    nbits = nbw[idx];
                if (nbits) {
                    // Every gather of the node is issued in one round and unconditionally (the
                    // neighbour values are cache-served), so the per-link selects below wait for
                    // memory once; loads inside the per-link branches were serialised, one
                    // memory latency per link.
                    const uint32_t ib = (uint32_t)idx * (uint32_t)sizeof(T);
                    const uint32_t is = (uint32_t)idx * (uint32_t)sizeof(S);
                    S fo[L::Q];  // reflected populations f_opp(i) written by k_collide_stream
                    T pn[L::Q];  // neighbour pseudopotentials
                    sfor<L::Q>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        if constexpr (i > 0) {
                            const uint32_t n = ne.template at<i>((uint32_t)idx);
                            mo[i] = ldb(mask, n * 4u);
                            fo[i] = ldb(fpost + (long long)Dir<i, L>::opp * Np, is);
                            pn[i] = ldb(psi, n * (uint32_t)sizeof(T));
                        }
                    });
                    rho = sizeof(S) == 2 ? ref_density(psi_prev[idx], p.rho0) : T(0);
                    sfor<L::Q>([&](auto I) { rho += (T)ldb(fin + (long long)I * Np, is); });
                    ps0 = ldb(psi, ib);
                    const T rown = sizeof(S) == 2 ? ref_density(ps0, p.rho0) : T(0);
                    const T gp = p.G * ps0;
                    sfor<L::Q>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        a[i] = T(0);
                        if constexpr (i > 0) {
                            if (nbits & (1u << i)) {
                                const uint32_t o = (uint32_t)owner_of(mo[i]);
                                own[i >> 3] |= o << (4 * (i & 7));
                                touched |= 1u << o;
                                a[i] = T(2) * pop_get<S>(fo[i], Dir<i, L>::template w<T>() * rown) +
                                       gp * Dir<i, L>::template w<T>() * pn[i];
                            }
                        }
                    });
                }
            } else if (rep) {
                // a solid node of body b1 within r_c of the solid radius of a body b2 > b1 may
                // have solid nodes of b2 within r_c: both bodies are marked, and the per-body
                // pass below finds the pairs (a pair-free mark adds zeros)
                b1 = owner_of(w0);
                for (int b2 = b1 + 1; b2 < nbod; ++b2) {
                    const double *BX = bt[wave][b2];
                    const double rx = mimg_r(x - BX[0], nx, p.inv_n[0]), ry = mimg_r(y - BX[1], ny, p.inv_n[1]),
                                 rz = mimg_r(z - BX[2], nz, p.inv_n[2]);
                    if (sqrt(rx * rx + ry * ry + rz * rz) < (double)st->srad[b2] + rc + 1e-3)
                        touched |= (1u << b1) | (1u << b2);
                }
            }
        }
        uint32_t wt = wave_or(touched);
        while (wt) {
            const int b = __ffs(wt) - 1;
            wt &= wt - 1;
            double v[6] = {0, 0, 0, 0, 0, 0};
            if ((touched & (1u << b)) && fluid) {
                // The link midpoint is x + c_i/2, so with r the node's offset from the centre:
                // c_i . u_w(x + c_i/2) = c_i . u_w(x) (the term c_i . (W x c_i)/2 vanishes) and
                // (r + c_i/2) x s c_i = r x s c_i.  The wall term needs the node's rigid velocity
                // only, and the torque is r x (sum of the link forces).
                const double *BX = bt[wave][b], *BV = BX + 3, *BW = BX + 6;
                const double rx = mimg_r(x - BX[0], nx, p.inv_n[0]), ry = mimg_r(y - BX[1], ny, p.inv_n[1]),
                             rz = mimg_r(z - BX[2], nz, p.inv_n[2]);
                const double u0x = BV[0] + (BW[1] * rz - BW[2] * ry), u0y = BV[1] + (BW[2] * rx - BW[0] * rz),
                             u0z = BV[2] + (BW[0] * ry - BW[1] * rx);
                double fx = 0.0, fy = 0.0, fz = 0.0;
                sfor<L::Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    if constexpr (i > 0) {
                        if ((nbits & (1u << i)) && ((own[i >> 3] >> (4 * (i & 7))) & 15u) == (uint32_t)b) {
                            double cuw = 0.0;
                            if constexpr (Dir<i, L>::x != 0) cuw += Dir<i, L>::x * u0x;
                            if constexpr (Dir<i, L>::y != 0) cuw += Dir<i, L>::y * u0y;
                            if constexpr (Dir<i, L>::z != 0) cuw += Dir<i, L>::z * u0z;
                            // moving-wall term g; the link carries 2 f*_i + g = 2 f_opp(i) - g to the
                            // body plus the pseudopotential reaction, both along c_i
                            const T g = T(-6.0 * Dir<i, L>::template w<double>() * cuw) * rho;
                            const double s = (double)(a[i] - g);
                            if constexpr (Dir<i, L>::x == 1) fx += s;
                            if constexpr (Dir<i, L>::x == -1) fx -= s;
                            if constexpr (Dir<i, L>::y == 1) fy += s;
                            if constexpr (Dir<i, L>::y == -1) fy -= s;
                            if constexpr (Dir<i, L>::z == 1) fz += s;
                            if constexpr (Dir<i, L>::z == -1) fz -= s;
                        }
                    }
                });
                v[0] = fx;
                v[1] = fy;
                v[2] = fz;
                v[3] = ry * fz - rz * fy;
                v[4] = rz * fx - rx * fz;
                v[5] = rx * fy - ry * fx;
            } else if (touched & (1u << b)) {
                // repulsion between this solid node p of body b1 and the solid nodes q = p + d of
                // bodies above b1: on b1 at p (b == b1), or the reaction on b at q (b != b1).  With
                // r the offset of p from the centre of b, the torque is r x (sum f) for b1 and
                // r x (sum f) + sum d x f for the reaction, so each pair costs a few additions.
                const bool react = b != b1;
                double sfx = 0.0, sfy = 0.0, sfz = 0.0, tdx = 0.0, tdy = 0.0, tdz = 0.0;
                const int nrep = st->n_rep;
                for (int j0 = 0; j0 < nrep; j0 += RC) {
                    cell_t mqs[RC];
#pragma unroll
                    for (int j = 0; j < RC; ++j) {
                        const int o = st->rep_off[j0 + j < nrep ? j0 + j : j0];
                        const int dx = (o & 255) - 8, dy = ((o >> 8) & 255) - 8, dz = (o >> 16) - 8;
                        mqs[j] = mask[wrapi(x + dx, nx) + nx * (wrapi(y + dy, ny) + ny * wrapi(z + dz, nz))];
                    }
#pragma unroll
                    for (int j = 0; j < RC; ++j) {
                        if (j0 + j >= nrep) break;
                        const cell_t mq = mqs[j];
                        if (!(mq & C_SOLID)) continue;
                        const int b2 = owner_of(mq);
                        if (b2 <= b1 || (react && b != b2)) continue;
                        // force on b1 at p, directed from q to p; its opposite on b2 at q
                        const double sg = react ? -1.0 : 1.0;
                        const double fx = sg * st->rep_f[j0 + j][0], fy = sg * st->rep_f[j0 + j][1],
                                     fz = sg * st->rep_f[j0 + j][2];
                        sfx += fx;
                        sfy += fy;
                        sfz += fz;
                        if (react) {
                            const int o = st->rep_off[j0 + j];
                            const double dx = (o & 255) - 8, dy = ((o >> 8) & 255) - 8, dz = (o >> 16) - 8;
                            tdx += dy * fz - dz * fy;
                            tdy += dz * fx - dx * fz;
                            tdz += dx * fy - dy * fx;
                        }
                    }
                }
                const double *BX = bt[wave][b];
                const double rx = mimg(x - BX[0], nx), ry = mimg(y - BX[1], ny), rz = mimg(z - BX[2], nz);
                v[0] = sfx;
                v[1] = sfy;
                v[2] = sfz;
                v[3] = ry * sfz - rz * sfy + tdx;
                v[4] = rz * sfx - rx * sfz + tdy;
                v[5] = rx * sfy - ry * sfx + tdz;
            }
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const double s = wave_sum(v[c]);
                if (lane == 0) acc[wave][b][c] += s;
            }
        }
    }
    __syncthreads();
    for (int k = tid; k < nbod * 6; k += NT) {
        const int b = k / 6, c = k % 6;
        double s = 0.0;
        for (int w = 0; w < W; ++w) s += acc[w][b][c];
        part[(long long)k * gridDim.x + blockIdx.x] = s;
    }
}

}  // namespace pfl
