// Fluid kernels of the step: the fluid pass (density and pseudopotential, force, Guo-BGK
// collision, push streaming with moving-wall bounce-back, in one read of the populations) and
// the per-body force/torque sums.
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

// ---- the fluid pass: density, pseudopotential, force, collision and push streaming -----------
//
// One pass over the populations per step.  A block owns a tile of 64 x TY nodes in the x-y plane
// and marches a chunk of tz planes along z.  The Shan-Chen/Benzi force at a node needs the
// pseudopotential of its 18 (26) neighbours at the same time level, so the block keeps a window
// of three planes of psi for its tile and a one-node halo in LDS: before colliding plane z it
// forms rho and psi of plane z + 1 from the post-stream populations (the tile's own nodes and
// the halo), so every population is read from HBM once.  The tile's own populations of plane
// z + 1 wait in LDS (each thread in its own slots) until plane z + 1 is collided; halo nodes
// and the two planes before and after the chunk cost a density-only read (mostly served by L2,
// where the neighbouring tiles read the same lines).  The pseudopotential of every node is
// written once, for the force scan and read-out.

// Collision and streaming of one fluid node (Sec. 3.2.1, 3.2.2, 3.2.3): sv holds its stored
// post-stream populations, psin(I) the pseudopotential of its neighbour in direction I, psi0 its
// own.  Forms the force from the neighbours' psi (solid neighbours act with their wetting
// density), collides with BGK + Guo forcing at the half-force velocity, and pushes each
// post-collision population to its neighbour, or, when the neighbour is solid (bit i of
// solid_dirs), reflects it half-way into the node's own opposite slot (with the moving-wall term
// where wall_in_fluid_pass).  rin: reference density of the node's stored inputs (FP16 storage).
//
// Arithmetic is organised by opposite pairs (c_opp = -c): with cu = c.v, cF = c.F,
//   f*_i = (1 - 1/tau) f_i + w (even + odd),  f*_opp = (1 - 1/tau) f_opp + w (even - odd),
//   even = rho/tau (1 - 3/2 v.v) - 3 g v.F + 9/2 rho/tau cu^2 + 9 g cu cF,  odd = 3 rho/tau cu + 3 g cF,
// g = 1 - 1/(2 tau), which is the BGK relaxation to the second-order equilibrium plus the Guo term.
// Where the moving-wall term of the bounce-back is added (Sec. 3.2.2).  FP32 and FP64: by the force
// scan, which visits exactly the nodes next to solids, so the fluid pass needs no body data and
// stays lean.  FP16 storage: in the fluid pass, so that the reflected population f*_i + g_i is
// rounded to FP16 once (adding g to an already rounded f*_i and rounding again was measured to
// triple the body-force error of the form).
template <typename S>
constexpr bool wall_in_fluid_pass() {
    return sizeof(S) == 2;
}

// Motion of every body for the moving-wall term of the FP16 form, staged in LDS by the fluid pass
// (centre FP64 for the minimum-image lever arm, velocities as the FP32 arithmetic uses them).
struct WallMot {
    double X[PF_LBM_MAX_BODIES][3];
    float V[PF_LBM_MAX_BODIES][3], W[PF_LBM_MAX_BODIES][3];
};

// psin(I): psi of the neighbour in direction I; FP16 form: refn(I) its reference density R (the
// encode of a population pushed there) and rown the node's own (the encode of its own slots),
// both R(psi) of this step's psi, formed once per node with the window
template <typename S, class L, typename PsiN, typename RefN>
__device__ __forceinline__ void collide_push(const Prm<ArT<S>> &p, const S *sv, ArT<S> rin, PsiN psin, RefN refn,
                                             ArT<S> psi0, ArT<S> rown, S *__restrict__ fout, uint32_t solid_dirs,
                                             int x, int y, int z,
                                             long long Np, const cell_t *__restrict__ mask,
                                             const WallMot *wm) {
    using T = ArT<S>;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const uint32_t idx = (uint32_t)(x + nx * (y + ny * z));
    const uint32_t is = idx * (uint32_t)sizeof(S);  // populations (storage type)
    const NbrU ns(x, y, z, nx, ny, nz, (int)sizeof(S));
    constexpr bool H = sizeof(S) == 2;  // FP16 storage: deviations from w_i R

    T f[L::Q];
    sfor<L::Q>([&](auto I) { f[I] = pop_get<S>(sv[I], Dir<decltype(I)::value, L>::template w<T>(), rin); });
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
    sfor<(L::Q - 1) / 2>([&](auto K) {
        constexpr int i = 2 * decltype(K)::value + 1;
        const T pa = psin(std::integral_constant<int, i>{}), pb = psin(std::integral_constant<int, i + 1>{});
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
    const T gp = -p.G * psi0;
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

    // streaming: push to the neighbour, or reflect half-way into the node's own opposite slot
    // when the neighbour is solid
    T drho = T(0);
    if (!solid_dirs) {
        sfor<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (i > 0)
                stb(fout + (long long)i * Np, ns.template at<i>(is), pop_put<S>(f[i], Dir<i, L>::template w<T>(), refn(I)));
        });
    } else if constexpr (!wall_in_fluid_pass<S>()) {
        // f*_i into slot opp(i); the force scan adds the moving-wall term and the mass correction
        sfor<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (i > 0) {
                if (!(solid_dirs & (1u << i)))
                    stb(fout + (long long)i * Np, ns.template at<i>(is), pop_put<S>(f[i], Dir<i, L>::template w<T>(), refn(I)));
                else
                    stb(fout + (long long)Dir<i, L>::opp * Np, is, pop_put<S>(f[i], Dir<i, L>::template w<T>(), rown));
            }
        });
    } else {
        // f*_i + g_i into slot opp(i), g_i = -2 rho w_i (c_i . u_w) / c_s^2 with u_w the rigid
        // velocity at the link midpoint x + c_i / 2; the rest population gives back the g_i.  The
        // solid neighbour's owner comes from its window entry and the bodies' motion from LDS, so
        // the links wait for no global load.
        sfor<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (i > 0) {
                if (!(solid_dirs & (1u << i))) {
                    stb(fout + (long long)i * Np, ns.template at<i>(is), pop_put<S>(f[i], Dir<i, L>::template w<T>(), refn(I)));
                } else {
                    // the FP16 form's collision arithmetic is FP32: the lever arm about the body
                    // centre (minimum image, FP64) and the wall velocity at the link midpoint in FP32
                    // (bounded to the body table whatever the entry holds)
                    const int o = __float_as_int(refn(I)) & (PF_LBM_MAX_BODIES - 1);
                    const T rx = (T)mimg_r(x - wm->X[o][0], nx, p.inv_n[0]) + T(0.5 * Dir<i, L>::x),
                            ry = (T)mimg_r(y - wm->X[o][1], ny, p.inv_n[1]) + T(0.5 * Dir<i, L>::y),
                            rz = (T)mimg_r(z - wm->X[o][2], nz, p.inv_n[2]) + T(0.5 * Dir<i, L>::z);
                    const T wx = wm->W[o][0], wy = wm->W[o][1], wz = wm->W[o][2];
                    const T uwx = wm->V[o][0] + (wy * rz - wz * ry), uwy = wm->V[o][1] + (wz * rx - wx * rz),
                            uwz = wm->V[o][2] + (wx * ry - wy * rx);
                    const T cuw = T(Dir<i, L>::x) * uwx + T(Dir<i, L>::y) * uwy + T(Dir<i, L>::z) * uwz;
                    const T gw = T(-6.0 * Dir<i, L>::template w<double>()) * cuw * rho;
                    stb(fout + (long long)Dir<i, L>::opp * Np, is, pop_put<S>(f[i] + gw, Dir<i, L>::template w<T>(), rown));
                    drho += gw;
                }
            }
        });
    }
    stb(fout, is, pop_put<S>(f[0] - drho, Dir<0, L>::template w<T>(), rown));
}

// LDS of the fluid pass: the psi window (3 planes of the tile and its halo, 66 x (TY + 2)), the
// tile's populations of the plane being collided ([direction][node of the tile], stored form),
// and, where the budget allows (DMA), the halo's populations, cell words and previous psi of
// two planes, loaded straight into LDS.
// entry of the psi window: psi, and in the FP16 form beside it the reference density R(psi) of a
// fluid node (formed once per node instead of once per population pushed to it) or, for a solid
// node (never a push destination), the index of its owner as an integer bit pattern (the moving-
// wall term of a link into it reads the owner from the window instead of the cell word)
template <typename S>
using WinE = std::conditional_t<sizeof(S) == 2, float2, ArT<S>>;
template <typename S>
__device__ __forceinline__ ArT<S> win_psi(const WinE<S> &e) {
    if constexpr (sizeof(S) == 2)
        return e.x;
    else
        return e;
}
template <typename S>
__device__ __forceinline__ ArT<S> win_ref(const WinE<S> &e) {
    if constexpr (sizeof(S) == 2)
        return e.y;
    else
        return ArT<S>(0);
}
template <typename S>
__device__ __forceinline__ WinE<S> win_entry(ArT<S> psi, ArT<S> rho0, cell_t m) {
    if constexpr (sizeof(S) == 2)
        return make_float2(psi, (m & C_SOLID) ? __int_as_float(owner_of(m)) : ref_density(psi, rho0));
    else
        return psi;
}

template <typename S, class L, int TY, bool DMA>
struct FluidLds {
    // halo entries: the rows below and above the tile (64 each), the two columns (TY + 2 each)
    static constexpr int NH = DMA ? 128 + 2 * (TY + 2) : 1, NB = DMA ? 2 : 1;
    WinE<S> ring[3][TY + 2][66];
    std::conditional_t<wall_in_fluid_pass<S>(), WallMot, char> wm;  // bodies' motion (FP16 form)
    S pop[L::Q][64 * TY];
    S hpop[NB][L::Q][NH];
    cell_t hmask[NB][NH];
};
// Tile shapes of the fluid pass: TY rows of 64 nodes, W waves per block, each thread owning
// RPT = TY / W rows.  LDS stays within 80 KB so that two blocks share a CU (160 KB).
template <int TY>
struct FluidShape {
    static constexpr int W = TY <= 4 ? 4 : 8, RPT = TY / W;
};
constexpr size_t FLUID_LDS_MAX = 80 * 1024;
template <typename S, class L, int TY>
constexpr bool fluid_tile_fits() {
    return sizeof(FluidLds<S, L, TY, false>) <= FLUID_LDS_MAX;
}
// direct loads into LDS move one dword per lane (a shorter element would still take a dword slot
// of LDS per lane): FP32 populations only
template <typename S, class L, int TY>
constexpr bool fluid_halo_dma() {
    return sizeof(S) == 4 && sizeof(FluidLds<S, L, TY, true>) <= FLUID_LDS_MAX;
}

// one node's inputs of one plane: its stored populations, cell word and (FP16) previous psi
template <typename S, class L>
struct NodeIn {
    S v[L::Q];
    cell_t m;
    ArT<S> pp;
};

// psi of a node from its inputs (Sec. 3.2.3): fluid 1 - exp(-rho/rho0) with rho the sum of the
// populations (FP16: rho = R + sum of the stored deviations, the weights summing to one); a
// solid node carries the value of its body's wetting density.  v(I): stored population I.
template <typename S, class L, typename V>
__device__ __forceinline__ ArT<S> node_psi_of(const Prm<ArT<S>> &p, const BodyDev *__restrict__ bodies, cell_t m,
                                              ArT<S> pp, V v) {
    using T = ArT<S>;
    if (m & C_SOLID) return (T)bodies[owner_of(m)].psi_s;
    T r = T(0);
    if constexpr (sizeof(S) == 2) r = ref_density(pp, p.rho0);
    sfor<L::Q>([&](auto I) { r += (T)v(I); });
    return -expm1(-r * p.inv_rho0);
}

// The fluid pass (see above).  Launch: 64 W threads per block (W waves, one x-row of 64 nodes
// per wave and row set), tiles of 64 x TY nodes (thread (tx, w) owns rows w, w + W, ..), a 1-D
// grid of ceil(nx/64) * ceil(ny/TY) * ceil(nz/tz) blocks; blocks are ordered so that each XCD
// holds a contiguous run of tiles (a z-chunk of neighbouring tiles shares an L2).
//
// Software pipeline along z: while plane z is collided, the tile's own populations of plane z + 2
// are in flight into registers and (DMA) the halo's straight into LDS; at the top of the next
// pass they have landed, psi of plane z + 2 is formed, and so on.  Instantiations whose halo
// buffers do not fit the LDS budget load the halo of each plane just before its psi is formed.
//
// With bodies, the first block also publishes the step's box, solid radii, volume terms and event
// flag from the previous reclassification (publish_step_state) before its own cells: that short
// reduction chain then hides behind the longest pass of the step instead of costing a launch.
template <typename S, class L, int TY>
__global__ __launch_bounds__(64 * FluidShape<TY>::W) void k_collide_stream(Prm<ArT<S>> p, const S *__restrict__ fin,
                                                                     S *__restrict__ fout, ArT<S> *__restrict__ psi,
                                                                     const ArT<S> *__restrict__ psi_prev,
                                                                     const cell_t *__restrict__ mask, BodyDev *bodies,
                                                                     int parity, StepState *st,
                                                                     const ClassifyPart *__restrict__ cpart, int cblk,
                                                                     const uint32_t *__restrict__ nbw, int tz) {
    using T = ArT<S>;
    constexpr int W = FluidShape<TY>::W, RPT = FluidShape<TY>::RPT;
    constexpr bool DMA = fluid_halo_dma<S, L, TY>();
    static_assert(fluid_tile_fits<S, L, TY>(), "LDS of the fluid pass above its budget");
    __shared__ FluidLds<S, L, TY, DMA> lds;
    constexpr bool H = sizeof(S) == 2;
    const int tid = (int)threadIdx.x, tx = tid & 63, wv = tid >> 6;
    if (cpart && blockIdx.x == 0)
        publish_step_state(wv, W, parity, p.nx, p.ny, p.nz, p.nb, p.eta, st, bodies, cpart, cblk);
    // FP16 form: the bodies' motion for the moving-wall term into LDS (ordered before its first
    // use by the prologue's barrier)
    if constexpr (wall_in_fluid_pass<S>()) {
        for (int k = tid; k < p.nb * 9; k += 64 * W) {
            const int b = k / 9, c = k % 9;
            if (c < 3)
                lds.wm.X[b][c] = bodies[b].X[c];
            else if (c < 6)
                lds.wm.V[b][c - 3] = (float)bodies[b].V[c - 3];
            else
                lds.wm.W[b][c - 6] = (float)bodies[b].W[c - 6];
        }
    }
    auto wall_mot = [&]() -> const WallMot * {
        if constexpr (wall_in_fluid_pass<S>())
            return &lds.wm;
        else
            return nullptr;
    };
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int tiles_x = (nx + 63) / 64, tiles_y = (ny + TY - 1) / TY, tiles = tiles_x * tiles_y;
    const int b = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int chunk = b / tiles, tile = b - chunk * tiles;
    const int tyi = tile / tiles_x, txi = tile - tyi * tiles_x;
    const int x0 = txi * 64, y0 = tyi * TY, zs = chunk * tz, ze = min(zs + tz, nz);
    const int x = x0 + tx;
    const uint32_t pl = (uint32_t)nx * (uint32_t)ny;
    // rows of this thread: ty = wv + W r; the node whose psi its window entry holds (a partial
    // tile's entries past the grid edge hold the periodic images the last nodes need)
    bool valid[RPT];
    uint32_t own_xy[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int y = y0 + wv + W * r;
        valid[r] = x < nx && y < ny;
        own_xy[r] = (uint32_t)wrapi(x, nx) + (uint32_t)nx * (uint32_t)wrapi(y, ny);
    }
    // halo entry of this thread: row ly = -1 (wave 0), row ly = TY (wave 1), the two columns
    // lx = -1 and 64 for ly = -1..TY (wave 3, lanes 0 .. 2 TY + 3); hs: the wave's 64 entries
    // in the halo buffers
    int hlx = 0, hly = 0, hs = 0;
    bool halo = false;
    if (wv == 0 || wv == 1) {
        halo = true;
        hlx = tx;
        hly = wv == 0 ? -1 : TY;
        hs = 64 * wv;
    } else if (wv == 3) {
        halo = tx < 2 * (TY + 2);
        hlx = (tx & 1) ? 64 : -1;
        hly = (tx >> 1) - 1;
        hs = 128;
    }
    const uint32_t halo_xy = (uint32_t)wrapi(x0 + hlx, nx) + (uint32_t)nx * (uint32_t)wrapi(y0 + hly, ny);
    auto slot = [&](int zz) { return (zz - zs + 1) % 3; };
    auto hbuf = [&](int zz) { return DMA ? ((zz - zs + 1) & 1) : 0; };
    // The plane stride is re-read (opaque to the compiler) in every pass of the loop, so the 2 Q
    // plane addresses are formed on the scalar unit where they are used instead of being hoisted
    // out of the loop, where they would occupy more scalar registers than there are.
    auto plane_stride = [&]() {
        long long np = p.Np;
        asm volatile("" : "+s"(np));
        return np;
    };
    // loads of the own nodes' inputs of plane zz (issued, not waited for)
    auto load_own = [&](int zz, NodeIn<S, L> (&o)[RPT]) {
        const uint32_t zo = pl * (uint32_t)wrapi(zz, nz);
        const long long np = plane_stride();
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const uint32_t idx = own_xy[r] + zo;
            o[r].m = mask[idx];
            o[r].pp = H ? psi_prev[idx] : T(0);
            const uint32_t is = idx * (uint32_t)sizeof(S);
            sfor<L::Q>([&](auto I) { o[r].v[I] = ldb(fin + (long long)I * np, is); });
        }
    };
    // the halo's inputs of plane zz straight into LDS buffer hb (DMA)
    // halo inputs of the plane in flight, where they go through registers (no DMA): prefetched one
    // pass ahead in the FP16 form; the FP64 form, short of registers, loads them when it needs them
    constexpr bool HPRE = !DMA && sizeof(S) == 2;
    NodeIn<S, L> hin;
    auto halo_load = [&](int zz, NodeIn<S, L> &o) {
        const uint32_t hidx = halo_xy + pl * (uint32_t)wrapi(zz, nz);
        const long long np = plane_stride();
        o.m = mask[hidx];
        o.pp = H ? psi_prev[hidx] : T(0);
        const uint32_t is = hidx * (uint32_t)sizeof(S);
        sfor<L::Q>([&](auto I) { o.v[I] = ldb(fin + (long long)I * np, is); });
    };
    // the halo's inputs of plane zz: straight into LDS buffer hb (DMA), else into registers
    // (issued, not waited for; in the prologue, prefetch = false, halo_psi loads them itself)
    auto halo_issue = [&](int zz, int hb, bool prefetch) {
        if constexpr (!DMA) {
            if (HPRE && prefetch && halo) halo_load(zz, hin);
        } else {
            if (!halo) return;
            const uint32_t hidx = halo_xy + pl * (uint32_t)wrapi(zz, nz);
            const long long np = plane_stride();
            sfor<L::Q>([&](auto I) {
                __builtin_amdgcn_global_load_lds(
                    (const __attribute__((address_space(1))) void *)(fin + (long long)I * np + hidx),
                    (__attribute__((address_space(3))) void *)&lds.hpop[hb][I][hs], 4, 0, 0);
            });
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(mask + hidx),
                                             (__attribute__((address_space(3))) void *)&lds.hmask[hb][hs], 4, 0, 0);
        }
    };
    // psi of the halo entry of plane zz into the window: from the LDS buffer (DMA), from the
    // registers prefetched one pass earlier (prefetched), or loaded now (prologue)
    auto halo_psi = [&](int zz, bool prefetched) {
        if (!halo) return;
        T hp;
        cell_t hm;
        if constexpr (DMA) {
            const int hb = hbuf(zz), k = hs + tx;
            hm = lds.hmask[hb][k];
            hp = node_psi_of<S, L>(p, bodies, hm, T(0), [&](auto I) { return lds.hpop[hb][decltype(I)::value][k]; });
        } else {
            if (!(HPRE && prefetched)) halo_load(zz, hin);
            hm = hin.m;
            hp = node_psi_of<S, L>(p, bodies, hin.m, hin.pp, [&](auto I) { return hin.v[decltype(I)::value]; });
        }
        lds.ring[slot(zz)][hly + 1][hlx + 1] = win_entry<S>(hp, p.rho0, hm);
    };
    auto own_psi = [&](int zz, const NodeIn<S, L> (&o)[RPT]) {
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            lds.ring[slot(zz)][wv + W * r + 1][tx + 1] = win_entry<S>(
                node_psi_of<S, L>(p, bodies, o[r].m, o[r].pp, [&](auto I) { return o[r].v[decltype(I)::value]; }),
                p.rho0, o[r].m);
    };

    NodeIn<S, L> A[RPT], B[RPT];
    // prologue: psi of planes zs - 1 and zs, populations of plane zs into LDS, plane zs + 1 in
    // flight
    load_own(zs - 1, A);
    own_psi(zs - 1, A);
    halo_issue(zs - 1, hbuf(zs - 1), false);
    halo_issue(zs, hbuf(zs), false);
    load_own(zs, A);
    load_own(zs + 1, B);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    halo_psi(zs - 1, false);
    halo_psi(zs, false);
    own_psi(zs, A);
#pragma unroll
    for (int r = 0; r < RPT; ++r) sfor<L::Q>([&](auto I) { lds.pop[I][tid + 64 * W * r] = A[r].v[I]; });
    cell_t cm[RPT];  // cell words of the plane being collided
    T cpp[RPT];      // and their previous psi (FP16)
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        cm[r] = A[r].m;
        cpp[r] = A[r].pp;
    }
    halo_issue(zs + 1, hbuf(zs + 1), true);
    for (int z = zs; z < ze; ++z) {
        // plane z + 1 has landed (own populations in B, halo in its LDS buffer); every wave is done
        // with the previous plane's window entries and halo buffer
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        own_psi(z + 1, B);
        halo_psi(z + 1, true);
#pragma unroll
        for (int r = 0; r < RPT; ++r) A[r] = B[r];
        if (z + 2 <= ze) {
            load_own(z + 2, B);
            halo_issue(z + 2, hbuf(z + 2), true);
        }
        __syncthreads();
        const uint32_t zo = pl * (uint32_t)z;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int ty = wv + W * r;
            // own populations of plane z from LDS, those of plane z + 1 in their place
            S cur[L::Q];
            sfor<L::Q>([&](auto I) { cur[I] = lds.pop[I][tid + 64 * W * r]; });
            sfor<L::Q>([&](auto I) { lds.pop[I][tid + 64 * W * r] = A[r].v[I]; });
            // the stores stay here, ahead of the collision (sunk below it, they would keep the next
            // plane's populations in registers through the collision)
            asm volatile("" ::: "memory");
            if (valid[r]) {
                const uint32_t idx = own_xy[r] + zo;
                // the node's entry in each window plane: neighbours are fixed offsets from it
                const WinE<S> *rm = &lds.ring[slot(z - 1)][ty + 1][tx + 1], *r0 = &lds.ring[slot(z)][ty + 1][tx + 1],
                              *rp = &lds.ring[slot(z + 1)][ty + 1][tx + 1];
                const T psi0 = win_psi<S>(*r0);
                psi[idx] = psi0;
                const cell_t w0 = cm[r];
                if (!(w0 & C_SOLID)) {
                    // bit i: the neighbour in direction i is solid (D3Q19: kept in the cell word;
                    // D3Q27: the neighbour-bit word of the node)
                    uint32_t solid_dirs;
                    if constexpr (L::kBits)
                        solid_dirs = w0 & C_NBMASK;
                    else
                        solid_dirs = nbw[idx];
                    const T rin = H ? ref_density(cpp[r], p.rho0) : T(0);  // reference of the inputs
                    // the neighbour's window entry: fixed offsets from the node's
                    auto nbr = [&](auto I) -> const WinE<S> & {
                        constexpr int i = decltype(I)::value;
                        constexpr int o = Dir<i, L>::y * 66 + Dir<i, L>::x;
                        return Dir<i, L>::z < 0 ? rm[o] : (Dir<i, L>::z > 0 ? rp[o] : r0[o]);
                    };
                    collide_push<S, L>(
                        p, cur, rin, [&](auto I) { return win_psi<S>(nbr(I)); },
                        [&](auto I) { return win_ref<S>(nbr(I)); }, psi0, win_ref<S>(*r0), fout, solid_dirs, x,
                        y0 + ty, z, plane_stride(), mask, wall_mot());
                }
            }
            cm[r] = A[r].m;
            cpp[r] = A[r].pp;
        }
    }
}

// Per-body force and torque sums of the step over the box nodes (Sec. 3.1.1, 3.1.2, 3.2.2):
//  * fluid nodes next to solid nodes: the fluid pass reflected each population f*_i heading into
//    a solid node into the node's opposite slot; unless the fluid pass did so (wall_in_fluid_pass),
//    this kernel completes the moving-wall bounce-back of Sec. 3.2.2 there -- the slot becomes
//    f*_i + g_i with g_i = -2 rho w_i (c_i . u_w) / c_s^2 and the rest population gives back the
//    sum of the g_i (mass correction) -- and it adds to body b the momentum exchange
//    c_i (2 f*_i + g_i) of each link into b, plus the pseudopotential reaction
//    +G psi(x) w_i psi(varrho_b) c_i (opposite of the fluid's share), with the link midpoint as
//    lever arm;
//  * solid nodes (repulsion enabled): between a node p of body b1 and a node q of body b2 > b1
//    with |p - q| < r_c, f = e0 (n/r_c) (p - q)/|p - q| |(|p - q| - r_c)/r_c|^(n-1) on b1 at p
//    and -f on b2 at q; only nodes within r_c of a higher-index body's solid radius search.
// Torques are about the body centres X_b (minimum image).  Each wave reduces its contributions
// per touched body (64-lane shuffles) into LDS in a fixed order and every block writes FP64
// partials [body * 6 + component][block], summed by the first advection sweep (k_advect), which
// also advances the bodies.
// waves per block of the force scan (one block per CU), sized so that the gathered link values
// (reflected populations and link forces of every direction) stay in registers: 8 on D3Q19, 8 in
// FP32 and 4 in FP64 on D3Q27
template <typename T, class L>
constexpr int force_waves() {
    return L::Q == 19 ? 8 : (sizeof(T) == 4 ? 8 : 4);
}

template <typename S, class L>
__global__ __launch_bounds__((64 * force_waves<ArT<S>, L>())) void k_body_forces(Prm<ArT<S>> p, int parity,
                                                     const StepState *st, const S *__restrict__ fin,
                                                     S *__restrict__ fpost, const ArT<S> *__restrict__ psi,
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
    constexpr int RC = 32;  // repulsion offsets per round of loads
    // Each wave takes U rows of 64 consecutive box cells, the rows nw * 64 cells apart (nw waves in
    // the grid), so that the cells with work -- clustered on the bodies' surfaces and, for the
    // repulsion, in the small caps where two bodies nearly touch -- spread over all waves.  A first
    // pass loads the U cell words of each lane in one round and keeps the cells that need the
    // per-link (or repulsion) work: fluid cells with a solid neighbour, and solid cells within r_c of
    // the solid radius of a higher-index body.  The second pass runs that work on the kept cells
    // only, 64 per round, so the cells without a link cost one load in a wide round each.
    constexpr int U = 8;
    __shared__ int keep[W][64 * U];
    __shared__ double rsum[W][9][64];  // per-lane repulsion sums of the current round
    const int gw = (int)blockIdx.x * W + wave, nw = (int)gridDim.x * W;
    for (int run = gw * 64; run < it.vol; run += nw * 64 * U) {
        int nkeep = 0;
        {
            cell_t wk[U];
            int ck[U][3];
            bool in[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = run + nw * 64 * u + lane;
                in[u] = k < it.vol;
                int uu[3];
                it.cell(in[u] ? k : 0, uu, ck[u]);
                wk[u] = in[u] ? mask[ck[u][0] + nx * (ck[u][1] + ny * ck[u][2])] : cell_t(C_SOLID);
            }
            uint32_t nbk[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if constexpr (L::kBits)
                    nbk[u] = wk[u] & C_NBMASK;
                else
                    nbk[u] = (in[u] && !(wk[u] & C_SOLID)) ? nbw[ck[u][0] + nx * (ck[u][1] + ny * ck[u][2])] : 0u;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                bool need = false;
                if (in[u]) {
                    if (!(wk[u] & C_SOLID)) {
                        need = nbk[u] != 0;
                    } else if (rep) {
                        const int o1 = owner_of(wk[u]);
                        for (int b2 = o1 + 1; b2 < nbod; ++b2) {
                            const double *BX = bt[wave][b2];
                            const double rx = mimg_r(ck[u][0] - BX[0], nx, p.inv_n[0]),
                                         ry = mimg_r(ck[u][1] - BX[1], ny, p.inv_n[1]),
                                         rz = mimg_r(ck[u][2] - BX[2], nz, p.inv_n[2]);
                            if (sqrt(rx * rx + ry * ry + rz * rz) < (double)st->srad[b2] + rc + 1e-3) need = true;
                        }
                    }
                }
                const uint64_t bal = __ballot(need);
                if (need) keep[wave][nkeep + __popcll(bal & ((1ull << lane) - 1ull))] = run + nw * 64 * u + lane;
                nkeep += __popcll(bal);
            }
        }
        __builtin_amdgcn_wave_barrier();
        for (int j0 = 0; j0 < nkeep; j0 += 64) {
            const bool has = j0 + lane < nkeep;
            const int k = has ? keep[wave][j0 + lane] : 0;
            uint32_t touched = 0;
            int x = 0, y = 0, z = 0, idx = 0, b1 = -1;
            // repulsion of a solid node p of body b1: the first body rb2 > b1 met in the search
            int rb2 = -1;
            bool rmulti = false;
            uint32_t nbits = 0;  // solid-neighbour bits of a fluid node
            bool fluid = false;
            T rho = T(0), ps0 = T(0), rown = T(0), drho = T(0);
            // per link i into a solid neighbour: its owner (4-bit fields), the reflected post-collision
            // population fr_i = f*_i and the body-independent part of the link force, a_i = 2 f*_i +
            // G psi(x) w_i psi(x + c_i); drho sums the moving-wall terms of the node's links
            uint32_t own[(L::Q + 7) / 8] = {};
            T a[L::Q], fr[L::Q];
            if (has) {
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
                        S fo[L::Q];  // reflected populations f*_i, in slot opp(i), written by the fluid pass
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
                        rown = sizeof(S) == 2 ? ref_density(ps0, p.rho0) : T(0);
                        const T gp = p.G * ps0;
                        sfor<L::Q>([&](auto I) {
                            constexpr int i = decltype(I)::value;
                            a[i] = T(0);
                            fr[i] = T(0);
                            if constexpr (i > 0) {
                                if (nbits & (1u << i)) {
                                    const uint32_t o = (uint32_t)owner_of(mo[i]);
                                    own[i >> 3] |= o << (4 * (i & 7));
                                    touched |= 1u << o;
                                    // reflected value: f*_i, or f*_i + g_i where the fluid pass added g
                                    fr[i] = pop_get<S>(fo[i], Dir<i, L>::template w<T>(), rown);
                                    a[i] = T(2) * fr[i] + gp * Dir<i, L>::template w<T>() * pn[i];
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
                    if (touched) {
                        // one pass over the offsets within r_c: the force on b1 from every body
                        // above it (rs1), and the reaction on the first such body met with its
                        // lever-arm part sum d x f (rs2, rt2), kept in the lane's LDS slots for the
                        // per-body loop; a second body met gets its reaction from a pass of its own
                        double rs1[3] = {0.0, 0.0, 0.0}, rs2[3] = {0.0, 0.0, 0.0}, rt2[3] = {0.0, 0.0, 0.0};
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
                                if (b2 <= b1) continue;
                                rs1[0] += st->rep_f[j0 + j][0];
                                rs1[1] += st->rep_f[j0 + j][1];
                                rs1[2] += st->rep_f[j0 + j][2];
                                if (rb2 < 0) rb2 = b2;
                                if (b2 != rb2) {
                                    rmulti = true;
                                    continue;
                                }
                                const double fx = -1.0 * st->rep_f[j0 + j][0], fy = -1.0 * st->rep_f[j0 + j][1],
                                             fz = -1.0 * st->rep_f[j0 + j][2];
                                rs2[0] += fx;
                                rs2[1] += fy;
                                rs2[2] += fz;
                                const int o = st->rep_off[j0 + j];
                                const double dx = (o & 255) - 8, dy = ((o >> 8) & 255) - 8, dz = (o >> 16) - 8;
                                rt2[0] += dy * fz - dz * fy;
                                rt2[1] += dz * fx - dx * fz;
                                rt2[2] += dx * fy - dy * fx;
                            }
                        }
                        for (int c = 0; c < 3; ++c) {
                            rsum[wave][c][lane] = rs1[c];
                            rsum[wave][3 + c][lane] = rs2[c];
                            rsum[wave][6 + c][lane] = rt2[c];
                        }
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
                                // moving-wall term g: the reflected population becomes f*_i + g (Sec.
                                // 3.2.2); the link carries 2 f*_i + g to the body plus the
                                // pseudopotential reaction, both along c_i
                                const T g = T(-6.0 * Dir<i, L>::template w<double>() * cuw) * rho;
                                double s;
                                if constexpr (!wall_in_fluid_pass<S>()) {
                                    stb(fpost + (long long)Dir<i, L>::opp * Np, (uint32_t)idx * (uint32_t)sizeof(S),
                                        pop_put<S>(fr[i] + g, Dir<i, L>::template w<T>(), rown));
                                    drho += g;
                                    s = (double)(a[i] + g);
                                } else {
                                    s = (double)(a[i] - g);  // 2 (f*_i + g) - g
                                }
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
                    if (b == b1) {
                        sfx = rsum[wave][0][lane];
                        sfy = rsum[wave][1][lane];
                        sfz = rsum[wave][2][lane];
                    } else if (b == rb2) {
                        sfx = rsum[wave][3][lane];
                        sfy = rsum[wave][4][lane];
                        sfz = rsum[wave][5][lane];
                        tdx = rsum[wave][6][lane];
                        tdy = rsum[wave][7][lane];
                        tdz = rsum[wave][8][lane];
                    }
                    // the reaction on a further body (rare): a pass of its own
                    const int nrep = react && b != rb2 && rmulti ? st->n_rep : 0;
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
            if (!wall_in_fluid_pass<S>() && fluid && nbits) {
                // the rest population gives back the moving-wall terms (mass correction, Sec. 3.2.2)
                const uint32_t is = (uint32_t)idx * (uint32_t)sizeof(S);
                const T f0 = pop_get<S>(ldb(fpost, is), Dir<0, L>::template w<T>(), rown);
                stb(fpost, is, pop_put<S>(f0 - drho, Dir<0, L>::template w<T>(), rown));
            }
        }
        __builtin_amdgcn_wave_barrier();
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
