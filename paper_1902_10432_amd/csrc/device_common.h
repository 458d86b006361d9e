// Device-side building blocks of the coupled phase-field / lattice-Boltzmann step for gfx950:
// the D3Q19 and D3Q27 velocity sets as compile-time constants, the mask byte layout, the body table and
// the per-step state shared by the kernels, wave64 reductions and the XCD-aware block order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "../../include/pf_lbm.h"

namespace pfl {

// ---- velocity sets.  Sec. 3.2.1 prints D3Q27; the named workloads run D3Q19 (both share
// c_s^2 = 1/3 and the second and fourth moments).  One direction table serves both: the rest
// direction, 6 faces, 12 edges (the D3Q19 set), then the 8 corners; pairs (2k-1, 2k) are
// opposite.  Weights by speed shell |c|^2 = 0..3.
constexpr int kCX[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
constexpr int kCY[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, -1, 1, 1, -1};
constexpr int kCZ[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, 1, -1};

struct D3Q19 {
    static constexpr int Q = 19;
    // the cell word carries one solid-neighbour bit per direction
    static constexpr bool kBits = true;
    static constexpr double wshell[4] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0, 0.0};
};
struct D3Q27 {
    static constexpr int Q = 27;
    // 26 neighbour bits do not fit beside the flags: they live in a word array of their own
    static constexpr bool kBits = false;
    static constexpr double wshell[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0};
};

template <int I, class L = D3Q19>
struct Dir {
    static constexpr int x = kCX[I], y = kCY[I], z = kCZ[I];
    static constexpr int opp = I == 0 ? 0 : ((I & 1) ? I + 1 : I - 1);
    static constexpr int c2 = x * x + y * y + z * z;
    template <typename T>
    __device__ static constexpr T w() {
        return T(L::wshell[c2]);
    }
};

// compile-time loop: f(std::integral_constant<int, i>) for i = 0..N-1
template <typename F, int... Is>
__device__ __forceinline__ void sfor_impl(F &&f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void sfor(F &&f) {
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// ---- cell word (one uint32 per node): bit 31 solid, bit 30 became solid this step, bit 29
// became fluid this step, bits 24-28 owning body of a solid node, bit i (1..18) set when the
// neighbour in direction i is solid (D3Q19 only; kept current inside the body box by k_post)
using cell_t = uint32_t;
constexpr uint32_t C_SOLID = 1u << 31, C_F2S = 1u << 30, C_S2F = 1u << 29, C_NBMASK = 0x7FFFEu;
__device__ __forceinline__ int owner_of(uint32_t w) { return (int)((w >> 24) & 31u); }
__device__ __forceinline__ uint32_t solid_word(int owner) { return C_SOLID | ((uint32_t)owner << 24); }

// load / store at a byte offset from a uniform base (lets the compiler use scalar-base addressing)
template <typename T>
__device__ __forceinline__ T ldb(const T *base, uint32_t byteoff) {
    return *(const T *)((const char *)base + byteoff);
}
template <typename T>
__device__ __forceinline__ void stb(T *base, uint32_t byteoff, T v) {
    *(T *)((char *)base + byteoff) = v;
}

// ---- body table (FP64, device resident)
struct BodyDev {
    double M, Iinv[9];
    double X[3], V[3], W[3];
    double F[3], T[3];   // totals of the last step
    double psi_s;        // psi(varrho) of the body's solid nodes
    double Vref;         // sum phi at t = 0
    double h;            // volume driving term (4 eta / pi^2) (Vref - V) / |interface|
    int32_t fixed, pad;
};

// Per-step state shared by the kernels.  Boxes are in unwrapped lattice coordinates
// [lo, hi] per axis (hi - lo + 1 <= n); box[p] is read by step parity p, written for the next.
struct StepState {
    int32_t box[2][6];            // lo x, lo y, lo z, hi x, hi y, hi z
    uint32_t err;                 // bit 0 non-finite body state, bit 1 advection CFL above 1
    uint32_t n_events;            // nodes that changed side in this step's reclassification
    uint32_t step_no, pad;        // steps started (counted by the step-state publish)
    unsigned long long n_f2s, n_s2f, n_lost;
    float srad[PF_LBM_MAX_BODIES];  // largest distance of a solid node from its body's centre
    // offsets (dx, dy, dz) with 0 < |d|^2 < r_c^2 in scan order (dz, dy, dx increasing), packed as
    // (dx + 8) | (dy + 8) << 8 | (dz + 8) << 16; at most 250 for r_c <= 4
    int32_t n_rep, rep_off[256];
    // force on p from a node q = p + d of another body (Sec. 3.1.2):
    // -(d / |d|) e0 (n / r_c) |(|d| - r_c) / r_c|^(n - 1)
    double rep_f[256][3];
};

// per-block results of the reclassification kernel, combined at the start of the next step
struct ClassifyPart {
    int32_t lo[3], hi[3];           // bounding box of the phase-field support (unwrapped)
    uint32_t f2s, s2f;              // nodes that became solid / fluid
    float srad[PF_LBM_MAX_BODIES];  // per-body largest solid-node distance from the centre
    double vol[PF_LBM_MAX_BODIES];  // per-body sum of phi
    uint32_t icnt[PF_LBM_MAX_BODIES];  // per-body count of interface nodes phi_floor < phi < 1
};

// Deterministic sum of v[0..n) by one wave: lane l accumulates v[l + 64 m] into four
// interleaved partial sums (independent loads in flight), combined in a fixed order, then a fixed
// xor-shuffle tree across the lanes.
__device__ __forceinline__ double wave_sum_array(const double *v, int n) {
    const int lane = (int)(threadIdx.x & 63);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int j = lane;
    for (; j + 192 < n; j += 256) {
        s0 += v[j];
        s1 += v[j + 64];
        s2 += v[j + 128];
        s3 += v[j + 192];
    }
    for (; j < n; j += 64) s0 += v[j];
    double s = (s0 + s1) + (s2 + s3);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    return s;
}

__device__ __forceinline__ double mimg(double d, double L) { return d - L * floor(d / L + 0.5); }
// the same with a precomputed 1/L (hot loops)
__device__ __forceinline__ double mimg_r(double d, double L, double invL) { return d - L * floor(d * invL + 0.5); }

__device__ __forceinline__ int wrapi(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

// consecutive workgroups go round-robin over the 8 XCDs; give each XCD a contiguous range of
// logical blocks so neighbouring cells share an L2
__device__ __forceinline__ int xcd_block(int bid, int nblk) {
    const int q = nblk >> 3, r = nblk & 7, xcd = bid & 7, k = bid >> 3;
    return xcd < r ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

template <typename V>
__device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// ---- population storage.  FP64 and FP32 store the populations themselves.  The FP16 form
// stores each f_i(x) as the deviation f_i - w_i R(x) from its rest equilibrium, with the
// reference density R(x) = -rho0 log(1 - psi(x)) taken from the node's pseudopotential of the
// previous step (its density up to FP32 rounding), and does all arithmetic in FP32.  Writer and
// reader evaluate R from the same stored psi with the same instructions, so they agree to the
// bit; the deviations stay small (non-equilibrium and velocity parts), which keeps the FP16
// rounding far below that of deviations from a fixed density.  Arith<S>::T is the arithmetic
// type of storage S.
using half_t = _Float16;
template <typename S>
struct Arith {
    using T = S;
};
template <>
struct Arith<half_t> {
    using T = float;
};
template <typename S>
using ArT = typename Arith<S>::T;

// reference density of the FP16 form from a stored pseudopotential value (hardware log2)
__device__ __forceinline__ float ref_density(float psi, float rho0) {
    const float q = fmaxf(1.0f - psi, 1e-6f);
    return -0.69314718f * rho0 * __log2f(q);
}

// stored value -> population, with weight w = w_i and reference density R: the FP16 form holds
// the deviation f - w R.  Both directions are one explicit fused multiply-add (a single rounding
// of w R + v and of f - w R), so the encode does not depend on how the compiler contracts the
// surrounding arithmetic.
template <typename S>
__device__ __forceinline__ ArT<S> pop_get(S v, ArT<S> w, ArT<S> R) {
    if constexpr (sizeof(S) == 2)
        return __builtin_fmaf(w, R, (float)v);
    else
        return v;
}
// population -> stored value
template <typename S>
__device__ __forceinline__ S pop_put(ArT<S> f, ArT<S> w, ArT<S> R) {
    if constexpr (sizeof(S) == 2)
        return (S)__builtin_fmaf(-w, R, f);
    else
        return f;
}

// ---- parameters passed by value to every kernel
template <typename T>
struct Prm {
    int nx, ny, nz, nb;
    int N;           // cells
    long long Np;    // plane stride of a population / phase-field plane (N rounded up)
    T omega;         // 1 / tau
    T guo;           // 1 - 1 / (2 tau)
    T G;
    T inv_rho0;
    T rho0;          // reference density of psi (the FP16 form's reference density uses it)
    T fext[3];
    int flags;       // PF_LBM_* step flags
    double threshold, mobility, eta, r_c, n_exp, e0, R_A;
    double phi_floor; // phase values at or below it count as absent (Sec. 3.3)
    double inv_n[3]; // 1 / nx, 1 / ny, 1 / nz
    int tn[3];       // phase-field tiles per axis (ceil(n / tile edge))
    int trad[3];     // tiles searched on each side for the activity of a tile (1, or 2 where the
                     // last tile of the axis holds fewer than 3 nodes)
};

// Tiles of the phase-field work: 8 x 8 x 4 nodes in grid coordinates (the last tile of an axis
// may be partial), one block of 256 threads per tile.  Each tile keeps a state word with two bits
// per body a: bit 2a "some node of the tile has phi_a != 0", bit 2a + 1 "some node has
// phi_a != 1" (all zero: 01, all one: 10, anything else: 11).  A body is active on a tile when
// the tile or one of its neighbour tiles is mixed, or a neighbour's state differs from the
// tile's, at the start of this step or of the previous one; elsewhere every stencil of the step
// sees one constant (0 or 1) within 3 nodes, the update is the identity, and both phase buffers
// already hold that constant, so the body's work is skipped there.  Pair-form masks: bit 2a.
constexpr int TLX = 8, TLY = 8, TLZ = 4;
constexpr uint32_t PAIR_LO = 0x55555555u;

__host__ __device__ __forceinline__ uint32_t pair_mask(int nb) {
    return nb >= 16 ? PAIR_LO : (PAIR_LO & ((1u << (2 * nb)) - 1u));
}
// bit a set where pair bit 2a is set
__device__ __forceinline__ uint32_t pairs_to_bodies(uint32_t pm) {
    uint32_t out = 0;
    while (pm) {
        const int b = __ffs(pm) - 1;
        pm &= pm - 1;
        out |= 1u << (b >> 1);
    }
    return out;
}

// the tiles that meet a box [lo, hi] (unwrapped coordinates, at most one period per axis):
// per axis a run of cnt tiles starting at t0 (wrapped); tile k of the run and the nodes of a tile
template <typename T>
struct TileIter {
    int lo[3], ext[3], n[3], t0[3], cnt[3], tn[3], total;
    __device__ __forceinline__ TileIter(const int32_t *b, const Prm<T> &p) {
        n[0] = p.nx;
        n[1] = p.ny;
        n[2] = p.nz;
        const int te[3] = {TLX, TLY, TLZ};
        total = 1;
        for (int d = 0; d < 3; ++d) {
            tn[d] = p.tn[d];
            lo[d] = b[d];
            ext[d] = b[3 + d] - b[d] + 1;
            if (ext[d] <= 0) {
                total = 0;
                t0[d] = cnt[d] = 0;
                continue;
            }
            int a = lo[d] % n[d];
            a += a < 0 ? n[d] : 0;
            const int e = a + ext[d] - 1;  // last cell, unwrapped from a
            const int ta = a / te[d];
            int c = e < n[d] ? e / te[d] - ta + 1 : (tn[d] - ta) + (e - n[d]) / te[d] + 1;
            if (ext[d] >= n[d] || c >= tn[d]) {
                t0[d] = 0;
                c = tn[d];
            } else {
                t0[d] = ta;
            }
            cnt[d] = c;
            total *= c;
        }
    }
    // wrapped tile coordinates of run entry k and the tile's linear index
    __device__ __forceinline__ int tile(int k, int *tc) const {
        const int kx = k % cnt[0], r = k / cnt[0], ky = r % cnt[1], kz = r / cnt[1];
        const int kk[3] = {kx, ky, kz};
        for (int d = 0; d < 3; ++d) {
            int t = t0[d] + kk[d];
            tc[d] = t >= tn[d] ? t - tn[d] : t;
        }
        return tc[0] + tn[0] * (tc[1] + tn[1] * tc[2]);
    }
    // node j (0..255) of tile tc: wrapped (c) and unwrapped (u) coordinates; false when it lies
    // outside the grid or the box
    __device__ __forceinline__ bool node(const int *tc, int j, int *c, int *u) const {
        const int l[3] = {j & 7, (j >> 3) & 7, j >> 6};
        const int te[3] = {TLX, TLY, TLZ};
        bool ok = true;
        for (int d = 0; d < 3; ++d) {
            c[d] = tc[d] * te[d] + l[d];
            ok = ok && c[d] < n[d];
            // (c - lo) mod n: the box's lo lies within one period below or above the grid
            int m = c[d] - lo[d];
            m += m < 0 ? n[d] : 0;
            m += m < 0 ? n[d] : 0;
            m -= m >= n[d] ? n[d] : 0;
            u[d] = lo[d] + m;
            ok = ok && m < ext[d];
        }
        return ok;
    }
    // does unwrapped coordinate v on axis d lie in the box
    __device__ __forceinline__ bool inside(int d, int v) const {
        return ext[d] >= n[d] || (v >= lo[d] && v < lo[d] + ext[d]);
    }
};

// floor(k / d) for 0 <= k < 2^31, 0 < d, through a double reciprocal and one correction
__device__ __forceinline__ int fast_div(int k, int d, double inv_d) {
    int q = (int)((double)k * inv_d);
    const int r = k - q * d;
    q += (r >= d) ? 1 : 0;
    q -= (r < 0) ? 1 : 0;
    return q;
}

// iteration over the cells of a box [lo, hi] (unwrapped coordinates, hi - lo + 1 <= n per axis)
struct BoxIter {
    int lo[3], ext[3], vol, n[3];
    double inv_ex, inv_ey;
    __device__ __forceinline__ BoxIter(const int32_t *b, int nx, int ny, int nz) {
        n[0] = nx;
        n[1] = ny;
        n[2] = nz;
        for (int d = 0; d < 3; ++d) {
            lo[d] = b[d];
            ext[d] = b[3 + d] - b[d] + 1;
        }
        vol = (ext[0] > 0 && ext[1] > 0 && ext[2] > 0) ? ext[0] * ext[1] * ext[2] : 0;
        inv_ex = ext[0] > 0 ? 1.0 / ext[0] : 0.0;
        inv_ey = ext[1] > 0 ? 1.0 / ext[1] : 0.0;
    }
    // cell k -> unwrapped (u) and wrapped (c) coordinates; the box spans at most one period
    __device__ __forceinline__ void cell(int k, int *u, int *c) const {
        const int t = fast_div(k, ext[0], inv_ex);
        const int zz = fast_div(t, ext[1], inv_ey);
        u[0] = lo[0] + (k - t * ext[0]);
        u[1] = lo[1] + (t - zz * ext[1]);
        u[2] = lo[2] + zz;
        for (int d = 0; d < 3; ++d) {
            int v = u[d];
            v += v < 0 ? n[d] : 0;
            v -= v >= n[d] ? n[d] : 0;
            c[d] = v;
        }
    }
    // does unwrapped coordinate v on axis d lie in the box (always, once the box spans the axis)
    __device__ __forceinline__ bool inside(int d, int v) const {
        return ext[d] >= n[d] || (v >= lo[d] && v < lo[d] + ext[d]);
    }
};

// periodic wrap of i when it lies within one period of [0, n)
__device__ __forceinline__ int wrap1(int i, int n) {
    i += i < 0 ? n : 0;
    return i - (i >= n ? n : 0);
}

// periodic wrap of i when it lies within two periods of [0, n) (offsets of up to 2 cells on axes
// as short as one cell)
__device__ __forceinline__ int wrap2(int i, int n) {
    i += i < 0 ? n : 0;
    i += i < 0 ? n : 0;
    i -= i >= n ? n : 0;
    i -= i >= n ? n : 0;
    return i;
}

// Run by the waves of one block at the start of a step: combine the per-block reclassification
// results of the previous step in a fixed order and publish
//  * this step's box (wave 0): phase-field support + 3-cell margin, the whole axis once it would
//    wrap onto itself, lower corner brought into [0, n) (so unwrapped coordinates stay below 2 n),
//    and count the step;
//  * per body (waves 1.., round robin; wave 0 alone in a one-wave block): the solid radius
//    (bounds the repulsion search) and the volume
//    driving term h_a = (4 eta / pi^2) (V_ref - sum phi_a) / #{phi_floor < phi_a < 1} (Sec. 3.3; 0
//    without interface nodes), into the body table;
// and clear the event count for this step's reclassification.  Each lane sums its parts with four
// independent accumulators, then a fixed xor-shuffle tree combines the lanes.
__device__ __forceinline__ void publish_step_state(int wave, int nwaves, int parity, int nx, int ny, int nz, int nb,
                                                   double eta, StepState *st, BodyDev *bodies,
                                                   const ClassifyPart *cpart, int nblk) {
    const int lane = (int)(threadIdx.x & 63);
    if (wave == 0) {
        int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
        for (int j = lane; j < nblk; j += 64)
            for (int d = 0; d < 3; ++d) {
                lo[d] = min(lo[d], cpart[j].lo[d]);
                hi[d] = max(hi[d], cpart[j].hi[d]);
            }
        for (int d = 0; d < 3; ++d) {
            lo[d] = wave_min(lo[d]);
            hi[d] = wave_max(hi[d]);
        }
        if (lane == 0) {
            const int n[3] = {nx, ny, nz};
            const bool empty = lo[0] > hi[0] || lo[1] > hi[1] || lo[2] > hi[2];
            for (int d = 0; d < 3; ++d) {
                int l = lo[d] - 3, h = hi[d] + 3;
                if (h - l + 1 >= n[d]) {
                    l = 0;
                    h = n[d] - 1;
                } else {
                    const int s = wrap2(l, n[d]) - l;
                    l += s;
                    h += s;
                }
                st->box[parity][d] = empty ? 0 : l;
                st->box[parity][3 + d] = empty ? -1 : h;
            }
            st->n_events = 0u;
            st->step_no += 1u;
        }
        if (nwaves > 1) return;
    }
    const double PI = 3.14159265358979323846;
    // bodies on waves 1.. (round robin), or on wave 0 when the block has a single wave
    const int bw = nwaves > 1 ? wave - 1 : 0, bstride = nwaves > 1 ? nwaves - 1 : 1;
    for (int b = bw; b < nb; b += bstride) {
        float r0 = 0.0f, r1 = 0.0f, r2 = 0.0f, r3 = 0.0f;
        double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
        int c0 = 0, c1 = 0, c2 = 0, c3 = 0;
        int j = lane;
        for (; j + 192 < nblk; j += 256) {
            r0 = fmaxf(r0, cpart[j].srad[b]);
            r1 = fmaxf(r1, cpart[j + 64].srad[b]);
            r2 = fmaxf(r2, cpart[j + 128].srad[b]);
            r3 = fmaxf(r3, cpart[j + 192].srad[b]);
            v0 += cpart[j].vol[b];
            v1 += cpart[j + 64].vol[b];
            v2 += cpart[j + 128].vol[b];
            v3 += cpart[j + 192].vol[b];
            c0 += (int)cpart[j].icnt[b];
            c1 += (int)cpart[j + 64].icnt[b];
            c2 += (int)cpart[j + 128].icnt[b];
            c3 += (int)cpart[j + 192].icnt[b];
        }
        for (; j < nblk; j += 64) {
            r0 = fmaxf(r0, cpart[j].srad[b]);
            v0 += cpart[j].vol[b];
            c0 += (int)cpart[j].icnt[b];
        }
        float r = fmaxf(fmaxf(r0, r1), fmaxf(r2, r3));
        double v = (v0 + v1) + (v2 + v3);
        int c = (c0 + c1) + (c2 + c3);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) r = fmaxf(r, __shfl_xor(r, off, 64));
        v = wave_sum(v);
        c = wave_sum(c);
        if (lane == 0) {
            st->srad[b] = r;
            bodies[b].h = c > 0 ? (4.0 * eta / (PI * PI)) * (bodies[b].Vref - v) / (double)c : 0.0;
        }
    }
}

}  // namespace pfl
