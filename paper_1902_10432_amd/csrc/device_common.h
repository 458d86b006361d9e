// Device-side building blocks of the coupled phase-field / lattice-Boltzmann step for gfx950:
// the D3Q19 velocity set as compile-time constants, the mask byte layout, the body table and
// the per-step state shared by the kernels, wave64 reductions and the XCD-aware block order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace pfl {

// ---- D3Q19 (Sec. 3.2.1 prints D3Q27; both share c_s^2 = 1/3 and the second and fourth
// moments).  Direction pairs (2k-1, 2k) are opposite.  Rest, 6 faces, 12 edges.
constexpr int kCX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

template <int I>
struct Dir {
    static constexpr int x = kCX[I], y = kCY[I], z = kCZ[I];
    static constexpr int opp = I == 0 ? 0 : ((I & 1) ? I + 1 : I - 1);
    static constexpr int c2 = x * x + y * y + z * z;
    template <typename T>
    __device__ static constexpr T w() {
        return c2 == 0 ? T(1.0 / 3.0) : (c2 == 1 ? T(1.0 / 18.0) : T(1.0 / 36.0));
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

// ---- mask byte: bit 7 solid, bit 6 became solid this step, bit 5 became fluid this step,
// bits 0-4 owning body of a solid node
constexpr uint8_t M_SOLID = 0x80, M_F2S = 0x40, M_S2F = 0x20, M_OWNER = 0x1f;

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
    int32_t box[2][6];           // lo x, lo y, lo z, hi x, hi y, hi z
    int32_t tight[6];            // atomic min / max accumulators of the phase-field support
    uint32_t done[4];            // last-block counters: 0 forces, 1 volume sums, 2 box
    uint32_t err;                // bit 0 non-finite body state, bit 1 advection CFL above 1
    uint32_t pad;
    unsigned long long n_f2s, n_s2f, n_lost;
};

__device__ __forceinline__ double mimg(double d, double L) { return d - L * floor(d / L + 0.5); }

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
    T fext[3];
    int flags;       // PF_LBM_* step flags
    double threshold, mobility, eta, r_c, n_exp, e0, R_A;
};

// box cell k (0 <= k < box volume) -> unwrapped coordinates
__device__ __forceinline__ void box_cell(const int32_t *b, long long k, int &ux, int &uy, int &uz) {
    const int ex = b[3] - b[0] + 1, ey = b[4] - b[1] + 1;
    ux = b[0] + (int)(k % ex);
    long long t = k / ex;
    uy = b[1] + (int)(t % ey);
    uz = b[2] + (int)(t / ey);
}
__device__ __forceinline__ long long box_volume(const int32_t *b) {
    if (b[3] < b[0] || b[4] < b[1] || b[5] < b[2]) return 0;
    return (long long)(b[3] - b[0] + 1) * (b[4] - b[1] + 1) * (b[5] - b[2] + 1);
}

}  // namespace pfl
