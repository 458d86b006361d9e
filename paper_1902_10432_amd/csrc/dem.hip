// Many-sphere rigid-body run with pairwise capillary-bridge forces from the learned surrogate.
// See include/pf_dem.h for the model; the kernels here are
//   k_dem_neighbours  one wave per sphere: bridged partners in ascending index order (ballot
//                     compaction), their count and the count of partners with a larger index;
//   k_dem_rows        one block: exclusive scan of the upper counts (one network row per
//                     bridge i < j, ordered by (i, j)), bridge features and network inputs;
//   k_dem_forces      one thread per sphere: bridge and contact forces summed in partner order;
//   k_dem_integrate   one thread per sphere: semi-implicit Euler and periodic wrap.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pf_dem.h"

// the network's stream, input width and batch limit (mlp.hip)
__attribute__((visibility("hidden"))) void pfm_internal_info(const pf_mlp *h, int *n_in, int *max_batch,
                                                             void **stream);

namespace pfd {

constexpr int MAX_OVERRIDES = 256;
constexpr double PI = 3.14159265358979323846;

struct DemDev {
    int n, cap, max_pairs, n_over;
    double L, dt, density, kn, gn, theta, cfrac, gmin, gmax;
    float ish[4], isc[4], osh, osc;
    const double *R;
    double *x, *v, *F;
    int *nbr, *deg, *nup, *off;
    int *pij;
    double *pfeat, *pforce;
    float *X;
    const float *Y;
    int *ctl;  // [0] bridges, [1] error bits (1: neighbours, 2: pairs)
    const int *over_ij;
    const double *over_f;
};

// minimum image; x_j - x_i and x_i - x_j give exactly negated results, and the surface gap is
// formed as r - (R_i + R_j), so "bridged" is symmetric in (i, j) to the bit
__device__ __forceinline__ double mimg(double d, double L) { return d - L * floor(d / L + 0.5); }

__global__ __launch_bounds__(256) void k_dem_neighbours(DemDev p) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= p.n) return;  // whole wave
    const double xi = p.x[3 * i], yi = p.x[3 * i + 1], zi = p.x[3 * i + 2], Ri = p.R[i];
    int cnt = 0, up = 0;
    for (int base = 0; base < p.n; base += 64) {
        const int j = base + lane;
        bool b = false;
        if (j < p.n && j != i) {
            const double dx = mimg(p.x[3 * j] - xi, p.L), dy = mimg(p.x[3 * j + 1] - yi, p.L),
                         dz = mimg(p.x[3 * j + 2] - zi, p.L);
            const double gap = sqrt(dx * dx + dy * dy + dz * dz) - (Ri + p.R[j]);
            b = gap < p.gmax;
        }
        const unsigned long long m = __ballot(b);
        const int rank = __popcll(m & ((1ull << lane) - 1ull));
        if (b && cnt + rank < p.cap) p.nbr[(long long)i * p.cap + cnt + rank] = j;
        cnt += __popcll(m);
        up += __popcll(__ballot(b && j > i));
    }
    if (lane == 0) {
        p.deg[i] = min(cnt, p.cap);
        p.nup[i] = up;
        if (cnt > p.cap) atomicOr(p.ctl + 1, 1);
    }
}

__device__ __forceinline__ void bridge_features(const DemDev &p, double Ri, double Rj, double gap, double *f,
                                                double *rstar) {
    const double rs = 2.0 * Ri * Rj / (Ri + Rj);
    const double vl = p.cfrac / (1.0 - p.cfrac) * (4.0 / 3.0) * PI * (Ri * Ri * Ri + Rj * Rj * Rj);
    f[0] = fmax(gap, p.gmin) / rs;
    f[1] = fmin(Ri, Rj) / fmax(Ri, Rj);
    f[2] = vl / (rs * rs * rs);
    f[3] = p.theta;
    *rstar = rs;
}

// one block of 1024 threads; thread t owns spheres [t * per, (t + 1) * per)
__global__ __launch_bounds__(1024) void k_dem_rows(DemDev p) {
    __shared__ int part[1024];
    const int t = threadIdx.x;
    const int per = (p.n + 1023) / 1024;
    const int i0 = min(t * per, p.n), i1 = min(i0 + per, p.n);
    int s = 0;
    for (int i = i0; i < i1; ++i) s += p.nup[i];
    part[t] = s;
    __syncthreads();
    // inclusive Hillis-Steele scan of the per-thread sums
    for (int d = 1; d < 1024; d <<= 1) {
        const int a = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += a;
        __syncthreads();
    }
    int o = part[t] - s;
    if (t == 1023) {
        p.ctl[0] = part[1023];
        if (part[1023] > p.max_pairs) atomicOr(p.ctl + 1, 2);
    }
    for (int i = i0; i < i1; ++i) {
        p.off[i] = o;
        const double xi = p.x[3 * i], yi = p.x[3 * i + 1], zi = p.x[3 * i + 2], Ri = p.R[i];
        int row = o;
        for (int k = 0; k < p.deg[i]; ++k) {
            const int j = p.nbr[(long long)i * p.cap + k];
            if (j < i) continue;
            if (row < p.max_pairs) {
                const double dx = mimg(p.x[3 * j] - xi, p.L), dy = mimg(p.x[3 * j + 1] - yi, p.L),
                             dz = mimg(p.x[3 * j + 2] - zi, p.L);
                const double gap = sqrt(dx * dx + dy * dy + dz * dz) - (Ri + p.R[j]);
                double f[4], rs;
                bridge_features(p, Ri, p.R[j], gap, f, &rs);
                p.pij[2 * row] = i;
                p.pij[2 * row + 1] = j;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    p.pfeat[4 * (long long)row + c] = f[c];
                    p.X[4 * (long long)row + c] = (float)((f[c] - (double)p.ish[c]) * (double)p.isc[c]);
                }
            }
            ++row;
        }
        o += p.nup[i];
    }
}

__global__ __launch_bounds__(256) void k_dem_forces(DemDev p) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= p.n) return;
    const double xi = p.x[3 * i], yi = p.x[3 * i + 1], zi = p.x[3 * i + 2], Ri = p.R[i];
    const double vxi = p.v[3 * i], vyi = p.v[3 * i + 1], vzi = p.v[3 * i + 2];
    const int di = p.deg[i], lower_i = di - p.nup[i];
    double Fx = 0.0, Fy = 0.0, Fz = 0.0;
    for (int k = 0; k < di; ++k) {
        const int j = p.nbr[(long long)i * p.cap + k];
        const double dx = mimg(p.x[3 * j] - xi, p.L), dy = mimg(p.x[3 * j + 1] - yi, p.L),
                     dz = mimg(p.x[3 * j + 2] - zi, p.L);
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        const double Rj = p.R[j], gap = r - (Ri + Rj);
        const double ex = dx / r, ey = dy / r, ez = dz / r;
        // network row of the bridge (min(i, j), max(i, j))
        int row;
        if (j > i) {
            row = p.off[i] + (k - lower_i);
        } else {
            const int dj = p.deg[j];
            int pos = 0;
            while (pos < dj && p.nbr[(long long)j * p.cap + pos] != i) ++pos;
            if (pos == dj) continue;  // unreachable: the gap is symmetric in (i, j) to the bit
            row = p.off[j] + (pos - (dj - p.nup[j]));
        }
        const double rs = 2.0 * Ri * Rj / (Ri + Rj);
        double Fb = ((double)p.Y[row] * (double)p.osc + (double)p.osh) * rs;
        const int a = min(i, j), b = max(i, j);
        for (int q = 0; q < p.n_over; ++q)
            if (p.over_ij[2 * q] == a && p.over_ij[2 * q + 1] == b) Fb = p.over_f[q];
        if (j > i) p.pforce[row] = Fb;
        double fn = Fb;  // along e (towards j)
        if (gap < 0.0) {
            const double vn = (p.v[3 * j] - vxi) * ex + (p.v[3 * j + 1] - vyi) * ey + (p.v[3 * j + 2] - vzi) * ez;
            fn += p.kn * gap + p.gn * vn;
        }
        Fx += fn * ex;
        Fy += fn * ey;
        Fz += fn * ez;
    }
    p.F[3 * i] = Fx;
    p.F[3 * i + 1] = Fy;
    p.F[3 * i + 2] = Fz;
}

__global__ __launch_bounds__(256) void k_dem_integrate(DemDev p) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= p.n) return;
    const double R = p.R[i];
    const double inv_m = 1.0 / (p.density * (4.0 / 3.0) * PI * R * R * R);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double v = p.v[3 * i + c] + p.F[3 * i + c] * inv_m * p.dt;
        double x = p.x[3 * i + c] + v * p.dt;
        x -= p.L * floor(x / p.L);
        if (x >= p.L) x -= p.L;  // x / L rounded up to 1
        p.v[3 * i + c] = v;
        p.x[3 * i + c] = x;
    }
}

}  // namespace pfd

using namespace pfd;

struct pf_dem {
    pf_dem_config cfg;
    hipStream_t stream = nullptr;
    pf_mlp *net = nullptr;
    char *ws = nullptr;
    DemDev d{};
    int *ctl_host = nullptr;  // pinned, 2 ints
    int last_pairs = 0;
    std::string err;
};

namespace {

thread_local std::string g_dem_init_error;

int dfail(pf_dem *h, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h)
        h->err = buf;
    else
        g_dem_init_error = buf;
    return code;
}

#define DCHK(h, call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return dfail((h), PF_LBM_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

int blocks(int n, int per) { return (n + per - 1) / per; }

}  // namespace

extern "C" {

int pf_dem_init(const pf_dem_config *cfg, const double *radii, const double *x0, const double *v0, pf_mlp *net,
                void *workspace, size_t ws_bytes, void *hip_stream, pf_dem **out, size_t *ws_bytes_needed) {
    g_dem_init_error.clear();
    if (!cfg) return dfail(nullptr, PF_LBM_EINVAL, "cfg is NULL");
    if (cfg->struct_size < sizeof(pf_dem_config)) return dfail(nullptr, PF_LBM_EINVAL, "bad struct_size");
    if (cfg->n < 2 || cfg->n > 16384) return dfail(nullptr, PF_LBM_EINVAL, "n must be in [2, 16384]");
    if (cfg->max_neighbours < 1 || cfg->max_neighbours > 64)
        return dfail(nullptr, PF_LBM_EINVAL, "max_neighbours must be in [1, 64]");
    if (cfg->max_pairs < 1 || cfg->max_pairs > 65536) return dfail(nullptr, PF_LBM_EINVAL, "max_pairs in [1, 65536]");
    if (!(cfg->dt > 0) || !(cfg->density > 0) || !(cfg->k_n >= 0) || !(cfg->gamma_n >= 0))
        return dfail(nullptr, PF_LBM_EINVAL, "dt and density must be positive, k_n and gamma_n non-negative");
    if (!(cfg->theta >= 0 && cfg->theta <= 0.5 * PI)) return dfail(nullptr, PF_LBM_EINVAL, "theta must be in [0, pi/2]");
    if (!(cfg->liquid_fraction > 0 && cfg->liquid_fraction < 1))
        return dfail(nullptr, PF_LBM_EINVAL, "liquid_fraction must be in (0, 1)");
    if (!(cfg->gap_min >= 0 && cfg->gap_max > cfg->gap_min)) return dfail(nullptr, PF_LBM_EINVAL, "need 0 <= gap_min < gap_max");
    const int n = cfg->n, cap = cfg->max_neighbours, P = cfg->max_pairs;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) / 256 * 256;
        return o;
    };
    const size_t oR = take(8 * (size_t)n), ox = take(24 * (size_t)n), ov = take(24 * (size_t)n),
                 oF = take(24 * (size_t)n), onbr = take(4 * (size_t)n * cap), odeg = take(4 * (size_t)n),
                 onup = take(4 * (size_t)n), ooff = take(4 * (size_t)n), opij = take(8 * (size_t)P),
                 opfeat = take(32 * (size_t)P), opforce = take(8 * (size_t)P), oX = take(16 * (size_t)P),
                 oY = take(4 * (size_t)P), octl = take(16), oover = take(8 * MAX_OVERRIDES),
                 overf = take(8 * MAX_OVERRIDES);
    if (ws_bytes_needed) *ws_bytes_needed = off;
    if (!workspace) return PF_LBM_OK;
    if (!out || !radii || !x0 || !v0 || !net) return dfail(nullptr, PF_LBM_EINVAL, "NULL argument");
    if (ws_bytes < off) return dfail(nullptr, PF_LBM_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, off);
    if ((uintptr_t)workspace % 256) return dfail(nullptr, PF_LBM_EINVAL, "workspace must be 256-byte aligned");
    int n_in = 0, max_batch = 0;
    void *net_stream = nullptr;
    pfm_internal_info(net, &n_in, &max_batch, &net_stream);
    if (n_in != 4) return dfail(nullptr, PF_LBM_EINVAL, "the network must take 4 inputs (it takes %d)", n_in);
    if (max_batch < P) return dfail(nullptr, PF_LBM_EINVAL, "network max_batch %d below max_pairs %d", max_batch, P);
    if (net_stream != hip_stream) return dfail(nullptr, PF_LBM_EINVAL, "the network is bound to another stream");
    double rmax = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!(radii[i] > 0)) return dfail(nullptr, PF_LBM_EINVAL, "radius %d is not positive", i);
        rmax = std::max(rmax, radii[i]);
        for (int c = 0; c < 3; ++c)
            if (!(x0[3 * i + c] >= 0 && x0[3 * i + c] < cfg->box) || !std::isfinite(v0[3 * i + c]))
                return dfail(nullptr, PF_LBM_EINVAL, "sphere %d: position outside [0, box) or velocity not finite", i);
    }
    if (!(cfg->box > 4.0 * rmax + 2.0 * cfg->gap_max))
        return dfail(nullptr, PF_LBM_EINVAL, "box must exceed 4 max radius + 2 gap_max (unique minimum image)");
    pf_dem *h = new (std::nothrow) pf_dem;
    if (!h) return dfail(nullptr, PF_LBM_ENOMEM, "host allocation failed");
    h->cfg = *cfg;
    h->stream = (hipStream_t)hip_stream;
    h->net = net;
    h->ws = (char *)workspace;
    DemDev &d = h->d;
    d.n = n;
    d.cap = cap;
    d.max_pairs = P;
    d.n_over = 0;
    d.L = cfg->box;
    d.dt = cfg->dt;
    d.density = cfg->density;
    d.kn = cfg->k_n;
    d.gn = cfg->gamma_n;
    d.theta = cfg->theta;
    d.cfrac = cfg->liquid_fraction;
    d.gmin = cfg->gap_min;
    d.gmax = cfg->gap_max;
    for (int c = 0; c < 4; ++c) {
        d.ish[c] = cfg->in_shift[c];
        d.isc[c] = cfg->in_scale[c];
    }
    d.osh = cfg->out_shift;
    d.osc = cfg->out_scale;
    char *w = h->ws;
    d.R = (const double *)(w + oR);
    d.x = (double *)(w + ox);
    d.v = (double *)(w + ov);
    d.F = (double *)(w + oF);
    d.nbr = (int *)(w + onbr);
    d.deg = (int *)(w + odeg);
    d.nup = (int *)(w + onup);
    d.off = (int *)(w + ooff);
    d.pij = (int *)(w + opij);
    d.pfeat = (double *)(w + opfeat);
    d.pforce = (double *)(w + opforce);
    d.X = (float *)(w + oX);
    d.Y = (const float *)(w + oY);
    d.ctl = (int *)(w + octl);
    d.over_ij = (const int *)(w + oover);
    d.over_f = (const double *)(w + overf);
    auto fail_init = [&](int rc) {
        g_dem_init_error = h->err;
        if (h->ctl_host) (void)hipHostFree(h->ctl_host);
        delete h;
        return rc;
    };
    if (hipHostMalloc((void **)&h->ctl_host, 16, hipHostMallocDefault) != hipSuccess) {
        h->ctl_host = nullptr;
        return fail_init(dfail(h, PF_LBM_EDEVICE, "hipHostMalloc failed"));
    }
    if (hipMemsetAsync(h->ws, 0, off, h->stream) != hipSuccess ||
        hipMemcpyAsync((void *)d.R, radii, 8 * (size_t)n, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(d.x, x0, 24 * (size_t)n, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(d.v, v0, 24 * (size_t)n, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return fail_init(dfail(h, PF_LBM_EDEVICE, "upload failed"));
    *out = h;
    return PF_LBM_OK;
}

int pf_dem_evaluate(pf_dem *h) {
    if (!h) return dfail(nullptr, PF_LBM_EINVAL, "handle is NULL");
    DemDev &d = h->d;
    DCHK(h, hipMemsetAsync(d.ctl, 0, 16, h->stream));
    k_dem_neighbours<<<blocks(d.n, 4), 256, 0, h->stream>>>(d);
    k_dem_rows<<<1, 1024, 0, h->stream>>>(d);
    DCHK(h, hipGetLastError());
    DCHK(h, hipMemcpyAsync(h->ctl_host, d.ctl, 8, hipMemcpyDeviceToHost, h->stream));
    DCHK(h, hipStreamSynchronize(h->stream));
    if (h->ctl_host[1] & 1) return dfail(h, PF_LBM_ENOMEM, "a sphere has more than max_neighbours bridged partners");
    if (h->ctl_host[1] & 2)
        return dfail(h, PF_LBM_ENOMEM, "%d bridges exceed max_pairs %d", h->ctl_host[0], d.max_pairs);
    const int P = h->ctl_host[0];
    if (P > 0) {
        const int rc = pf_mlp_forward(h->net, d.X, P, (float *)d.Y);
        if (rc != PF_LBM_OK) return dfail(h, rc, "network: %s", pf_mlp_last_error(h->net));
    }
    k_dem_forces<<<blocks(d.n, 256), 256, 0, h->stream>>>(d);
    DCHK(h, hipGetLastError());
    h->last_pairs = P;
    return PF_LBM_OK;
}

int pf_dem_step(pf_dem *h, int32_t n_steps) {
    if (!h) return dfail(nullptr, PF_LBM_EINVAL, "handle is NULL");
    if (n_steps < 0) return dfail(h, PF_LBM_EINVAL, "n_steps must be >= 0");
    for (int s = 0; s < n_steps; ++s) {
        const int rc = pf_dem_evaluate(h);
        if (rc != PF_LBM_OK) return rc;
        k_dem_integrate<<<blocks(h->d.n, 256), 256, 0, h->stream>>>(h->d);
        DCHK(h, hipGetLastError());
    }
    return PF_LBM_OK;
}

int pf_dem_state(pf_dem *h, double *x, double *v, double *f) {
    if (!h) return dfail(nullptr, PF_LBM_EINVAL, "handle is NULL");
    const size_t b = 24 * (size_t)h->d.n;
    if (x) DCHK(h, hipMemcpyAsync(x, h->d.x, b, hipMemcpyDeviceToHost, h->stream));
    if (v) DCHK(h, hipMemcpyAsync(v, h->d.v, b, hipMemcpyDeviceToHost, h->stream));
    if (f) DCHK(h, hipMemcpyAsync(f, h->d.F, b, hipMemcpyDeviceToHost, h->stream));
    DCHK(h, hipStreamSynchronize(h->stream));
    return PF_LBM_OK;
}

int pf_dem_pairs(pf_dem *h, int32_t max_out, int32_t *ij, double *features, double *force, int32_t *n_out) {
    if (!h || !n_out) return dfail(h, PF_LBM_EINVAL, "NULL argument");
    if (max_out < 0) return dfail(h, PF_LBM_EINVAL, "max_out must be >= 0");
    const int k = std::min(max_out, h->last_pairs);
    *n_out = h->last_pairs;
    if (k > 0) {
        if (ij) DCHK(h, hipMemcpyAsync(ij, h->d.pij, 8 * (size_t)k, hipMemcpyDeviceToHost, h->stream));
        if (features) DCHK(h, hipMemcpyAsync(features, h->d.pfeat, 32 * (size_t)k, hipMemcpyDeviceToHost, h->stream));
        if (force) DCHK(h, hipMemcpyAsync(force, h->d.pforce, 8 * (size_t)k, hipMemcpyDeviceToHost, h->stream));
    }
    DCHK(h, hipStreamSynchronize(h->stream));
    return PF_LBM_OK;
}

int pf_dem_set_overrides(pf_dem *h, int32_t n, const int32_t *ij, const double *force) {
    if (!h) return dfail(nullptr, PF_LBM_EINVAL, "handle is NULL");
    if (n < 0 || n > MAX_OVERRIDES) return dfail(h, PF_LBM_EINVAL, "n must be in [0, %d]", MAX_OVERRIDES);
    if (n > 0 && (!ij || !force)) return dfail(h, PF_LBM_EINVAL, "NULL argument");
    std::vector<int> pairs(2 * (size_t)n);
    for (int k = 0; k < n; ++k) {
        const int a = ij[2 * k], b = ij[2 * k + 1];
        if (a < 0 || b < 0 || a >= h->d.n || b >= h->d.n || a == b || !std::isfinite(force[k]))
            return dfail(h, PF_LBM_EINVAL, "override %d: bad pair or force", k);
        pairs[2 * k] = std::min(a, b);
        pairs[2 * k + 1] = std::max(a, b);
    }
    if (n > 0) {
        DCHK(h, hipMemcpyAsync((void *)h->d.over_ij, pairs.data(), 8 * (size_t)n, hipMemcpyHostToDevice, h->stream));
        DCHK(h, hipMemcpyAsync((void *)h->d.over_f, force, 8 * (size_t)n, hipMemcpyHostToDevice, h->stream));
    }
    DCHK(h, hipStreamSynchronize(h->stream));
    h->d.n_over = n;
    return PF_LBM_OK;
}

void pf_dem_destroy(pf_dem *h) {
    if (!h) return;
    if (h->ctl_host) (void)hipHostFree(h->ctl_host);
    delete h;
}

const char *pf_dem_last_error(const pf_dem *h) { return h ? h->err.c_str() : g_dem_init_error.c_str(); }

}  // extern "C"
