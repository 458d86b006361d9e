// C-ABI of the MI355X coupled multi-phase-field / lattice-Boltzmann step: workspace layout,
// host-side body moments, the per-step launch sequence and read-out.  See include/pf_lbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pf_lbm.h"
#include "kernels_lbm.h"
#include "kernels_pf.h"

using namespace pfl;

namespace {

thread_local std::string g_init_error;

constexpr size_t ALIGN = 256;
// capacity of the per-step list of nodes that changed side (beyond it the closing kernels scan
// the whole box)
constexpr uint32_t EV_CAP = 1u << 16;
// steps of per-body force / torque history kept on the device (ring)
constexpr int HIST_CAP = 8192;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }
// largest grid of the force scan (per-block partials of every body)
constexpr int FORCE_GRID_MAX = 256;
// per-block FP64 force / torque partials of one step: FORCE_GRID_MAX blocks x PF_LBM_MAX_BODIES
// bodies x 6 components (192 KiB)
constexpr size_t STATIC_PARTS = (size_t)FORCE_GRID_MAX * PF_LBM_MAX_BODIES * 6;
constexpr int MAX_DEVICES = 64;

struct Layout {
    size_t fA, fB, psi, psiB, phiA, phiB, mask, nbw, bodies, state, sigma, pforce, cpart, evlist, hist, tstate, thot,
        tact, total;
};

}  // namespace

// Force partials of pf_lbm_step_noalloc: one copy per GPU (each device holds its own instance of
// the array), shared by every such call on that GPU.  Host code never uses this name as an
// address: the device address comes from hipGetSymbolAddress (static_parts below).
static __device__ __align__(256) double scratch[STATIC_PARTS];

struct pf_lbm {
    pf_lbm_config cfg;
    int nb = 0;
    int prec = PF_LBM_FP32;
    int q = 19;  // velocities of the lattice (D3Q19 or D3Q27)
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    Layout L{};
    long long N = 0, Np = 0;
    int dense_blocks = 0, box_blocks = 1;
    int box_grid = 1, force_grid = 1;  // grids of the box kernels and of the force scan
    int cgrid = 1;  // classification partials written per step (grid of the phase update)
    // tile shape of the fluid pass, which leaves the arithmetic unchanged (pf_lbm_autotune): rows
    // of the 64-wide tile (block of 64 x fluid_ty threads) and planes per z-chunk
    int fluid_ty = 8, fluid_tz = 32;
    // entries of the per-step event list in use (at most EV_CAP; fewer only to exercise the
    // box-scan path that an overflowing list takes)
    uint32_t ev_cap = EV_CAP;
    // launch-shape generation: raised whenever captured graphs of the handle become stale, so a
    // batch graph that holds its steps recaptures too
    unsigned gen = 0;
    long long steps = 0;
    std::vector<double> sigma;
    std::string err;
    // measurement events (pf_lbm_timing)
    bool timing = false;
    int timed = 0;
    std::vector<hipEvent_t> ev;  // 4 per timed step: step start, kernel start, kernel end, step end
    // two steps (even, odd parity) captured once and replayed
    // captured step sequences of GRAPH_STEPS[k] steps (k = 0: a pair, 1: a longer run that
    // spreads the launch gap between replays over more steps)
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    bool graph_failed = false;
};

namespace {

int fail(pf_lbm *h, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h)
        h->err = buf;
    else
        g_init_error = buf;
    return code;
}

#define HIPCHK(h, call)                                                                           \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) return fail((h), PF_LBM_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// bytes per stored population and per arithmetic value (pseudopotential) of a precision form
size_t pop_size(int prec) { return prec == PF_LBM_FP64 ? 8 : (prec == PF_LBM_FP16_STORE ? 2 : 4); }
size_t real_size(int prec) { return prec == PF_LBM_FP64 ? 8 : 4; }

Layout make_layout(long long Np, int nb, int prec, int q, int cpart_n, int force_grid, long long ntiles) {
    const size_t rs = real_size(prec), ps = pop_size(prec);
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.fA = take((size_t)q * Np * ps);
    L.fB = take((size_t)q * Np * ps);
    // pseudopotential of this step and of the previous one (by step parity)
    L.psi = take((size_t)Np * rs);
    L.psiB = take((size_t)Np * rs);
    // phase fields are FP64 in every form: the advection increments of slow, heavy bodies lie
    // far below the FP32 resolution of phi
    L.phiA = take((size_t)std::max(nb, 1) * Np * sizeof(double));
    L.phiB = take((size_t)std::max(nb, 1) * Np * sizeof(double));
    L.mask = take((size_t)Np * sizeof(cell_t));
    // D3Q27: one word of solid-neighbour bits per node (D3Q19 keeps them in the cell word)
    L.nbw = q == 27 ? take((size_t)Np * sizeof(uint32_t)) : 0;
    L.bodies = take(2 * sizeof(BodyDev) * std::max(nb, 1));  // current / next, by step parity
    L.state = take(sizeof(StepState));
    L.sigma = take(sizeof(double) * (nb + 1) * (nb + 1));
    L.pforce = take(sizeof(double) * force_grid * std::max(nb, 1) * 6);
    L.cpart = take(sizeof(ClassifyPart) * cpart_n);
    L.evlist = take(sizeof(uint32_t) * EV_CAP);
    L.hist = take(sizeof(double) * HIST_CAP * std::max(nb, 1) * 6);
    // phase-field tiles: state word, hot masks of this and the previous step, active masks
    L.tstate = take(sizeof(uint32_t) * 4 * ntiles);  // one word per z-layer of the tile
    L.thot = take(sizeof(uint32_t) * 2 * ntiles);
    L.tact = take(sizeof(uint32_t) * ntiles);
    L.total = off;
    return L;
}

double mimg_h(double d, double L) { return d - L * std::floor(d / L + 0.5); }

// Support of a set of fields along one axis: occupied planes; the support is taken as the
// contiguous run that starts right after the longest cyclic run of empty planes (first one on
// ties).  Returns false when every plane is occupied.
bool axis_gap(const std::vector<char> &occ, int &start, int &extent) {
    const int L = (int)occ.size();
    int best_len = 0, best_end = -1;
    for (int k0 = 0; k0 < L; ++k0) {
        if (occ[k0] || !occ[(k0 - 1 + L) % L]) continue;
        int len = 0;
        while (len < L && !occ[(k0 + len) % L]) ++len;
        if (len > best_len) {
            best_len = len;
            best_end = (k0 + len - 1) % L;
        }
    }
    if (best_len == 0) return false;
    start = (best_end + 1) % L;
    extent = L - best_len;
    return true;
}

struct HostBody {
    double M, Iinv[9], X[3], Vref;
};

// mass, centre (phi-weighted centroid in unwrapped coordinates; an axis without an empty plane
// uses the circular mean), inertia tensor about the centre with minimum-image lever arms, and
// the reference volume sum(phi), from the phase field at t = 0 (Sec. 3.1.1, 3.3)
HostBody body_moments(const double *phi, int nx, int ny, int nz, double rho_s) {
    const int n[3] = {nx, ny, nz};
    HostBody hb{};
    std::vector<char> occ[3] = {std::vector<char>(nx, 0), std::vector<char>(ny, 0), std::vector<char>(nz, 0)};
    double sc[3] = {0, 0, 0}, ss[3] = {0, 0, 0};
    const double PI = 3.14159265358979323846;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const double p = phi[x + (long long)nx * (y + (long long)ny * z)];
                if (p == 0.0) continue;
                const int c[3] = {x, y, z};
                for (int d = 0; d < 3; ++d) {
                    occ[d][c[d]] = 1;
                    sc[d] += p * std::cos(2.0 * PI * c[d] / n[d]);
                    ss[d] += p * std::sin(2.0 * PI * c[d] / n[d]);
                }
            }
    int start[3] = {0, 0, 0}, ext[3];
    bool gap[3];
    double c0[3];
    for (int d = 0; d < 3; ++d) {
        gap[d] = axis_gap(occ[d], start[d], ext[d]);
        double a = std::atan2(ss[d], sc[d]);
        if (a < 0) a += 2.0 * PI;
        c0[d] = a * n[d] / (2.0 * PI);
    }
    auto unwrap = [&](int d, int k) {
        return gap[d] ? (double)start[d] + (double)(((k - start[d]) % n[d] + n[d]) % n[d]) : c0[d] + mimg_h(k - c0[d], n[d]);
    };
    double vol = 0.0, m1[3] = {0, 0, 0};
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const double p = phi[x + (long long)nx * (y + (long long)ny * z)];
                if (p == 0.0) continue;
                vol += p;
                m1[0] += p * unwrap(0, x);
                m1[1] += p * unwrap(1, y);
                m1[2] += p * unwrap(2, z);
            }
    hb.Vref = vol;
    hb.M = rho_s * vol;
    for (int d = 0; d < 3; ++d) {
        double X = vol > 0 ? m1[d] / vol : 0.0;
        X -= n[d] * std::floor(X / n[d]);
        hb.X[d] = X;
    }
    double I[9] = {0};
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const double p = phi[x + (long long)nx * (y + (long long)ny * z)];
                if (p == 0.0) continue;
                const double r[3] = {mimg_h(x - hb.X[0], nx), mimg_h(y - hb.X[1], ny), mimg_h(z - hb.X[2], nz)};
                const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) I[3 * i + j] += rho_s * p * ((i == j ? r2 : 0.0) - r[i] * r[j]);
            }
    // inverse by the adjugate; a degenerate tensor gets a zero inverse (no rotation)
    double adj[9] = {I[4] * I[8] - I[5] * I[7], I[2] * I[7] - I[1] * I[8], I[1] * I[5] - I[2] * I[4],
                     I[5] * I[6] - I[3] * I[8], I[0] * I[8] - I[2] * I[6], I[2] * I[3] - I[0] * I[5],
                     I[3] * I[7] - I[4] * I[6], I[1] * I[6] - I[0] * I[7], I[0] * I[4] - I[1] * I[3]};
    const double det = I[0] * adj[0] + I[1] * adj[3] + I[2] * adj[6];
    const double scale = std::fabs(I[0]) + std::fabs(I[4]) + std::fabs(I[8]);
    const bool ok = scale > 0.0 && std::fabs(det) > 1e-12 * scale * scale * scale;
    for (int k = 0; k < 9; ++k) hb.Iinv[k] = ok ? adj[k] / det : 0.0;
    return hb;
}

template <typename T>
Prm<T> make_prm(const pf_lbm *h) {
    Prm<T> p{};
    p.nx = h->cfg.nx;
    p.ny = h->cfg.ny;
    p.nz = h->cfg.nz;
    p.nb = h->nb;
    p.N = (int)h->N;
    p.Np = h->Np;
    p.omega = (T)(1.0 / h->cfg.tau);
    p.guo = (T)(1.0 - 0.5 / h->cfg.tau);
    p.G = (T)h->cfg.G;
    p.inv_rho0 = (T)(1.0 / h->cfg.rho0);
    p.rho0 = (T)h->cfg.rho0;
    for (int d = 0; d < 3; ++d) p.fext[d] = (T)h->cfg.fext[d];
    p.flags = h->cfg.flags;
    p.threshold = h->cfg.solid_threshold;
    p.mobility = h->cfg.mobility;
    p.eta = h->cfg.eta;
    p.r_c = h->cfg.r_c;
    p.n_exp = h->cfg.n_exp;
    p.e0 = h->cfg.e0;
    p.R_A = h->cfg.R_A;
    p.phi_floor = h->cfg.phi_floor;
    p.inv_n[0] = 1.0 / h->cfg.nx;
    p.inv_n[1] = 1.0 / h->cfg.ny;
    p.inv_n[2] = 1.0 / h->cfg.nz;
    const int n[3] = {h->cfg.nx, h->cfg.ny, h->cfg.nz}, te[3] = {TLX, TLY, TLZ};
    for (int d = 0; d < 3; ++d) {
        p.tn[d] = (n[d] + te[d] - 1) / te[d];
        // a last tile of fewer than 3 nodes lets a 3-node reach skip a whole tile
        const int last = n[d] - (p.tn[d] - 1) * te[d];
        p.trad[d] = (p.tn[d] >= 3 && last < 3) ? 2 : 1;
    }
    return p;
}

// Tile rows the fluid pass is built for with storage S on lattice Lat (4, 8 or 16, as its LDS
// budget allows)
template <typename S, class Lat>
bool fluid_ty_ok(int ty) {
    return ty == 4 || (ty == 8 && fluid_tile_fits<S, Lat, 8>()) || (ty == 16 && fluid_tile_fits<S, Lat, 16>());
}


// planes per z-chunk: the longest power of two in [4, 64] that still gives the grid 1024 blocks
// (four per CU), 4 when none does
int default_tz(int nx, int ny, int nz, int ty) {
    const long long tiles = (long long)((nx + 63) / 64) * ((ny + ty - 1) / ty);
    int tz = 64;
    while (tz > 4 && tiles * ((nz + tz - 1) / tz) < 1024) tz /= 2;
    return tz;
}

template <typename S, class Lat, int TY>
void launch_fluid_ty(pf_lbm *h, const Prm<ArT<S>> &p, const S *fc, S *fn, ArT<S> *psi, const ArT<S> *psi_prev,
                     const cell_t *mask, BodyDev *cur, int par, StepState *st, const ClassifyPart *cpart,
                     const uint32_t *nbw) {
    if constexpr (fluid_tile_fits<S, Lat, TY>()) {
        const int tz = h->fluid_tz;
        const unsigned tiles = (unsigned)(((h->cfg.nx + 63) / 64) * ((h->cfg.ny + TY - 1) / TY));
        const unsigned chunks = (unsigned)((h->cfg.nz + tz - 1) / tz);
        k_collide_stream<S, Lat, TY><<<dim3(tiles * chunks), dim3(64 * FluidShape<TY>::W), 0, h->stream>>>(
            p, fc, fn, psi, psi_prev, mask, cur, par, st, cpart, h->cgrid, nbw, tz);
    }
}

template <typename S, class Lat>
void launch_fluid(pf_lbm *h, const Prm<ArT<S>> &p, const S *fc, S *fn, ArT<S> *psi, const ArT<S> *psi_prev,
                  const cell_t *mask, BodyDev *cur, int par, StepState *st, const ClassifyPart *cpart,
                  const uint32_t *nbw) {
    if (h->fluid_ty == 16)
        launch_fluid_ty<S, Lat, 16>(h, p, fc, fn, psi, psi_prev, mask, cur, par, st, cpart, nbw);
    else if (h->fluid_ty == 8)
        launch_fluid_ty<S, Lat, 8>(h, p, fc, fn, psi, psi_prev, mask, cur, par, st, cpart, nbw);
    else
        launch_fluid_ty<S, Lat, 4>(h, p, fc, fn, psi, psi_prev, mask, cur, par, st, cpart, nbw);
}

template <typename T>
T *fbuf(pf_lbm *h, int which) {
    return (T *)(h->ws + (which ? h->L.fB : h->L.fA));
}

template <typename T>
void launch_phase_update(pf_lbm *h, const Prm<T> &p, int par, StepState *st, const BodyDev *bodies,
                         const double *sigma, const double *src, double *dst, cell_t *mask, ClassifyPart *cpart,
                         uint32_t *evlist, const uint32_t *tact, uint4 *tstate) {
    dim3 g(h->cgrid), b(256);
    if (h->nb <= 1)
        k_phase_update<T, 1><<<g, b, 0, h->stream>>>(p, par, st, bodies, sigma, src, dst, mask, cpart, evlist, h->ev_cap,
                                                      tact, tstate);
    else if (h->nb <= 2)
        k_phase_update<T, 2><<<g, b, 0, h->stream>>>(p, par, st, bodies, sigma, src, dst, mask, cpart, evlist, h->ev_cap,
                                                      tact, tstate);
    else if (h->nb <= 4)
        k_phase_update<T, 4><<<g, b, 0, h->stream>>>(p, par, st, bodies, sigma, src, dst, mask, cpart, evlist, h->ev_cap,
                                                      tact, tstate);
    else if (h->nb <= 8)
        k_phase_update<T, 8><<<g, b, 0, h->stream>>>(p, par, st, bodies, sigma, src, dst, mask, cpart, evlist, h->ev_cap,
                                                      tact, tstate);
    else
        k_phase_update<T, 16><<<g, b, 0, h->stream>>>(p, par, st, bodies, sigma, src, dst, mask, cpart, evlist, h->ev_cap,
                                                      tact, tstate);
}

// the three advection sweeps x (with the rigid-body update), y, z: a -> b -> a -> b
template <typename T, int NBMAX>
void launch_advect_n(pf_lbm *h, const Prm<T> &p, int par, StepState *st, const BodyDev *next, double *a, double *b,
                     const uint32_t *tact) {
    const dim3 g(h->box_grid), bl(256);
    hipStream_t s = h->stream;
    k_advect<T, 0, NBMAX><<<g, bl, 0, s>>>(p, par, st, next, a, b, tact);
    k_advect<T, 1, NBMAX><<<g, bl, 0, s>>>(p, par, st, next, b, a, tact);
    k_advect<T, 2, NBMAX><<<g, bl, 0, s>>>(p, par, st, next, a, b, tact);
}

template <typename T>
void launch_advect(pf_lbm *h, const Prm<T> &p, int par, StepState *st, const BodyDev *next, double *a, double *b,
                   const uint32_t *tact) {
    if (h->nb <= 1)
        launch_advect_n<T, 1>(h, p, par, st, next, a, b, tact);
    else if (h->nb <= 2)
        launch_advect_n<T, 2>(h, p, par, st, next, a, b, tact);
    else if (h->nb <= 4)
        launch_advect_n<T, 4>(h, p, par, st, next, a, b, tact);
    else if (h->nb <= 8)
        launch_advect_n<T, 8>(h, p, par, st, next, a, b, tact);
    else
        launch_advect_n<T, 16>(h, p, par, st, next, a, b, tact);
}

// one time step (Sec. 3): fluid, body forces + rigid update, phase fields, reclassification
template <typename S, class Lat>
int enqueue_step(pf_lbm *h, double *parts = nullptr) {
    using T = ArT<S>;
    const Prm<T> p = make_prm<T>(h);
    const int par = (int)(h->steps & 1);
    S *fc = fbuf<S>(h, par), *fn = fbuf<S>(h, par ^ 1);
    T *psi = (T *)(h->ws + (par ? h->L.psiB : h->L.psi));         // this step
    T *psi_prev = (T *)(h->ws + (par ? h->L.psi : h->L.psiB));    // the previous step
    double *phiA = (double *)(h->ws + h->L.phiA), *phiB = (double *)(h->ws + h->L.phiB);
    cell_t *mask = (cell_t *)(h->ws + h->L.mask);
    uint32_t *nbw = Lat::Q == 27 ? (uint32_t *)(h->ws + h->L.nbw) : nullptr;
    BodyDev *btab = (BodyDev *)(h->ws + h->L.bodies);
    const int nbm = std::max(h->nb, 1);
    BodyDev *cur = btab + par * nbm, *next = btab + (par ^ 1) * nbm;
    StepState *st = (StepState *)(h->ws + h->L.state);
    const double *sigma = (const double *)(h->ws + h->L.sigma);
    // per-block force partials: the workspace's, or the caller-supplied static copy
    double *pforce = parts ? parts : (double *)(h->ws + h->L.pforce);
    ClassifyPart *cpart = (ClassifyPart *)(h->ws + h->L.cpart);
    const dim3 b(256);
    hipStream_t s = h->stream;
    hipEvent_t *ev = nullptr;
    if (h->timing && h->timed < 4096) {
        if ((int)h->ev.size() < 4 * (h->timed + 1)) {
            for (int k = 0; k < 4; ++k) {
                hipEvent_t e;
                HIPCHK(h, hipEventCreate(&e));
                h->ev.push_back(e);
            }
        }
        ev = &h->ev[4 * h->timed];
        ++h->timed;
    }
    if (ev) HIPCHK(h, hipEventRecord(ev[0], s));
    uint32_t *evlist = (uint32_t *)(h->ws + h->L.evlist);
    if (ev) HIPCHK(h, hipEventRecord(ev[1], s));
    launch_fluid<S, Lat>(h, p, fc, fn, psi, psi_prev, mask, cur, par, st, h->nb > 0 ? cpart : nullptr, nbw);
    if (ev) HIPCHK(h, hipEventRecord(ev[2], s));
    if (h->nb > 0) {
        const int fbk = h->force_grid;
        uint4 *tstate = (uint4 *)(h->ws + h->L.tstate);
        uint32_t *thot = (uint32_t *)(h->ws + h->L.thot), *tact = (uint32_t *)(h->ws + h->L.tact);
        k_body_forces<S, Lat><<<dim3(fbk), dim3(64 * force_waves<T, Lat>()), 0, s>>>(p, par, st, fc, fn, psi, psi_prev,
                                                                                      mask, cur, pforce, nbw);
        // tile activity, and in its last block the rigid-body update from the force partials
        k_tile_activity<T><<<dim3(std::min(h->box_grid, 64) + 1), b, 0, s>>>(
            p, par, st, tstate, thot, tact, cur, next, pforce, fbk, (double *)(h->ws + h->L.hist), HIST_CAP);
        // one kernel per sweep; the phase fields end in buffer A every step
        launch_advect<T>(h, p, par, st, next, phiA, phiB, tact);
        launch_phase_update<T>(h, p, par, st, next, sigma, phiB, phiA, mask, cpart, evlist, tact, tstate);
        // conversion gather, then its closing pass: both usually return at once (no node changed
        // side), so a small grid
        const dim3 ge(std::min(h->box_grid, 64));
        k_convert_gather<S, Lat><<<ge, b, 0, s>>>(p, par, st, mask, fn, psi, evlist, h->ev_cap);
        k_close_events<S, Lat><<<ge, b, 0, s>>>(p, par, st, fn, mask, nbw, psi, evlist, h->ev_cap);
    }
    if (ev) HIPCHK(h, hipEventRecord(ev[3], s));
    HIPCHK(h, hipGetLastError());
    ++h->steps;
    return PF_LBM_OK;
}

template <typename S, class Lat>
int init_device(pf_lbm *h, const pf_lbm_body *bodies_in, const double *rho0, const double *phi0,
                const std::vector<BodyDev> &bodies, const StepState &st0) {
    using T = ArT<S>;
    const Prm<T> p = make_prm<T>(h);
    hipStream_t s = h->stream;
    double *phiA = (double *)(h->ws + h->L.phiA), *phiB = (double *)(h->ws + h->L.phiB);
    cell_t *mask = (cell_t *)(h->ws + h->L.mask);
    double *tmp = (double *)(h->ws + h->L.fB);  // staging for FP64 host fields
    StepState *st = (StepState *)(h->ws + h->L.state);
    const dim3 b(256);
    const int gd = std::max(1, std::min(h->dense_blocks, 65535));
    (void)bodies_in;
    const size_t tab = sizeof(BodyDev) * std::max(h->nb, 1);
    HIPCHK(h, hipMemcpyAsync(h->ws + h->L.bodies, bodies.data(), tab, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->ws + h->L.bodies + tab, bodies.data(), tab, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(st, &st0, sizeof(StepState), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->ws + h->L.sigma, h->sigma.data(), sizeof(double) * h->sigma.size(),
                             hipMemcpyHostToDevice, s));
    k_zero_mask<T><<<gd, b, 0, s>>>(p, mask);
    uint32_t *nbw = Lat::Q == 27 ? (uint32_t *)(h->ws + h->L.nbw) : nullptr;
    if (nbw) k_zero_mask<T><<<gd, b, 0, s>>>(p, nbw);
    // phase fields, one body at a time through the staging area
    for (int a = 0; a < h->nb; ++a) {
        HIPCHK(h, hipMemcpyAsync(tmp, phi0 + (size_t)a * h->N, sizeof(double) * h->N, hipMemcpyHostToDevice, s));
        Prm<T> q = p;
        q.nb = 1;
        k_init_phi<T><<<gd, b, 0, s>>>(q, tmp, phiA + (size_t)a * h->Np, phiB + (size_t)a * h->Np);
        HIPCHK(h, hipStreamSynchronize(s));
    }
    // solid / owner bits and the classification partials that the first step publishes
    if (h->nb > 0) {
        ClassifyPart *cpart = (ClassifyPart *)(h->ws + h->L.cpart);
        k_classify_init<T><<<dim3(h->cgrid), b, 0, s>>>(p, 0, st, (const BodyDev *)(h->ws + h->L.bodies), phiA,
                                                             mask, cpart);
        k_tile_init<T><<<dim3(std::max(1, std::min(gd, 4096))), b, 0, s>>>(p, phiA, (uint32_t *)(h->ws + h->L.tstate),
                                                                           (uint32_t *)(h->ws + h->L.thot));
    }
    HIPCHK(h, hipMemcpyAsync(tmp, rho0, sizeof(double) * h->N, hipMemcpyHostToDevice, s));
    S *fA = fbuf<S>(h, 0), *fB = fbuf<S>(h, 1);
    // populations at rest into fA (reads the staged density in the fB area) ...
    T *psi_init = (T *)(h->ws + h->L.psiB);  // the "previous step" of step 0
    k_init_f<S, Lat><<<gd, b, 0, s>>>(p, tmp, mask, (const BodyDev *)(h->ws + h->L.bodies), psi_init, fA);
    HIPCHK(h, hipStreamSynchronize(s));
    // ... then clear fB (solid nodes keep empty populations in both buffers)
    HIPCHK(h, hipMemsetAsync(fB, 0, (size_t)Lat::Q * h->Np * sizeof(S), s));
    // neighbour bits of the cell words
    if (h->nb > 0)
        k_post<S, Lat><<<dim3(h->box_grid), b, 0, s>>>(p, 0, st, mask, nbw, fA, psi_init);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipStreamSynchronize(s));
    return PF_LBM_OK;
}

template <typename S, class Lat>
void launch_fields(pf_lbm *h, int which, int par, void *dst, int dst_dtype) {
    using T = ArT<S>;
    const dim3 g(std::max(1, std::min(h->dense_blocks, 65535))), b(256);
    const cell_t *mask = (const cell_t *)(h->ws + h->L.mask);
    const Prm<T> p = make_prm<T>(h);
    const S *f = fbuf<S>(h, par);
    // pseudopotential of the last step taken (before the first step: that of the initial state)
    const T *psi = (const T *)(h->ws + (par ? h->L.psi : h->L.psiB));
    const double *phi = (const double *)(h->ws + h->L.phiA);
    if (dst_dtype == PF_LBM_DST_F64)
        k_fields<S, double, Lat><<<g, b, 0, h->stream>>>(p, which, f, mask, psi, phi, (double *)dst);
    else
        k_fields<S, float, Lat><<<g, b, 0, h->stream>>>(p, which, f, mask, psi, phi, (float *)dst);
}

}  // namespace

extern "C" {

int pf_lbm_init(const pf_lbm_config *cfg, int32_t n_bodies, const pf_lbm_body *bodies, const double *rho0,
                const double *phi0, void *workspace, size_t ws_bytes, void *hip_stream, pf_lbm **out,
                size_t *ws_bytes_needed) {
    g_init_error.clear();
    if (!cfg) return fail(nullptr, PF_LBM_EINVAL, "cfg is NULL");
    if (cfg->struct_size < sizeof(pf_lbm_config))
        return fail(nullptr, PF_LBM_EINVAL, "cfg->struct_size %u < %zu", cfg->struct_size, sizeof(pf_lbm_config));
    if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1) return fail(nullptr, PF_LBM_EINVAL, "grid sizes must be >= 1");
    const long long N = (long long)cfg->nx * cfg->ny * cfg->nz;
    if (N * 27 >= (1LL << 31) * 8LL || N >= (1LL << 31)) return fail(nullptr, PF_LBM_EINVAL, "grid too large");
    if (n_bodies < 0 || n_bodies > PF_LBM_MAX_BODIES)
        return fail(nullptr, PF_LBM_EINVAL, "n_bodies must be in [0, %d]", PF_LBM_MAX_BODIES);
    if (cfg->lattice != PF_LBM_D3Q19 && cfg->lattice != PF_LBM_D3Q27)
        return fail(nullptr, PF_LBM_EUNSUPPORTED, "lattice must be PF_LBM_D3Q19 or PF_LBM_D3Q27");
    if (cfg->precision != PF_LBM_FP64 && cfg->precision != PF_LBM_FP32 && cfg->precision != PF_LBM_FP16_STORE)
        return fail(nullptr, PF_LBM_EUNSUPPORTED, "precision must be PF_LBM_FP64, PF_LBM_FP32 or PF_LBM_FP16_STORE");
    if (!(cfg->tau > 0.5)) return fail(nullptr, PF_LBM_EINVAL, "tau must exceed 1/2");
    if (!(cfg->rho0 > 0.0)) return fail(nullptr, PF_LBM_EINVAL, "rho0 must be positive");
    if (!(cfg->eta > 0.0)) return fail(nullptr, PF_LBM_EINVAL, "eta must be positive");
    if (!(cfg->R_A >= 1.0 - 1e-12 && cfg->R_A <= std::sqrt(3.0) + 1e-12))
        return fail(nullptr, PF_LBM_EUNSUPPORTED, "R_A must lie in [1, sqrt(3)]");
    if ((cfg->flags & PF_LBM_REPULSION) && !(cfg->r_c > 0.0 && cfg->r_c <= 4.0))
        return fail(nullptr, PF_LBM_EUNSUPPORTED, "r_c must lie in (0, 4]");
    if (!(cfg->phi_floor >= 0.0 && cfg->phi_floor < 0.5)) return fail(nullptr, PF_LBM_EINVAL, "phi_floor must lie in [0, 0.5)");
    if (!(cfg->solid_threshold > 0.0 && cfg->solid_threshold < 1.0))
        return fail(nullptr, PF_LBM_EINVAL, "solid_threshold must lie in (0, 1)");
    if (n_bodies > 0 && (!bodies || !phi0)) return fail(nullptr, PF_LBM_EINVAL, "bodies and phi0 are required");
    for (int a = 0; a < n_bodies; ++a)
        if (!(bodies[a].mass_density > 0.0)) return fail(nullptr, PF_LBM_EINVAL, "body %d: mass_density must be > 0", a);

    const long long Np = (N + 63) / 64 * 64;
    std::vector<char> occ[3] = {std::vector<char>(cfg->nx, 0), std::vector<char>(cfg->ny, 0),
                                std::vector<char>(cfg->nz, 0)};
    bool any = false;
    if (n_bodies > 0) {
        for (int a = 0; a < n_bodies; ++a)
            for (long long i = 0; i < N; ++i)
                if (phi0[(size_t)a * N + i] > 0.0) {
                    const int x = (int)(i % cfg->nx), y = (int)((i / cfg->nx) % cfg->ny), z = (int)(i / ((long long)cfg->nx * cfg->ny));
                    occ[0][x] = occ[1][y] = occ[2][z] = 1;
                    any = true;
                }
    }
    int box[6] = {0, 0, 0, -1, -1, -1};
    if (any) {
        const int n[3] = {cfg->nx, cfg->ny, cfg->nz};
        for (int d = 0; d < 3; ++d) {
            int start = 0, ext = n[d];
            if (!axis_gap(occ[d], start, ext)) {
                start = 0;
                ext = n[d];
            }
            int lo = start - 3, hi = start + ext - 1 + 3;
            if (hi - lo + 1 >= n[d]) {
                lo = 0;
                hi = n[d] - 1;
            } else if (lo < 0) {  // lower corner in [0, n): unwrapped coordinates stay below 2 n
                lo += n[d];
                hi += n[d];
            }
            box[d] = lo;
            box[3 + d] = hi;
        }
    }
    const long long vol0 = any ? (long long)(box[3] - box[0] + 1) * (box[4] - box[1] + 1) * (box[5] - box[2] + 1) : 0;
    // box kernels: one tile of 256 nodes per block, about one block per tile of the initial box
    // with room to grow, at most 4096 (larger boxes are covered by grid-stride loops): each tile's
    // work is a short chain of dependent loads, which many resident blocks overlap
    const int box_blocks = (int)std::max(1LL, std::min(4096LL, (3 * vol0 / 2 + 255) / 256));
    const int box_grid = box_blocks;
    const int force_grid = std::min((box_blocks + 3) / 4, FORCE_GRID_MAX);
    // phase update (and the classification partials it leaves): grid-stride over the tiles.  With
    // up to 4 bodies and a box above 2^19 cells, three 4-wave blocks per CU, as many as a CU holds
    // at that variant's registers, in one round (four per CU ran a second round and were no
    // faster); otherwise two blocks per CU, four for boxes above 2^20 cells.  Each block's partials
    // are summed at the start of the next step, so more blocks cost there.
    const int cgrid = std::min(box_blocks, (n_bodies <= 4 && vol0 > (1LL << 19)) ? 768
                                           : (vol0 > (1LL << 20) ? 1024 : 512));
    const long long ntiles = (long long)((cfg->nx + TLX - 1) / TLX) * ((cfg->ny + TLY - 1) / TLY) * ((cfg->nz + TLZ - 1) / TLZ);
    const Layout L = make_layout(Np, n_bodies, cfg->precision, cfg->lattice, std::max(cgrid, box_grid), force_grid,
                                 ntiles);
    if (ws_bytes_needed) *ws_bytes_needed = L.total;
    if (!workspace) return PF_LBM_OK;
    if (!out) return fail(nullptr, PF_LBM_EINVAL, "out is NULL");
    if (ws_bytes < L.total) return fail(nullptr, PF_LBM_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
    if ((uintptr_t)workspace % ALIGN) return fail(nullptr, PF_LBM_EINVAL, "workspace must be 256-byte aligned");
    if (!rho0) return fail(nullptr, PF_LBM_EINVAL, "rho0 is NULL");

    pf_lbm *h = new (std::nothrow) pf_lbm();
    if (!h) return fail(nullptr, PF_LBM_ENOMEM, "host allocation failed");
    h->cfg = *cfg;
    h->cfg.sigma = nullptr;
    h->nb = n_bodies;
    h->prec = cfg->precision;
    h->q = cfg->lattice;
    h->stream = (hipStream_t)hip_stream;
    h->ws = (char *)workspace;
    h->L = L;
    h->N = N;
    h->Np = Np;
    h->dense_blocks = (int)((N + 255) / 256);
    h->box_blocks = box_blocks;
    h->box_grid = box_grid;
    h->force_grid = force_grid;
    h->cgrid = cgrid;
    h->fluid_ty = cfg->precision == PF_LBM_FP64 ? 4 : 8;
    h->fluid_tz = default_tz(cfg->nx, cfg->ny, cfg->nz, h->fluid_ty);
    const int np1 = n_bodies + 1;
    h->sigma.assign((size_t)np1 * np1, 0.0);
    for (int a = 0; a < np1; ++a)
        for (int b = 0; b < np1; ++b)
            h->sigma[a * np1 + b] = cfg->sigma ? cfg->sigma[a * np1 + b] : (a == b ? 0.0 : ((a == 0 || b == 0) ? 1.0 : 0.5));

    std::vector<BodyDev> bd(std::max(n_bodies, 1));
    std::memset(bd.data(), 0, sizeof(BodyDev) * bd.size());
    for (int a = 0; a < n_bodies; ++a) {
        const HostBody hb = body_moments(phi0 + (size_t)a * N, cfg->nx, cfg->ny, cfg->nz, bodies[a].mass_density);
        BodyDev &B = bd[a];
        B.M = hb.M;
        for (int k = 0; k < 9; ++k) B.Iinv[k] = hb.Iinv[k];
        for (int d = 0; d < 3; ++d) {
            B.X[d] = hb.X[d];
            B.V[d] = bodies[a].v[d];
            B.W[d] = bodies[a].w[d];
        }
        B.psi_s = 1.0 - std::exp(-bodies[a].wetting_rho / cfg->rho0);
        B.Vref = hb.Vref;
        B.fixed = bodies[a].fixed ? 1 : 0;
    }
    StepState st0;
    std::memset(&st0, 0, sizeof st0);
    for (int d = 0; d < 6; ++d) st0.box[0][d] = st0.box[1][d] = box[d];
    if ((h->cfg.flags & PF_LBM_REPULSION) && h->cfg.r_c > 0.0 && h->cfg.r_c <= 4.0) {
        const double rc = h->cfg.r_c;
        const int R = (int)std::ceil(rc);
        for (int dz = -R; dz <= R; ++dz)
            for (int dy = -R; dy <= R; ++dy)
                for (int dx = -R; dx <= R; ++dx) {
                    const int d2 = dx * dx + dy * dy + dz * dz;
                    if (d2 == 0 || !((double)d2 < rc * rc)) continue;
                    // Sec. 3.1.2: e0 (n / r_c) |(r - r_c) / r_c|^(n - 1) at node distance r < r_c
                    const double r = std::sqrt((double)d2);
                    const double mag =
                        r < rc ? h->cfg.e0 * (h->cfg.n_exp / rc) * std::pow(std::fabs((r - rc) / rc), h->cfg.n_exp - 1.0) : 0.0;
                    st0.rep_f[st0.n_rep][0] = -dx / r * mag;
                    st0.rep_f[st0.n_rep][1] = -dy / r * mag;
                    st0.rep_f[st0.n_rep][2] = -dz / r * mag;
                    st0.rep_off[st0.n_rep++] = (dx + 8) | (dy + 8) << 8 | (dz + 8) << 16;
                }
    }
    int rc = h->q == 27 ? (h->prec == PF_LBM_FP64   ? init_device<double, D3Q27>(h, bodies, rho0, phi0, bd, st0)
                           : h->prec == PF_LBM_FP32 ? init_device<float, D3Q27>(h, bodies, rho0, phi0, bd, st0)
                                                    : init_device<half_t, D3Q27>(h, bodies, rho0, phi0, bd, st0))
                        : (h->prec == PF_LBM_FP64   ? init_device<double, D3Q19>(h, bodies, rho0, phi0, bd, st0)
                           : h->prec == PF_LBM_FP32 ? init_device<float, D3Q19>(h, bodies, rho0, phi0, bd, st0)
                                                    : init_device<half_t, D3Q19>(h, bodies, rho0, phi0, bd, st0));
    if (rc != PF_LBM_OK) {
        g_init_error = h->err;
        delete h;
        return rc;
    }
    *out = h;
    return PF_LBM_OK;
}

namespace {

int eager_step(pf_lbm *h, double *parts = nullptr) {
    if (h->q == 27)
        return h->prec == PF_LBM_FP64 ? enqueue_step<double, D3Q27>(h, parts)
               : h->prec == PF_LBM_FP32 ? enqueue_step<float, D3Q27>(h, parts)
                                        : enqueue_step<half_t, D3Q27>(h, parts);
    return h->prec == PF_LBM_FP64 ? enqueue_step<double, D3Q19>(h, parts)
           : h->prec == PF_LBM_FP32 ? enqueue_step<float, D3Q19>(h, parts)
                                    : enqueue_step<half_t, D3Q19>(h, parts);
}

// Device address of this GPU's copy of the static force partials, looked up once per device
// (with that device current) and kept.
std::mutex g_static_mu;
double *g_static_ptr[MAX_DEVICES] = {};

int static_parts(pf_lbm *h, double **out) {
    int dev = -1;
    HIPCHK(h, hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(h, PF_LBM_EUNSUPPORTED, "device %d beyond %d", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *ptr = nullptr;
        HIPCHK(h, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_static_ptr[dev] = (double *)ptr;
    }
    *out = g_static_ptr[dev];
    return PF_LBM_OK;
}

constexpr int GRAPH_STEPS[2] = {2, 32};

void drop_graphs(pf_lbm *h) {
    for (hipGraphExec_t &g : h->graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    h->graph_failed = false;
    ++h->gen;
}

// capture GRAPH_STEPS[k] steps (an even number, starting at an even step) on the handle's
// stream into an executable graph; on any failure the handle keeps launching kernels one by one
bool ensure_graph(pf_lbm *h, int k) {
    if (h->graph[k]) return true;
    if (h->graph_failed || !h->stream || (h->steps & 1)) return false;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
        (void)hipGetLastError();
        h->graph_failed = true;
        return false;
    }
    const long long s0 = h->steps;
    int rc = PF_LBM_OK;
    for (int j = 0; j < GRAPH_STEPS[k] && rc == PF_LBM_OK; ++j) rc = eager_step(h);
    h->steps = s0;
    const hipError_t e = hipStreamEndCapture(h->stream, &g);
    if (rc != PF_LBM_OK || e != hipSuccess || !g) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        h->graph_failed = true;
        return false;
    }
    const hipError_t e2 = hipGraphInstantiate(&h->graph[k], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
        (void)hipGetLastError();
        h->graph[k] = nullptr;
        h->graph_failed = true;
        return false;
    }
    return true;
}

}  // namespace

int pf_lbm_step(pf_lbm *h, int32_t n_steps) {
    if (!h) return fail(nullptr, PF_LBM_EINVAL, "handle is NULL");
    if (n_steps < 0) return fail(h, PF_LBM_EINVAL, "n_steps must be >= 0");
    int n = n_steps;
    if (n > 0 && (h->steps & 1)) {
        const int rc = eager_step(h);
        if (rc != PF_LBM_OK) return rc;
        --n;
    }
    for (int k = 1; k >= 0; --k) {
        while (n >= GRAPH_STEPS[k] && !h->timing && ensure_graph(h, k)) {
            HIPCHK(h, hipGraphLaunch(h->graph[k], h->stream));
            h->steps += GRAPH_STEPS[k];
            n -= GRAPH_STEPS[k];
        }
    }
    for (; n > 0; --n) {
        const int rc = eager_step(h);
        if (rc != PF_LBM_OK) return rc;
    }
    return PF_LBM_OK;
}

int pf_lbm_step_noalloc(pf_lbm *h, int32_t n_steps) {
    if (!h) return fail(nullptr, PF_LBM_EINVAL, "handle is NULL");
    if (n_steps < 0) return fail(h, PF_LBM_EINVAL, "n_steps must be >= 0");
    if (h->timing) return fail(h, PF_LBM_EINVAL, "pf_lbm_step_noalloc does not record timing events");
    const size_t need = (size_t)h->force_grid * std::max(h->nb, 1) * 6;
    if (need > STATIC_PARTS)
        return fail(h, PF_LBM_EUNSUPPORTED, "force partials of %zu doubles exceed the static %zu", need, STATIC_PARTS);
    double *parts = nullptr;
    const int rc0 = static_parts(h, &parts);
    if (rc0 != PF_LBM_OK) return rc0;
    // kernels launched one by one (no graph is captured or replayed): every step writes all the
    // partials it reads, so the array needs no clearing
    for (int k = 0; k < n_steps; ++k) {
        const int rc = eager_step(h, parts);
        if (rc != PF_LBM_OK) return rc;
    }
    return PF_LBM_OK;
}

int pf_lbm_forces(pf_lbm *h, double *F, double *T, double *X, double *V, double *W) {
    if (!h) return fail(nullptr, PF_LBM_EINVAL, "handle is NULL");
    std::vector<BodyDev> bd(std::max(h->nb, 1));
    StepState st;
    const size_t tab = sizeof(BodyDev) * bd.size();
    HIPCHK(h, hipMemcpyAsync(bd.data(), h->ws + h->L.bodies + (h->steps & 1) * tab, tab, hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipMemcpyAsync(&st, h->ws + h->L.state, sizeof st, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int a = 0; a < h->nb; ++a)
        for (int d = 0; d < 3; ++d) {
            if (F) F[3 * a + d] = bd[a].F[d];
            if (T) T[3 * a + d] = bd[a].T[d];
            if (X) X[3 * a + d] = bd[a].X[d];
            if (V) V[3 * a + d] = bd[a].V[d];
            if (W) W[3 * a + d] = bd[a].W[d];
        }
    if (st.err & 1u) return fail(h, PF_LBM_ENONFINITE, "non-finite body force or state");
    if (st.err & 2u) return fail(h, PF_LBM_ENONFINITE, "advection velocity above one cell per step");
    return PF_LBM_OK;
}

int pf_lbm_fields(pf_lbm *h, int32_t which, void *dst, int32_t dst_dtype) {
    if (!h) return fail(nullptr, PF_LBM_EINVAL, "handle is NULL");
    if (!dst) return fail(h, PF_LBM_EINVAL, "dst is NULL");
    const bool ok = (which >= 0 && which <= 6) || (which >= PF_LBM_FIELD_PHI && which < PF_LBM_FIELD_PHI + h->nb);
    if (!ok) return fail(h, PF_LBM_EINVAL, "unknown field %d", which);
    if (dst_dtype != PF_LBM_DST_F64 && dst_dtype != PF_LBM_DST_F32) return fail(h, PF_LBM_EINVAL, "bad dst dtype");
    const int par = (int)(h->steps & 1);
    if (h->q == 27) {
        if (h->prec == PF_LBM_FP64)
            launch_fields<double, D3Q27>(h, which, par, dst, dst_dtype);
        else if (h->prec == PF_LBM_FP32)
            launch_fields<float, D3Q27>(h, which, par, dst, dst_dtype);
        else
            launch_fields<half_t, D3Q27>(h, which, par, dst, dst_dtype);
    } else {
        if (h->prec == PF_LBM_FP64)
            launch_fields<double, D3Q19>(h, which, par, dst, dst_dtype);
        else if (h->prec == PF_LBM_FP32)
            launch_fields<float, D3Q19>(h, which, par, dst, dst_dtype);
        else
            launch_fields<half_t, D3Q19>(h, which, par, dst, dst_dtype);
    }
    HIPCHK(h, hipGetLastError());
    return PF_LBM_OK;
}

int pf_lbm_diagnostics(pf_lbm *h, double *out4) {
    if (!h || !out4) return fail(h, PF_LBM_EINVAL, "handle or output is NULL");
    StepState st;
    HIPCHK(h, hipMemcpyAsync(&st, h->ws + h->L.state, sizeof st, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    out4[0] = (double)h->steps;
    out4[1] = (double)st.n_f2s;
    out4[2] = (double)st.n_s2f;
    out4[3] = (double)st.n_lost;
    return PF_LBM_OK;
}

int pf_lbm_timing(pf_lbm *h, int32_t enable, double *out4) {
    if (!h) return fail(nullptr, PF_LBM_EINVAL, "handle is NULL");
    if (enable) {
        h->timing = true;
        h->timed = 0;
        return PF_LBM_OK;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    double kern = 0.0, step = 0.0;
    for (int k = 0; k < h->timed; ++k) {
        float a = 0.f, b = 0.f;
        HIPCHK(h, hipEventElapsedTime(&a, h->ev[4 * k + 1], h->ev[4 * k + 2]));
        HIPCHK(h, hipEventElapsedTime(&b, h->ev[4 * k + 0], h->ev[4 * k + 3]));
        kern += a;
        step += b;
    }
    if (out4) {
        out4[0] = h->timed;
        out4[1] = h->timed ? kern / h->timed : 0.0;
        out4[2] = h->timed ? step / h->timed : 0.0;
        out4[3] = 0.0;
    }
    h->timing = false;
    return PF_LBM_OK;
}

int pf_lbm_force_history(pf_lbm *h, int32_t max_steps, double *out, int32_t *n_out) {
    if (!h) return fail(nullptr, PF_LBM_EINVAL, "handle is NULL");
    if (max_steps < 0 || (max_steps > 0 && !out)) return fail(h, PF_LBM_EINVAL, "bad output");
    const long long avail = std::min<long long>(h->nb > 0 ? h->steps : 0, HIST_CAP);
    const int n = (int)std::min<long long>(avail, max_steps);
    if (n_out) *n_out = n;
    if (n == 0) return PF_LBM_OK;
    const size_t row = sizeof(double) * h->nb * 6;
    std::vector<double> ring((size_t)HIST_CAP * h->nb * 6);
    HIPCHK(h, hipMemcpyAsync(ring.data(), h->ws + h->L.hist, ring.size() * sizeof(double), hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int k = 0; k < n; ++k) {
        const long long step = h->steps - n + k;  // 0-based index of the step
        std::memcpy((char *)out + (size_t)k * row, (const char *)ring.data() + (size_t)(step % HIST_CAP) * row, row);
    }
    return PF_LBM_OK;
}

int pf_lbm_step_batch(pf_lbm *const *handles, int32_t n, int32_t n_steps) {
    if (!handles || n < 0) return fail(nullptr, PF_LBM_EINVAL, "handles is NULL or n < 0");
    if (n_steps < 0) return fail(nullptr, PF_LBM_EINVAL, "n_steps must be >= 0");
    for (int i = 0; i < n; ++i)
        if (!handles[i]) return fail(nullptr, PF_LBM_EINVAL, "handle %d is NULL", i);
    // step pairs round robin over the instances: each handle launches on its own stream, so the
    // launches of different instances queue side by side and their kernels overlap
    for (int done = 0; done < n_steps; done += 2) {
        const int chunk = std::min(2, n_steps - done);
        for (int i = 0; i < n; ++i) {
            const int rc = pf_lbm_step(handles[i], chunk);
            if (rc != PF_LBM_OK) return rc;
        }
    }
    return PF_LBM_OK;
}

}  // extern "C"

// A batch: the steps of many instances captured as one HIP graph (a fork from the first
// instance's stream, each instance's kernels on its own stream, a join back), replayed as one
// launch.
struct pf_lbm_batch {
    std::vector<pf_lbm *> hs;
    int graph_steps = 2;
    hipGraphExec_t graph = nullptr;
    std::vector<int> parity;              // step parity of each instance at capture
    std::vector<unsigned> gen;            // launch-shape generation of each instance at capture
    std::vector<hipEvent_t> ev;           // one per instance (fork, join and ordering)
    std::string err;
};

namespace {

int bfail(pf_lbm_batch *b, int code, const std::string &msg) {
    b->err = msg;
    return code;
}

#define BCHK(b, call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return bfail((b), PF_LBM_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

// capture graph_steps steps of every instance into one executable graph
int batch_capture(pf_lbm_batch *b) {
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    hipStream_t origin = b->hs[0]->stream;
    const int n = (int)b->hs.size();
    std::vector<long long> s0(n);
    for (int i = 0; i < n; ++i) s0[i] = b->hs[i]->steps;
    BCHK(b, hipStreamBeginCapture(origin, hipStreamCaptureModeRelaxed));
    int rc = PF_LBM_OK;
    hipError_t he = hipEventRecord(b->ev[0], origin);
    for (int i = 1; i < n && he == hipSuccess; ++i)
        if (b->hs[i]->stream != origin) he = hipStreamWaitEvent(b->hs[i]->stream, b->ev[0], 0);
    for (int k = 0; k < b->graph_steps && rc == PF_LBM_OK && he == hipSuccess; ++k)
        for (int i = 0; i < n && rc == PF_LBM_OK; ++i) rc = eager_step(b->hs[i]);
    for (int i = 1; i < n && he == hipSuccess; ++i)
        if (b->hs[i]->stream != origin) {
            he = hipEventRecord(b->ev[i], b->hs[i]->stream);
            if (he == hipSuccess) he = hipStreamWaitEvent(origin, b->ev[i], 0);
        }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(origin, &g);
    for (int i = 0; i < n; ++i) b->hs[i]->steps = s0[i];
    if (rc != PF_LBM_OK || he != hipSuccess || e != hipSuccess || !g) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        return bfail(b, rc != PF_LBM_OK ? rc : PF_LBM_EDEVICE, "capture of the batch failed");
    }
    const hipError_t e2 = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
        b->graph = nullptr;
        return bfail(b, PF_LBM_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
    }
    for (int i = 0; i < n; ++i) {
        b->parity[i] = (int)(b->hs[i]->steps & 1);
        b->gen[i] = b->hs[i]->gen;
    }
    return PF_LBM_OK;
}

}  // namespace

extern "C" {

int pf_lbm_batch_create(pf_lbm *const *handles, int32_t n, int32_t graph_steps, pf_lbm_batch **out) {
    if (!handles || n < 1 || !out) return fail(nullptr, PF_LBM_EINVAL, "handles or out is NULL, or n < 1");
    if (graph_steps < 2 || (graph_steps & 1)) return fail(nullptr, PF_LBM_EINVAL, "graph_steps must be even and >= 2");
    for (int i = 0; i < n; ++i) {
        if (!handles[i]) return fail(nullptr, PF_LBM_EINVAL, "handle %d is NULL", i);
        if (!handles[i]->stream) return fail(nullptr, PF_LBM_EINVAL, "handle %d is bound to the default stream", i);
        for (int j = 0; j < i; ++j)
            if (handles[j] == handles[i]) return fail(nullptr, PF_LBM_EINVAL, "handle %d repeats handle %d", i, j);
    }
    pf_lbm_batch *b = new (std::nothrow) pf_lbm_batch();
    if (!b) return fail(nullptr, PF_LBM_ENOMEM, "host allocation failed");
    b->hs.assign(handles, handles + n);
    b->graph_steps = graph_steps;
    b->parity.assign(n, -1);
    b->gen.assign(n, 0u);
    b->ev.resize(n, nullptr);
    for (int i = 0; i < n; ++i)
        if (hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming) != hipSuccess) {
            pf_lbm_batch_destroy(b);
            return fail(nullptr, PF_LBM_EDEVICE, "hipEventCreateWithFlags failed");
        }
    *out = b;
    return PF_LBM_OK;
}

int pf_lbm_batch_step(pf_lbm_batch *b, int32_t n_steps) {
    if (!b) return fail(nullptr, PF_LBM_EINVAL, "batch is NULL");
    if (n_steps < 0) return bfail(b, PF_LBM_EINVAL, "n_steps must be >= 0");
    const int n = (int)b->hs.size();
    for (pf_lbm *h : b->hs)
        if (h->timing) return bfail(b, PF_LBM_EINVAL, "a handle of the batch is timing");
    hipStream_t origin = b->hs[0]->stream;
    int left = n_steps;
    while (left >= b->graph_steps) {
        bool same = b->graph != nullptr;
        for (int i = 0; i < n && same; ++i)
            same = b->parity[i] == (int)(b->hs[i]->steps & 1) && b->gen[i] == b->hs[i]->gen;
        if (!same) {
            const int rc = batch_capture(b);
            if (rc != PF_LBM_OK) return rc;
        }
        // work queued on the instances' own streams precedes the replay, which precedes any
        // later work on them
        for (int i = 1; i < n; ++i)
            if (b->hs[i]->stream != origin) {
                BCHK(b, hipEventRecord(b->ev[i], b->hs[i]->stream));
                BCHK(b, hipStreamWaitEvent(origin, b->ev[i], 0));
            }
        BCHK(b, hipGraphLaunch(b->graph, origin));
        BCHK(b, hipEventRecord(b->ev[0], origin));
        for (int i = 1; i < n; ++i)
            if (b->hs[i]->stream != origin) BCHK(b, hipStreamWaitEvent(b->hs[i]->stream, b->ev[0], 0));
        for (pf_lbm *h : b->hs) h->steps += b->graph_steps;
        left -= b->graph_steps;
    }
    if (left > 0) {
        pf_lbm *const *hs = b->hs.data();
        const int rc = pf_lbm_step_batch(hs, n, left);
        if (rc != PF_LBM_OK) return bfail(b, rc, "remainder steps failed");
    }
    return PF_LBM_OK;
}

void pf_lbm_batch_destroy(pf_lbm_batch *b) {
    if (!b) return;
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    for (hipEvent_t e : b->ev)
        if (e) (void)hipEventDestroy(e);
    delete b;
}

const char *pf_lbm_batch_last_error(const pf_lbm_batch *b) { return b ? b->err.c_str() : g_init_error.c_str(); }

int pf_lbm_autotune(pf_lbm *h, int32_t steps_per_candidate, double *out3) {
    if (!h) return fail(nullptr, PF_LBM_EINVAL, "handle is NULL");
    if (steps_per_candidate < 2) return fail(h, PF_LBM_EINVAL, "steps_per_candidate must be >= 2");
    if (h->timing) return fail(h, PF_LBM_EINVAL, "autotune while timing is on");
    const int ty_c[3] = {4, 8, 16}, tz_c[5] = {4, 8, 16, 32, 64};
    auto ty_ok = [&](int ty) {
        if (h->q == 27)
            return h->prec == PF_LBM_FP64 ? fluid_ty_ok<double, D3Q27>(ty)
                   : h->prec == PF_LBM_FP32 ? fluid_ty_ok<float, D3Q27>(ty) : fluid_ty_ok<half_t, D3Q27>(ty);
        return h->prec == PF_LBM_FP64 ? fluid_ty_ok<double, D3Q19>(ty)
               : h->prec == PF_LBM_FP32 ? fluid_ty_ok<float, D3Q19>(ty) : fluid_ty_ok<half_t, D3Q19>(ty);
    };
    hipEvent_t e0, e1;
    HIPCHK(h, hipEventCreate(&e0));
    HIPCHK(h, hipEventCreate(&e1));
    double best = 1e300;
    int best_ty = h->fluid_ty, best_tz = h->fluid_tz;
    for (int ty : ty_c)
        for (int tz : tz_c) {
            if (!ty_ok(ty) || (tz > h->cfg.nz && tz != tz_c[0])) continue;
            h->fluid_ty = ty;
            h->fluid_tz = tz;
            // one untimed step with the candidate, then the timed ones (launched one by one)
            int rc = eager_step(h);
            if (rc == PF_LBM_OK) {
                HIPCHK(h, hipEventRecord(e0, h->stream));
                for (int k = 0; k < steps_per_candidate && rc == PF_LBM_OK; ++k) rc = eager_step(h);
                HIPCHK(h, hipEventRecord(e1, h->stream));
            }
            if (rc != PF_LBM_OK) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return rc;
            }
            HIPCHK(h, hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(h, hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                best_ty = ty;
                best_tz = tz;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->fluid_ty = best_ty;
    h->fluid_tz = best_tz;
    // the captured steps used the old shapes: capture again on the next pf_lbm_step
    drop_graphs(h);
    if (out3) {
        out3[0] = best_ty;
        out3[1] = best_tz;
        out3[2] = best / steps_per_candidate;
    }
    return PF_LBM_OK;
}

int pf_lbm_set_tile(pf_lbm *h, int32_t rows, int32_t planes) {
    if (!h) return fail(nullptr, PF_LBM_EINVAL, "handle is NULL");
    bool ok;
    if (h->q == 27)
        ok = h->prec == PF_LBM_FP64 ? fluid_ty_ok<double, D3Q27>(rows)
             : h->prec == PF_LBM_FP32 ? fluid_ty_ok<float, D3Q27>(rows) : fluid_ty_ok<half_t, D3Q27>(rows);
    else
        ok = h->prec == PF_LBM_FP64 ? fluid_ty_ok<double, D3Q19>(rows)
             : h->prec == PF_LBM_FP32 ? fluid_ty_ok<float, D3Q19>(rows) : fluid_ty_ok<half_t, D3Q19>(rows);
    if (!ok) return fail(h, PF_LBM_EUNSUPPORTED, "tile of %d rows not built for this precision and lattice", rows);
    if (planes < 1 || planes > 4096) return fail(h, PF_LBM_EINVAL, "planes per chunk must lie in [1, 4096]");
    h->fluid_ty = rows;
    h->fluid_tz = planes;
    drop_graphs(h);
    return PF_LBM_OK;
}

int pf_lbm_set_event_capacity(pf_lbm *h, int32_t entries) {
    if (!h) return fail(nullptr, PF_LBM_EINVAL, "handle is NULL");
    if (entries < 0 || (uint32_t)entries > EV_CAP)
        return fail(h, PF_LBM_EINVAL, "event capacity must lie in [0, %u]", EV_CAP);
    h->ev_cap = (uint32_t)entries;
    drop_graphs(h);
    return PF_LBM_OK;
}

void pf_lbm_destroy(pf_lbm *h) {
    if (!h) return;
    drop_graphs(h);
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    delete h;
}

const char *pf_lbm_last_error(const pf_lbm *h) { return h ? h->err.c_str() : g_init_error.c_str(); }

}  // extern "C"
