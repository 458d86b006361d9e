// Learned pairwise bridge-force surrogate: an MLP whose forward and backward matrix products run
// as hand-written BF16 MFMA kernels (v_mfma_f32_16x16x32_bf16, FP32 accumulation) on gfx950.
// See include/pf_mlp.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pf_mlp.h"

namespace pfm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_grad(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// C[M][N] = A[M][K] B[K][N] (+ bias[n]) with arbitrary element strides, BF16 operands, FP32
// accumulation.  One wave per 16 x 16 output tile, four tiles per block; K advances 32 at a time
// through one MFMA.  Operand layout of v_mfma_f32_16x16x32_bf16: lane l holds A[l % 16][8 (l / 16)
// + j] and B[8 (l / 16) + j][l % 16], j = 0..7; the result D[4 (l / 16) + r][l % 16], r = 0..3.
// Epilogue: Cf (FP32, may be NULL) receives the sum z; Cb (BF16, may be NULL) receives z, or
// silu(z) when act != 0.  Elements outside [M) x [N) x [K) read as zero and are not written.
struct Gemm {
    const __bf16 *A;
    long long sam, sak;
    const __bf16 *B;
    long long sbk, sbn;
    float *Cf;
    __bf16 *Cb;
    long long scm, scn;
    const float *bias;
    int M, N, K, act;
    int vec;  // k_gemm_bf16_rows: 16-byte operand loads (K, row strides multiples of 8, aligned bases)
};

__global__ __launch_bounds__(256) void k_gemm_bf16(Gemm g) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tiles_n = (g.N + 15) / 16;
    const int tile = blockIdx.x * 4 + wave;
    const int tiles = ((g.M + 15) / 16) * tiles_n;
    if (tile >= tiles) return;  // whole wave
    const int tm = tile / tiles_n, tn = tile - tm * tiles_n;
    const int row = tm * 16 + (lane & 15), col = tn * 16 + (lane & 15), kq = 8 * (lane >> 4);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += 32) {
        bf16x8 a, b;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = k0 + kq + j;
            a[j] = (row < g.M && k < g.K) ? g.A[row * g.sam + k * g.sak] : (__bf16)0.0f;
            b[j] = (col < g.N && k < g.K) ? g.B[k * g.sbk + col * g.sbn] : (__bf16)0.0f;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int m = tm * 16 + 4 * (lane >> 4) + r, n = col;
        if (m >= g.M || n >= g.N) continue;
        const float z = acc[r] + (g.bias ? g.bias[n] : 0.0f);
        const long long o = m * g.scm + n * g.scn;
        if (g.Cf) g.Cf[o] = z;
        if (g.Cb) g.Cb[o] = (__bf16)(g.act ? silu(z) : z);
    }
}

// The same product when A and B are contiguous along K (sak = sbk = 1) and N >= 16, with the
// BF16 result written row-major (scn = 1).  A block of 4 waves computes 64 rows across up to
// 16 NT columns (blockIdx.y picks the column chunk): the B columns are staged in LDS, 128 K values
// at a time (rows padded by 16 bytes so that the 16 lanes reading one K chunk of 16 columns hit
// distinct banks), and each wave takes a 16-row strip, loading its A fragment (one 16-byte load
// per lane when g.vec, else element by element) and reusing it for the NT products of the strip.
// The BF16 strip is written through LDS as 16-byte row segments.  Every wave takes part in the
// staging, also one past the last row.
template <int NT>
__global__ __launch_bounds__(256) void k_gemm_bf16_rows(Gemm g) {
    constexpr int KC = 128, LD = KC + 8;
    __shared__ __attribute__((aligned(16))) __bf16 wl[16 * NT][LD];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int tm = blockIdx.x * 4 + wave;
    const int n0 = blockIdx.y * 16 * NT;
    const int row = tm * 16 + (lane & 15), kq = 8 * (lane >> 4);
    const bool active = tm * 16 < g.M;
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero = {};
    for (int kc = 0; kc < g.K; kc += KC) {
        for (int e = tid * 8; e < 16 * NT * KC; e += 256 * 8) {
            const int r = e / KC, c = e - r * KC;
            bf16x8 v = zero;
            if (n0 + r < g.N) {
                const __bf16 *src = g.B + (long long)(n0 + r) * g.sbn + kc + c;
                if (g.vec) {
                    if (kc + c < g.K) v = *(const bf16x8 *)src;
                } else {
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        if (kc + c + j < g.K) v[j] = src[j];
                }
            }
            *(bf16x8 *)&wl[r][c] = v;
        }
        __syncthreads();
        if (active) {
            for (int k0 = 0; k0 < KC && kc + k0 < g.K; k0 += 32) {
                const int k = kc + k0 + kq;
                bf16x8 a = zero;
                if (row < g.M) {
                    const __bf16 *src = g.A + row * g.sam + k;
                    if (g.vec) {
                        if (k < g.K) a = *(const bf16x8 *)src;
                    } else {
#pragma unroll
                        for (int j = 0; j < 8; ++j)
                            if (k + j < g.K) a[j] = src[j];
                    }
                }
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    if (n0 + 16 * t >= g.N) break;  // uniform
                    const bf16x8 b = *(const bf16x8 *)&wl[16 * t + (lane & 15)][k0 + kq];
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    // epilogue: z = acc + bias; FP32 z element by element; the BF16 strip (16 x 16 NT) goes to
    // this wave's part of the (now free) staging area, then out as 16-byte row segments
    __bf16 *strip = &wl[0][0] + wave * (16 * 16 * NT);
    const int ncols = min(16 * NT, g.N - n0);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (16 * t >= ncols) break;
        const int nl = 16 * t + (lane & 15), n = n0 + nl;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ml = 4 * (lane >> 4) + r, m = tm * 16 + ml;
            const float z = acc[t][r] + (g.bias && n < g.N ? g.bias[n] : 0.0f);
            if (active && g.Cf && m < g.M && n < g.N) g.Cf[m * g.scm + n] = z;
            strip[ml * (16 * NT) + nl] = (__bf16)(g.act ? silu(z) : z);
        }
    }
    __syncthreads();
    if (!active || !g.Cb) return;
    // 16 rows x ncols columns, ncols a multiple of 16: 8-element segments
    const int segs = ncols / 8;
    for (int q = lane; q < 16 * segs; q += 64) {
        const int ml = q / segs, c = (q - ml * segs) * 8, m = tm * 16 + ml;
        if (m >= g.M) continue;
        __bf16 *dst = g.Cb + m * g.scm + n0 + c;
        const bf16x8 v = *(const bf16x8 *)&strip[ml * (16 * NT) + c];
        if (g.vec)
            *(bf16x8 *)dst = v;
        else
            for (int j = 0; j < 8; ++j) dst[j] = v[j];
    }
}

// Output layer with one output: y = A w + b over K (a multiple of 8) BF16 inputs, 16 lanes per
// row (each takes 8 consecutive inputs per 128), summed across the 16 lanes in a fixed order.
__global__ __launch_bounds__(256) void k_last_layer(const __bf16 *__restrict__ A, int M, int K,
                                                    const __bf16 *__restrict__ w, const float *__restrict__ bias,
                                                    float *__restrict__ y) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    const int row = (int)(t >> 4), sub = (int)(t & 15);
    float acc = 0.0f;
    if (row < M) {
        for (int k = 8 * sub; k < K; k += 128) {
            const bf16x8 a = *(const bf16x8 *)(A + (long long)row * K + k);
            const bf16x8 b = *(const bf16x8 *)(w + k);
#pragma unroll
            for (int j = 0; j < 8; ++j) acc = fmaf((float)a[j], (float)b[j], acc);
        }
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
    if (row < M && sub == 0) y[row] = acc + bias[0];
}

// BF16 copy of an FP32 array
__global__ void k_to_bf16(const float *__restrict__ x, __bf16 *__restrict__ y, int n) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) y[i] = (__bf16)x[i];
}

// BF16 copies of the weights of every layer, row-major [out][in] and transposed [in][out]
struct LayerMap {
    int n;                       // layers incl. the output layer
    int in[10], out[10];
    long long w[10], b[10];      // offsets in the parameter vector
    long long wb[10];            // offsets in the BF16 weight copies
};
__global__ void k_refresh_weights(LayerMap lm, const float *__restrict__ p, __bf16 *__restrict__ wb,
                                  __bf16 *__restrict__ wt) {
    for (int l = 0; l < lm.n; ++l) {
        const int I = lm.in[l], O = lm.out[l];
        for (int i = blockIdx.x * 256 + threadIdx.x; i < I * O; i += gridDim.x * 256) {
            const int o = i / I, k = i - o * I;
            const __bf16 v = (__bf16)p[lm.w[l] + i];
            wb[lm.wb[l] + i] = v;
            wt[lm.wb[l] + (long long)k * O + o] = v;
        }
    }
}

// Whole forward pass for hidden width 128 and up to 32 inputs (inference): a block of 4 waves
// carries 64 rows through every layer.  Each wave keeps its 16-row activation strip in LDS (BF16,
// rows padded by 16 bytes), the block stages one layer's weights at a time in LDS, and every
// hidden product runs on v_mfma_f32_16x16x32_bf16 with the A fragment read from the strip; the
// first layer takes the FP32 inputs rounded to BF16 (K padded with zeros to 32) and the output
// layer is a dot product of each strip row with the output weights (4 lanes per row, fixed
// order).  Only the inputs and outputs cross HBM.  The arithmetic of each product is that of the
// layer-by-layer path; the output sum runs in another fixed order.
__global__ __launch_bounds__(256) void k_mlp_forward_fused(const float *__restrict__ x, int M, int nin, LayerMap lm,
                                                           const __bf16 *__restrict__ Wb, const float *__restrict__ P,
                                                           float *__restrict__ y) {
    constexpr int H = 128, LD = H + 8, NT = H / 16;
    __shared__ __attribute__((aligned(16))) __bf16 wl[H][LD];
    __shared__ __attribute__((aligned(16))) __bf16 act[4][16][LD];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int tm = blockIdx.x * 4 + wave;
    const int rowl = lane & 15, kq = 8 * (lane >> 4);
    const int row = tm * 16 + rowl;
    const bool active = tm * 16 < M;
    const bf16x8 zero = {};
    f32x4 acc[NT];
    // ---- layer 0 (K = nin <= 32, one product step)
    {
        const __bf16 *W = Wb + lm.wb[0];
        for (int e = tid; e < H * 32; e += 256) {
            const int r = e >> 5, c = e & 31;
            wl[r][c] = c < nin ? W[r * nin + c] : (__bf16)0.0f;
        }
        __syncthreads();
        bf16x8 a = zero;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (active && row < M && kq + j < nin) a[j] = (__bf16)x[(long long)row * nin + kq + j];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const bf16x8 b = *(const bf16x8 *)&wl[16 * t + rowl][kq];
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        }
        const float *bias = P + lm.b[0];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                act[wave][4 * (lane >> 4) + r][16 * t + rowl] = (__bf16)silu(acc[t][r] + bias[16 * t + rowl]);
        __syncthreads();
    }
    // ---- hidden layers
    for (int l = 1; l < lm.n - 1; ++l) {
        const __bf16 *W = Wb + lm.wb[l];
        for (int e = tid * 8; e < H * H; e += 256 * 8) {
            const int r = e / H, c = e - r * H;
            *(bf16x8 *)&wl[r][c] = *(const bf16x8 *)(W + e);
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < H; k0 += 32) {
            const bf16x8 a = *(const bf16x8 *)&act[wave][rowl][k0 + kq];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const bf16x8 b = *(const bf16x8 *)&wl[16 * t + rowl][k0 + kq];
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
            }
        }
        __syncthreads();  // every wave is done with the staged weights and its strip
        const float *bias = P + lm.b[l];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                act[wave][4 * (lane >> 4) + r][16 * t + rowl] = (__bf16)silu(acc[t][r] + bias[16 * t + rowl]);
        __syncthreads();
    }
    // ---- output layer: row 4 lanes x 32 inputs
    const int L = lm.n - 1;
    const __bf16 *w = Wb + lm.wb[L];
    const int rr = lane >> 2, part = lane & 3;
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = 32 * part + 8 * q;
        const bf16x8 a = *(const bf16x8 *)&act[wave][rr][k];
        const bf16x8 b = *(const bf16x8 *)(w + k);
#pragma unroll
        for (int j = 0; j < 8; ++j) s = fmaf((float)a[j], (float)b[j], s);
    }
    s += __shfl_xor(s, 1, 4);
    s += __shfl_xor(s, 2, 4);
    const int m = tm * 16 + rr;
    if (active && part == 0 && m < M) y[m] = s + P[lm.b[L]];
}

// dZ = dA * silu'(Z) (FP32 and BF16)
__global__ void k_silu_back(const float *__restrict__ dA, const float *__restrict__ Z, float *__restrict__ dZ,
                            __bf16 *__restrict__ dZb, int n) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const float v = dA[i] * silu_grad(Z[i]);
        dZ[i] = v;
        dZb[i] = (__bf16)v;
    }
}

// db[j] = sum_b dZ[b][j], one thread per output column, fixed order
__global__ void k_bias_grad(const float *__restrict__ dZ, int B, int O, float *__restrict__ db) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= O) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += dZ[(long long)b * O + j];
    db[j] = s;
}

// mean-squared-error loss (FP64 sum, one block, fixed order) and dY = 2 (y - t) / n
__global__ __launch_bounds__(256) void k_loss(const float *__restrict__ y, const float *__restrict__ t, int n,
                                              float *__restrict__ dy, __bf16 *__restrict__ dyb,
                                              double *__restrict__ loss) {
    __shared__ double part[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const float e = y[i] - t[i];
        s += (double)e * e;
        const float g = 2.0f * e / (float)n;
        dy[i] = g;
        dyb[i] = (__bf16)g;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = part[0] / n;
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float c1, float c2) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

}  // namespace pfm

using namespace pfm;

struct pf_mlp {
    pf_mlp_config cfg;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    LayerMap lm{};
    long long np = 0, nwb = 0;
    // workspace offsets
    size_t P, G, Mo, Vo, Wb, Wt, Xb, Y, dY, dYb, loss, dA, dZ, dZb, Z[10], A[10];
    int adam_t = 0;
    std::string err;
};

namespace {

thread_local std::string g_mlp_init_error;

int mfail(pf_mlp *h, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h)
        h->err = buf;
    else
        g_mlp_init_error = buf;
    return code;
}

#define MCHK(h, call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return mfail((h), PF_LBM_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

template <typename X>
X *at(pf_mlp *h, size_t off) {
    return (X *)(h->ws + off);
}

void gemm(pf_mlp *h, const __bf16 *A, long long sam, long long sak, const __bf16 *B, long long sbk, long long sbn,
          float *Cf, __bf16 *Cb, long long scm, long long scn, const float *bias, int M, int N, int K, int act) {
    Gemm g{A, sam, sak, B, sbk, sbn, Cf, Cb, scm, scn, bias, M, N, K, act, 0};
    g.vec = K % 8 == 0 && sam % 8 == 0 && sbn % 8 == 0 && scm % 8 == 0 && ((uintptr_t)A % 16) == 0 &&
            ((uintptr_t)B % 16) == 0 && ((uintptr_t)Cb % 16) == 0;
    const bool rows = sak == 1 && sbk == 1 && scn == 1 && N >= 16 && N % 16 == 0;
    if (rows) {
        constexpr int NT = 8;
        const dim3 grid((unsigned)(((M + 15) / 16 + 3) / 4), (unsigned)((N + 16 * NT - 1) / (16 * NT)));
        k_gemm_bf16_rows<NT><<<grid, 256, 0, h->stream>>>(g);
        return;
    }
    const int tiles = ((M + 15) / 16) * ((N + 15) / 16);
    k_gemm_bf16<<<(tiles + 3) / 4, 256, 0, h->stream>>>(g);
}

int grid_for(long long n) { return (int)std::max(1LL, std::min(4096LL, (n + 255) / 256)); }

// forward pass of n samples; leaves A_l (and with keep_z the FP32 pre-activations Z_l, which only
// the backward pass needs) and the output in the workspace
int run_forward(pf_mlp *h, const float *x, int n, bool keep_z, float *y_out = nullptr) {
    const LayerMap &lm = h->lm;
    const int nin = h->cfg.n_in;
    k_to_bf16<<<grid_for((long long)n * nin), 256, 0, h->stream>>>(x, at<__bf16>(h, h->Xb), n * nin);
    for (int l = 0; l < lm.n; ++l) {
        const int I = lm.in[l], O = lm.out[l];
        const __bf16 *Ain = l == 0 ? at<__bf16>(h, h->Xb) : at<__bf16>(h, h->A[l - 1]);
        const bool last = l == lm.n - 1;
        const __bf16 *Wl = at<__bf16>(h, h->Wb) + lm.wb[l];
        const float *bl = at<float>(h, h->P) + lm.b[l];
        float *Zl = last ? (y_out ? y_out : at<float>(h, h->Y)) : (keep_z ? at<float>(h, h->Z[l]) : nullptr);
        if (last && O == 1 && I % 8 == 0) {
            const long long th = (long long)n * 16;
            k_last_layer<<<(unsigned)((th + 255) / 256), 256, 0, h->stream>>>(Ain, n, I, Wl, bl, Zl);
        } else {
            // Z = A_in W^T + b: B[k][n] = W[n][k]
            gemm(h, Ain, I, 1, Wl, 1, I, Zl, last ? nullptr : at<__bf16>(h, h->A[l]), O, 1, bl, n, O, I, last ? 0 : 1);
        }
    }
    MCHK(h, hipGetLastError());
    return PF_LBM_OK;
}

// backward pass after run_forward and the loss kernel: parameter gradients into G
int run_backward(pf_mlp *h, int n) {
    const LayerMap &lm = h->lm;
    float *G = at<float>(h, h->G);
    // gradient of the output layer's pre-activation: dY
    const float *dZf = at<float>(h, h->dY);
    const __bf16 *dZb = at<__bf16>(h, h->dYb);
    for (int l = lm.n - 1; l >= 0; --l) {
        const int I = lm.in[l], O = lm.out[l];
        const __bf16 *Ain = l == 0 ? at<__bf16>(h, h->Xb) : at<__bf16>(h, h->A[l - 1]);
        // dW[o][i] = sum_b dZ[b][o] A_in[b][i]: A-operand (m = o, k = b), B-operand (k = b, n = i)
        gemm(h, dZb, 1, O, Ain, I, 1, G + lm.w[l], nullptr, I, 1, nullptr, O, I, n, 0);
        k_bias_grad<<<(O + 255) / 256, 256, 0, h->stream>>>(dZf, n, O, G + lm.b[l]);
        if (l == 0) break;
        // dA_in[b][i] = sum_o dZ[b][o] W[o][i]: B-operand (k = o, n = i) from the transposed copy
        gemm(h, dZb, O, 1, at<__bf16>(h, h->Wt) + lm.wb[l], 1, O, at<float>(h, h->dA), nullptr, I, 1, nullptr, n, I, O,
             0);
        // dZ of the layer below
        float *dZn = at<float>(h, h->dZ) + (size_t)(l & 1) * h->cfg.max_batch * h->cfg.hidden;
        __bf16 *dZbn = at<__bf16>(h, h->dZb) + (size_t)(l & 1) * h->cfg.max_batch * h->cfg.hidden;
        k_silu_back<<<grid_for((long long)n * I), 256, 0, h->stream>>>(at<float>(h, h->dA), at<float>(h, h->Z[l - 1]), dZn,
                                                                        dZbn, n * I);
        dZf = dZn;
        dZb = dZbn;
    }
    MCHK(h, hipGetLastError());
    return PF_LBM_OK;
}

int loss_and_grad(pf_mlp *h, const float *x, const float *t, int n) {
    int rc = run_forward(h, x, n, true);
    if (rc != PF_LBM_OK) return rc;
    k_loss<<<1, 256, 0, h->stream>>>(at<float>(h, h->Y), t, n, at<float>(h, h->dY), at<__bf16>(h, h->dYb),
                                     at<double>(h, h->loss));
    return run_backward(h, n);
}

uint64_t splitmix64(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int upload_params(pf_mlp *h, const float *params) {
    MCHK(h, hipMemcpyAsync(h->ws + h->P, params, sizeof(float) * h->np, hipMemcpyHostToDevice, h->stream));
    MCHK(h, hipMemsetAsync(h->ws + h->Mo, 0, sizeof(float) * h->np, h->stream));
    MCHK(h, hipMemsetAsync(h->ws + h->Vo, 0, sizeof(float) * h->np, h->stream));
    k_refresh_weights<<<grid_for(h->nwb), 256, 0, h->stream>>>(h->lm, at<float>(h, h->P), at<__bf16>(h, h->Wb),
                                                                 at<__bf16>(h, h->Wt));
    MCHK(h, hipGetLastError());
    MCHK(h, hipStreamSynchronize(h->stream));
    h->adam_t = 0;
    return PF_LBM_OK;
}

}  // namespace

__attribute__((visibility("hidden"))) void pfm_internal_info(const pf_mlp *h, int *n_in, int *max_batch,
                                                             void **stream) {
    *n_in = h ? h->cfg.n_in : 0;
    *max_batch = h ? h->cfg.max_batch : 0;
    *stream = h ? (void *)h->stream : nullptr;
}

extern "C" {

int pf_mlp_init(const pf_mlp_config *cfg, uint64_t seed, void *workspace, size_t ws_bytes, void *hip_stream,
                pf_mlp **out, size_t *ws_bytes_needed) {
    g_mlp_init_error.clear();
    if (!cfg) return mfail(nullptr, PF_LBM_EINVAL, "cfg is NULL");
    if (cfg->struct_size < sizeof(pf_mlp_config)) return mfail(nullptr, PF_LBM_EINVAL, "bad struct_size");
    if (cfg->n_in < 1 || cfg->n_in > 16) return mfail(nullptr, PF_LBM_EINVAL, "n_in must be in [1, 16]");
    if (cfg->hidden < 16 || cfg->hidden > 512 || cfg->hidden % 16)
        return mfail(nullptr, PF_LBM_EINVAL, "hidden must be a multiple of 16 in [16, 512]");
    if (cfg->layers < 1 || cfg->layers > 8) return mfail(nullptr, PF_LBM_EINVAL, "layers must be in [1, 8]");
    if (cfg->max_batch < 1 || cfg->max_batch > 65536) return mfail(nullptr, PF_LBM_EINVAL, "max_batch in [1, 65536]");
    pf_mlp tmp;
    tmp.cfg = *cfg;
    LayerMap &lm = tmp.lm;
    lm.n = cfg->layers + 1;
    long long np = 0, nwb = 0;
    for (int l = 0; l < lm.n; ++l) {
        lm.in[l] = l == 0 ? cfg->n_in : cfg->hidden;
        lm.out[l] = l == lm.n - 1 ? 1 : cfg->hidden;
        lm.w[l] = np;
        np += (long long)lm.in[l] * lm.out[l];
        lm.b[l] = np;
        np += lm.out[l];
        lm.wb[l] = nwb;
        nwb += (long long)lm.in[l] * lm.out[l];
    }
    tmp.np = np;
    tmp.nwb = nwb;
    const long long B = cfg->max_batch, H = cfg->hidden;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) / 256 * 256;
        return o;
    };
    tmp.P = take(4 * np);
    tmp.G = take(4 * np);
    tmp.Mo = take(4 * np);
    tmp.Vo = take(4 * np);
    tmp.Wb = take(2 * nwb);
    tmp.Wt = take(2 * nwb);
    tmp.Xb = take(2 * B * cfg->n_in);
    tmp.Y = take(4 * B);
    tmp.dY = take(4 * B);
    tmp.dYb = take(2 * B);
    tmp.loss = take(8);
    tmp.dA = take(4 * B * H);
    tmp.dZ = take(4 * 2 * B * H);
    tmp.dZb = take(2 * 2 * B * H);
    for (int l = 0; l < lm.n - 1; ++l) {
        tmp.Z[l] = take(4 * B * H);
        tmp.A[l] = take(2 * B * H);
    }
    if (ws_bytes_needed) *ws_bytes_needed = off;
    if (!workspace) return PF_LBM_OK;
    if (!out) return mfail(nullptr, PF_LBM_EINVAL, "out is NULL");
    if (ws_bytes < off) return mfail(nullptr, PF_LBM_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, off);
    if ((uintptr_t)workspace % 256) return mfail(nullptr, PF_LBM_EINVAL, "workspace must be 256-byte aligned");
    pf_mlp *h = new (std::nothrow) pf_mlp(tmp);
    if (!h) return mfail(nullptr, PF_LBM_ENOMEM, "host allocation failed");
    h->ws = (char *)workspace;
    h->stream = (hipStream_t)hip_stream;
    // seeded initialisation: W ~ U(-sqrt(6 / in), sqrt(6 / in)), b = 0
    std::vector<float> p((size_t)np, 0.0f);
    uint64_t s = seed;
    for (int l = 0; l < lm.n; ++l) {
        const double a = std::sqrt(6.0 / lm.in[l]);
        for (long long i = 0; i < (long long)lm.in[l] * lm.out[l]; ++i) {
            const double u = (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
            p[lm.w[l] + i] = (float)((2.0 * u - 1.0) * a);
        }
    }
    const int rc = upload_params(h, p.data());
    if (rc != PF_LBM_OK) {
        g_mlp_init_error = h->err;
        delete h;
        return rc;
    }
    *out = h;
    return PF_LBM_OK;
}

int32_t pf_mlp_num_params(const pf_mlp *h) { return h ? (int32_t)h->np : 0; }

int pf_mlp_set_params(pf_mlp *h, const float *params) {
    if (!h || !params) return mfail(h, PF_LBM_EINVAL, "handle or params is NULL");
    return upload_params(h, params);
}

int pf_mlp_get_params(pf_mlp *h, float *params) {
    if (!h || !params) return mfail(h, PF_LBM_EINVAL, "handle or params is NULL");
    MCHK(h, hipMemcpyAsync(params, h->ws + h->P, sizeof(float) * h->np, hipMemcpyDeviceToHost, h->stream));
    MCHK(h, hipStreamSynchronize(h->stream));
    return PF_LBM_OK;
}

int pf_mlp_forward(pf_mlp *h, const float *x, int32_t n, float *y) {
    if (!h || !x || !y) return mfail(h, PF_LBM_EINVAL, "NULL argument");
    if (n < 1 || n > h->cfg.max_batch) return mfail(h, PF_LBM_EINVAL, "n must be in [1, max_batch]");
    if (h->cfg.hidden == 128 && h->cfg.n_in <= 32) {
        k_mlp_forward_fused<<<(unsigned)((n + 63) / 64), 256, 0, h->stream>>>(x, n, h->cfg.n_in, h->lm,
                                                                            at<__bf16>(h, h->Wb), at<float>(h, h->P), y);
        MCHK(h, hipGetLastError());
        return PF_LBM_OK;
    }
    return run_forward(h, x, n, false, y);
}

int pf_mlp_gradients(pf_mlp *h, const float *x, const float *t, int32_t n, float *grad, double *loss) {
    if (!h || !x || !t || !grad) return mfail(h, PF_LBM_EINVAL, "NULL argument");
    if (n < 1 || n > h->cfg.max_batch) return mfail(h, PF_LBM_EINVAL, "n must be in [1, max_batch]");
    const int rc = loss_and_grad(h, x, t, n);
    if (rc != PF_LBM_OK) return rc;
    MCHK(h, hipMemcpyAsync(grad, h->ws + h->G, sizeof(float) * h->np, hipMemcpyDeviceToHost, h->stream));
    if (loss) MCHK(h, hipMemcpyAsync(loss, h->ws + h->loss, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    MCHK(h, hipStreamSynchronize(h->stream));
    return PF_LBM_OK;
}

int pf_mlp_train_step(pf_mlp *h, const float *x, const float *t, int32_t n, float lr, double *loss) {
    if (!h || !x || !t) return mfail(h, PF_LBM_EINVAL, "NULL argument");
    if (n < 1 || n > h->cfg.max_batch) return mfail(h, PF_LBM_EINVAL, "n must be in [1, max_batch]");
    if (!(lr > 0.0f)) return mfail(h, PF_LBM_EINVAL, "lr must be positive");
    int rc = loss_and_grad(h, x, t, n);
    if (rc != PF_LBM_OK) return rc;
    ++h->adam_t;
    const float c1 = 1.0f - std::pow(0.9f, (float)h->adam_t), c2 = 1.0f - std::pow(0.999f, (float)h->adam_t);
    k_adam<<<grid_for(h->np), 256, 0, h->stream>>>(at<float>(h, h->P), at<float>(h, h->G), at<float>(h, h->Mo),
                                                    at<float>(h, h->Vo), (int)h->np, lr, c1, c2);
    k_refresh_weights<<<grid_for(h->nwb), 256, 0, h->stream>>>(h->lm, at<float>(h, h->P), at<__bf16>(h, h->Wb),
                                                                 at<__bf16>(h, h->Wt));
    MCHK(h, hipGetLastError());
    if (loss) {
        MCHK(h, hipMemcpyAsync(loss, h->ws + h->loss, sizeof(double), hipMemcpyDeviceToHost, h->stream));
        MCHK(h, hipStreamSynchronize(h->stream));
    }
    return PF_LBM_OK;
}

void pf_mlp_destroy(pf_mlp *h) { delete h; }

const char *pf_mlp_last_error(const pf_mlp *h) { return h ? h->err.c_str() : g_mlp_init_error.c_str(); }

}  // extern "C"
