// Learned warm start: a three-layer perceptron (two GELU hidden layers)
// that maps a world's state features to the dual impulses of the coming
// step.  Not part of the paper, whose only warm start is the previous
// step's impulses (Sec. 4.1): the network only moves the starting point of
// the ADMM iteration, whose exit test is unchanged.
//
// Every contraction runs on the matrix cores: v_mfma_f32_16x16x32_bf16 with
// BF16 operands (round to nearest even from FP32) and FP32 accumulation.
// Master weights, biases, Adam moments and gradients stay FP32.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "kamx_internal.h"

namespace kamx {

namespace {

constexpr int kTileM = 64, kTileN = 64, kTileK = 32;
constexpr int kLdsRow = kTileK + 8;  // bf16 per LDS tile row (16-byte pad)
constexpr int kGemmThreads = 256;
constexpr int kColBlocks = 32;  // row blocks of the bias-gradient column sums

// Weight gradients are sums over the batch (K): split K so that the
// launch has about 512 workgroups, each slice at least 128 rows long.
inline int grad_splits(int M, int N, int K) {
    const int tiles = (M / kTileM) * (N / kTileN);
    int s = 1;
    while (tiles * s < 512 && K % (2 * s * kTileK) == 0 && K / (2 * s) >= 128) s *= 2;
    return s;
}


// element (i, k) of an operand at p[i * si + k * sk]; one of the strides is 1
struct Operand {
    const __bf16 *p;
    long si, sk;
};

enum Epilogue { kEpiHidden = 0, kEpiOut = 1, kEpiBackward = 2, kEpiStore = 3 };

struct EpiArgs {
    const float *bias;  // [N] (hidden, out)
    float *f32;         // hidden: z; out: normalised output; backward: dz; store: C
    __bf16 *b16;        // hidden: gelu(z); backward: dz
    long ld;            // row stride of f32 / b16 / z
    const float *z;     // backward: pre-activation
    float *y;           // out: de-standardised output [batch, n_out] (may be null)
    long ldy;
    int batch, n_out;
    const float *mu, *sigma;
    long split;         // store: stride between the K slices' partial results
};


// Stage a 64 x 32 tile of an operand (rows i0.., columns k0..) into LDS as
// [row][k] so that every matrix-core operand is one 16-byte LDS read.
__device__ inline void stage(const Operand &o, long i0, long k0, __bf16 *tile) {
    const int t = threadIdx.x;
    if (o.sk == 1) {
        const int r = t >> 2, kc = (t & 3) * 8;
        bf16x8 v = *reinterpret_cast<const bf16x8 *>(o.p + (i0 + r) * o.si + k0 + kc);
        *reinterpret_cast<bf16x8 *>(tile + r * kLdsRow + kc) = v;
    } else {
        const int k = t >> 3, ic = (t & 7) * 8;
        bf16x8 v = *reinterpret_cast<const bf16x8 *>(o.p + (k0 + k) * o.sk + i0 + ic);
#pragma unroll
        for (int j = 0; j < 8; ++j) tile[(ic + j) * kLdsRow + k] = v[j];
    }
}

// C[M, N] = sum_k A(m, k) B(n, k), M, N multiples of 64 and K of 32 (the
// host pads every dimension).  Four waves, each a 32 x 32 quarter of the
// tile as 2 x 2 matrix-core blocks of 16 x 16.
template <int EPI>
__global__ __launch_bounds__(kGemmThreads) void gemm_kernel(Operand A, Operand B, int M, int N, int K, EpiArgs e) {
    __shared__ __attribute__((aligned(16))) __bf16 As[kTileM * kLdsRow];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[kTileN * kLdsRow];
    const long m0 = (long)blockIdx.y * kTileM, n0 = (long)blockIdx.x * kTileN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // split K: slice blockIdx.z of gridDim.z takes K / gridDim.z of the sum
    const int kspan = K / (int)gridDim.z, kb = (int)blockIdx.z * kspan;
    for (int k0 = kb; k0 < kb + kspan; k0 += kTileK) {
        __syncthreads();
        stage(A, m0, k0, As);
        stage(B, n0, k0, Bs);
        __syncthreads();
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8 *>(As + (wm + 16 * i + fr) * kLdsRow + fk);
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(Bs + (wn + 16 * j + fr) * kLdsRow + fk);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    // lane holds rows 4 (lane / 16) + c of column lane % 16 of each block
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const long m = m0 + wm + 16 * i + (lane >> 4) * 4 + c;
                const long n = n0 + wn + 16 * j + (lane & 15);
                const float v = acc[i][j][c];
                if (EPI == kEpiHidden) {
                    float z = v + e.bias[n];
                    if (e.f32) e.f32[m * e.ld + n] = z;
                    e.b16[m * e.ld + n] = to_bf16(gelu(z));
                } else if (EPI == kEpiOut) {
                    float yn = v + e.bias[n];
                    if (e.f32) e.f32[m * e.ld + n] = yn;
                    if (e.y && m < e.batch && n < e.n_out) e.y[m * e.ldy + n] = __builtin_fmaf(e.sigma[n], yn, e.mu[n]);
                } else if (EPI == kEpiBackward) {
                    float dz = v * gelu_grad(e.z[m * e.ld + n]);
                    e.f32[m * e.ld + n] = dz;
                    e.b16[m * e.ld + n] = to_bf16(dz);
                } else {
                    e.f32[(long)blockIdx.z * e.split + m * e.ld + n] = v;
                }
            }
}

// x^ = (x - mu) * s in BF16, zero in padded rows and columns.
__global__ void normalise_kernel(const float *x, long ldx, int batch, int n_in, const float *mu, const float *s,
                                 __bf16 *xh, int rows, int fp) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)rows * fp) return;
    int b = (int)(idx / fp), i = (int)(idx - (long)b * fp);
    float v = 0.f;
    if (b < batch && i < n_in) v = (x[(long)b * ldx + i] - mu[i]) * s[i];
    xh[idx] = to_bf16(v);
}

// Output gradient of the mean squared error on standardised targets, and
// per-block partial sums of the squared error (fixed order).
__global__ void loss_grad_kernel(const float *yn, const float *t, int batch, int n_out, int op, const float *mu,
                                 const float *sigma, float *dy, __bf16 *dyb, int rows, float *partial) {
    __shared__ float red[256];
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    float sq = 0.f;
    if (idx < (long)rows * op) {
        int b = (int)(idx / op), o = (int)(idx - (long)b * op);
        float g = 0.f;
        if (b < batch && o < n_out) {
            float tn = (t[(long)b * n_out + o] - mu[o]) / sigma[o];
            float err = yn[idx] - tn;
            sq = err * err;
            g = 2.f * err / ((float)batch * (float)n_out);
        }
        dy[idx] = g;
        dyb[idx] = to_bf16(g);
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void loss_final_kernel(const float *partial, int n, float scale, float *loss) {
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] * scale;
}

// Column sums of a [rows, n] FP32 matrix (bias gradients) in two passes
// with a fixed order: block (x, y) sums rows y*rows/ny .. of 64 columns in
// 4 row groups into partial[y][col]; then every column adds its ny partials.
__global__ __launch_bounds__(256) void colsum_partial_kernel(const float *a, int rows, int n, float *partial) {
    __shared__ float red[4][64];
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + c;
    const int span = rows / (int)gridDim.y, r0 = (int)blockIdx.y * span;
    float s = 0.f;
    if (col < n)
        for (int r = r0 + g; r < r0 + span; r += 4) s += a[(long)r * n + col];
    red[g][c] = s;
    __syncthreads();
    if (g == 0 && col < n) partial[(long)blockIdx.y * n + col] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
}

// out[i] = sum over s of part[s * stride + i], s in order (the partial
// results of a split sum)
__global__ void sum_slices_kernel(const float *part, long stride, int ns, long n, float *out) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float t = 0.f;
    for (int k = 0; k < ns; ++k) t += part[(long)k * stride + i];
    out[i] = t;
}

struct Layout {
    long oW1, ob1, oW2, ob2, oW3, ob3, total;  // packed FP32 parameters
    long bW1, bW2, bW3, btotal;                // BF16 weight copies
};

// Bias-corrected Adam on the packed FP32 parameters; weights also refresh
// their BF16 copies.
__global__ void adam_kernel(float *w, const float *g, float *m, float *v, long n, float lr, float c1, float c2,
                            Layout L, __bf16 *wb) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = 0.9f * m[i] + 0.1f * gi;
    float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
    w[i] = wi;
    long bi = -1;
    if (i >= L.oW1 && i < L.ob1) bi = L.bW1 + (i - L.oW1);
    else if (i >= L.oW2 && i < L.ob2) bi = L.bW2 + (i - L.oW2);
    else if (i >= L.oW3 && i < L.ob3) bi = L.bW3 + (i - L.oW3);
    if (bi >= 0) wb[bi] = to_bf16(wi);
}

__global__ void refresh_bf16_kernel(const float *w, Layout L, __bf16 *wb) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.total) return;
    long bi = -1;
    if (i >= L.oW1 && i < L.ob1) bi = L.bW1 + (i - L.oW1);
    else if (i >= L.oW2 && i < L.ob2) bi = L.bW2 + (i - L.oW2);
    else if (i >= L.oW3 && i < L.ob3) bi = L.bW3 + (i - L.oW3);
    if (bi >= 0) wb[bi] = to_bf16(w[i]);
}

// s = 1 / sigma (0 for constant features); sigma_out floored at 1e-12 -> 1.
__global__ void set_norm_kernel(const float *mu_in, const float *sd_in, int n_in, const float *mu_out,
                                const float *sd_out, int n_out, float *mu_i, float *s_i, float *mu_o, float *sd_o) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_in) {
        float sd = sd_in[i];
        mu_i[i] = mu_in[i];
        s_i[i] = sd > 1e-12f ? 1.f / sd : 0.f;
    }
    if (i < n_out) {
        float sd = sd_out[i];
        mu_o[i] = mu_out[i];
        sd_o[i] = sd > 1e-12f ? sd : 1.f;
    }
}

inline int pad64(int n) { return (n + 63) / 64 * 64; }

}  // namespace
}  // namespace kamx

using namespace kamx;

struct kamx_mlp_s {
    int n_in = 0, fp = 0, H = 0, n_out = 0, op = 0, cap = 0;
    Layout L{};
    int t = 0;  // Adam steps taken
    float *w = nullptr, *g = nullptr, *am = nullptr, *av = nullptr;
    __bf16 *wb = nullptr;
    float *mu_in = nullptr, *s_in = nullptr, *mu_out = nullptr, *sd_out = nullptr;
    __bf16 *xh = nullptr, *h1 = nullptr, *h2 = nullptr, *dyb = nullptr, *dz2b = nullptr, *dz1b = nullptr;
    float *z1 = nullptr, *z2 = nullptr, *yn = nullptr, *dy = nullptr, *dz2 = nullptr, *dz1 = nullptr;
    float *partial = nullptr;
    float *ws = nullptr;  // partial sums of split weight gradients and bias gradients
    long ws_floats = 0;
    std::vector<void *> allocs;
};

namespace kamx {
// errors of this file go through the library's thread-local message
kamx_status mlp_fail(kamx_status st, const char *fmt, ...);
}  // namespace kamx

#define MLP_HIP(expr)                                                                                 \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) return mlp_fail(KAMX_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
static kamx_status mlp_alloc(kamx_mlp n, T **p, size_t count) {
    void *ptr = nullptr;
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&ptr, bytes);
    if (e != hipSuccess) return mlp_fail(KAMX_ENOMEM, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
    e = hipMemset(ptr, 0, bytes);
    if (e != hipSuccess) return mlp_fail(KAMX_EDEVICE, "hipMemset: %s", hipGetErrorString(e));
    n->allocs.push_back(ptr);
    *p = reinterpret_cast<T *>(ptr);
    return KAMX_OK;
}

static void mlp_free(kamx_mlp n) {
    for (void *p : n->allocs) (void)hipFree(p);
    delete n;
}

// splitmix64 (Steele, Lea and Flood 2014) for the initial weights
static uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

extern "C" kamx_status kamx_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t max_batch, uint64_t seed,
                                       kamx_mlp *out) {
    if (!out) return mlp_fail(KAMX_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_in < 1 || n_in > 65536 || n_out < 1 || n_out > 65536 || n_hidden < 64 || n_hidden > 4096 ||
        n_hidden % 64 != 0 || max_batch < 1 || max_batch > (1 << 22))
        return mlp_fail(KAMX_EINVAL, "bad sizes (n_hidden must be a multiple of 64 in [64, 4096])");
    kamx_mlp n = new kamx_mlp_s;
    n->n_in = n_in;
    n->fp = pad64(n_in);
    n->H = n_hidden;
    n->n_out = n_out;
    n->op = pad64(n_out);
    n->cap = pad64(max_batch);
    Layout &L = n->L;
    const long H = n_hidden, fp = n->fp, op = n->op;
    L.oW1 = 0;
    L.ob1 = L.oW1 + H * fp;
    L.oW2 = L.ob1 + H;
    L.ob2 = L.oW2 + H * H;
    L.oW3 = L.ob2 + H;
    L.ob3 = L.oW3 + op * H;
    L.total = L.ob3 + op;
    L.bW1 = 0;
    L.bW2 = H * fp;
    L.bW3 = L.bW2 + H * H;
    L.btotal = L.bW3 + op * H;
#define C_TRY(expr)                      \
    do {                                 \
        kamx_status s_ = (expr);         \
        if (s_ != KAMX_OK) {             \
            mlp_free(n);                 \
            return s_;                   \
        }                                \
    } while (0)
    C_TRY(mlp_alloc(n, &n->w, L.total));
    C_TRY(mlp_alloc(n, &n->g, L.total));
    C_TRY(mlp_alloc(n, &n->am, L.total));
    C_TRY(mlp_alloc(n, &n->av, L.total));
    C_TRY(mlp_alloc(n, &n->wb, L.btotal));
    C_TRY(mlp_alloc(n, &n->mu_in, fp));
    C_TRY(mlp_alloc(n, &n->s_in, fp));
    C_TRY(mlp_alloc(n, &n->mu_out, op));
    C_TRY(mlp_alloc(n, &n->sd_out, op));
    const long R = n->cap;
    C_TRY(mlp_alloc(n, &n->xh, R * fp));
    C_TRY(mlp_alloc(n, &n->h1, R * H));
    C_TRY(mlp_alloc(n, &n->h2, R * H));
    C_TRY(mlp_alloc(n, &n->dyb, R * op));
    C_TRY(mlp_alloc(n, &n->dz2b, R * H));
    C_TRY(mlp_alloc(n, &n->dz1b, R * H));
    C_TRY(mlp_alloc(n, &n->z1, R * H));
    C_TRY(mlp_alloc(n, &n->z2, R * H));
    C_TRY(mlp_alloc(n, &n->yn, R * op));
    C_TRY(mlp_alloc(n, &n->dy, R * op));
    C_TRY(mlp_alloc(n, &n->dz2, R * H));
    C_TRY(mlp_alloc(n, &n->dz1, R * H));
    C_TRY(mlp_alloc(n, &n->partial, (R * std::max<long>(op, 1) + 255) / 256));
    {
        // split-K weight gradients: each of M x N outputs gets up to
        // grad_splits(...) partials for the padded batch K of a training
        // call (any multiple of 64 up to the capacity: a smaller batch can
        // take more slices than the capacity itself); bias gradients up to
        // kColBlocks
        long most = (long)kColBlocks * std::max(H, op);
        for (long K = 64; K <= R; K += 64) {
            const long a = (long)grad_splits(op, H, (int)K) * op * H, b = (long)grad_splits(H, H, (int)K) * H * H,
                       c = (long)grad_splits(H, fp, (int)K) * H * fp;
            most = std::max(most, std::max(a, std::max(b, c)));
        }
        n->ws_floats = most;
        C_TRY(mlp_alloc(n, &n->ws, n->ws_floats));
    }
    // initial weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)) on the active
    // entries, zero on padding; identity normalisation
    std::vector<float> w(L.total, 0.f), one_in(fp, 1.f), one_out(op, 1.f);
    uint64_t s = seed;
    auto uni = [&](float a) { return a * (2.f * (float)((splitmix(s) >> 40) * (1.0 / 16777216.0)) - 1.f); };
    const float a1 = 1.f / sqrtf((float)n_in), a2 = 1.f / sqrtf((float)H);
    for (long h = 0; h < H; ++h)
        for (long i = 0; i < n_in; ++i) w[L.oW1 + h * fp + i] = uni(a1);
    for (long h = 0; h < H; ++h) w[L.ob1 + h] = uni(a1);
    for (long h = 0; h < H * H; ++h) w[L.oW2 + h] = uni(a2);
    for (long h = 0; h < H; ++h) w[L.ob2 + h] = uni(a2);
    for (long o = 0; o < n_out; ++o)
        for (long h = 0; h < H; ++h) w[L.oW3 + o * H + h] = uni(a2);
    for (long o = 0; o < n_out; ++o) w[L.ob3 + o] = uni(a2);
    hipError_t e = hipMemcpy(n->w, w.data(), sizeof(float) * L.total, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(n->s_in, one_in.data(), sizeof(float) * fp, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(n->sd_out, one_out.data(), sizeof(float) * op, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        mlp_free(n);
        return mlp_fail(KAMX_EDEVICE, "weight upload: %s", hipGetErrorString(e));
    }
    hipLaunchKernelGGL(refresh_bf16_kernel, dim3((unsigned)((L.total + 255) / 256)), dim3(256), 0, 0, n->w, L, n->wb);
    e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        mlp_free(n);
        return mlp_fail(KAMX_EDEVICE, "weight conversion: %s", hipGetErrorString(e));
    }
#undef C_TRY
    *out = n;
    return KAMX_OK;
}

extern "C" kamx_status kamx_mlp_destroy(kamx_mlp n) {
    if (!n) return KAMX_OK;
    (void)hipDeviceSynchronize();
    mlp_free(n);
    return KAMX_OK;
}

extern "C" kamx_status kamx_mlp_info(kamx_mlp n, int32_t *n_in_pad, int32_t *n_out_pad, int64_t *n_params) {
    if (!n) return mlp_fail(KAMX_EINVAL, "network is NULL");
    if (n_in_pad) *n_in_pad = n->fp;
    if (n_out_pad) *n_out_pad = n->op;
    if (n_params) *n_params = n->L.total;
    return KAMX_OK;
}

extern "C" kamx_status kamx_mlp_set_normalization(kamx_mlp n, const float *mu_in, const float *sigma_in,
                                                  const float *mu_out, const float *sigma_out, kamx_stream stream) {
    if (!n || !mu_in || !sigma_in || !mu_out || !sigma_out) return mlp_fail(KAMX_EINVAL, "NULL argument");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int m = std::max(n->n_in, n->n_out);
    hipLaunchKernelGGL(set_norm_kernel, dim3((m + 255) / 256), dim3(256), 0, s, mu_in, sigma_in, n->n_in, mu_out,
                       sigma_out, n->n_out, n->mu_in, n->s_in, n->mu_out, n->sd_out);
    MLP_HIP(hipGetLastError());
    return KAMX_OK;
}

template <int EPI>
static hipError_t gemm(const Operand &A, const Operand &B, int M, int N, int K, const EpiArgs &e, hipStream_t s) {
    if (M % kTileM || N % kTileN || K % kTileK || M <= 0 || N <= 0 || K <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gemm_kernel<EPI>, dim3(N / kTileN, M / kTileM), dim3(kGemmThreads), 0, s, A, B, M, N, K, e);
    return hipGetLastError();
}

// C = A B^T summed over K into c (ldc = N), split over K with the partial
// results reduced in slice order
static hipError_t gemm_store(kamx_mlp n, const Operand &A, const Operand &B, int M, int N, int K, float *c,
                             hipStream_t s) {
    if (M % kTileM || N % kTileN || K % kTileK || M <= 0 || N <= 0 || K <= 0) return hipErrorInvalidValue;
    const int ns = grad_splits(M, N, K);
    if ((long)ns * M * N > n->ws_floats) return hipErrorInvalidValue;
    EpiArgs e{};
    e.f32 = ns > 1 ? n->ws : c;
    e.ld = N;
    e.split = (long)M * N;
    hipLaunchKernelGGL(gemm_kernel<kEpiStore>, dim3(N / kTileN, M / kTileM, ns), dim3(kGemmThreads), 0, s, A, B, M,
                       N, K, e);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess || ns == 1) return err;
    const long cnt = (long)M * N;
    hipLaunchKernelGGL(sum_slices_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, n->ws, cnt, ns, cnt,
                       c);
    return hipGetLastError();
}

// bias gradient: column sums of a [rows, cols] matrix
static hipError_t colsum(kamx_mlp n, const float *a, int rows, int cols, float *out, hipStream_t s) {
    int nb = kColBlocks;
    while (nb > 1 && rows % nb) nb >>= 1;
    hipLaunchKernelGGL(colsum_partial_kernel, dim3((cols + 63) / 64, nb), dim3(256), 0, s, a, rows, cols, n->ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_slices_kernel, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, s, n->ws, (long)cols, nb,
                       (long)cols, out);
    return hipGetLastError();
}

// Activations of one forward pass: the normalised BF16 input, the two
// BF16 hidden activations and, for training, the FP32 pre-activations and
// normalised outputs (null when only the prediction is wanted).
struct Acts {
    __bf16 *xh, *h1, *h2;
    float *z1, *z2, *yn;
};

// forward over rows padded to a multiple of 64; y (optional) receives the
// de-standardised outputs of the first batch rows
static kamx_status mlp_forward_rows(kamx_mlp n, const Acts &a, const float *x, long ldx, int batch, float *y,
                                    long ldy, hipStream_t s) {
    const int R = pad64(batch), H = n->H, fp = n->fp, op = n->op;
    const Layout &L = n->L;
    long cnt = (long)R * fp;
    hipLaunchKernelGGL(normalise_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, x, ldx, batch, n->n_in,
                       n->mu_in, n->s_in, a.xh, R, fp);
    MLP_HIP(hipGetLastError());
    EpiArgs e{};
    e.bias = n->w + L.ob1;
    e.f32 = a.z1;
    e.b16 = a.h1;
    e.ld = H;
    MLP_HIP((gemm<kEpiHidden>(Operand{a.xh, fp, 1}, Operand{n->wb + L.bW1, fp, 1}, R, H, fp, e, s)));
    e.bias = n->w + L.ob2;
    e.f32 = a.z2;
    e.b16 = a.h2;
    MLP_HIP((gemm<kEpiHidden>(Operand{a.h1, H, 1}, Operand{n->wb + L.bW2, H, 1}, R, H, H, e, s)));
    EpiArgs o{};
    o.bias = n->w + L.ob3;
    o.f32 = a.yn;
    o.ld = op;
    o.y = y;
    o.ldy = ldy;
    o.batch = batch;
    o.n_out = n->n_out;
    o.mu = n->mu_out;
    o.sigma = n->sd_out;
    MLP_HIP((gemm<kEpiOut>(Operand{a.h2, H, 1}, Operand{n->wb + L.bW3, H, 1}, R, op, H, o, s)));
    return KAMX_OK;
}

static Acts own_acts(kamx_mlp n, bool keep) {
    Acts a{n->xh, n->h1, n->h2, nullptr, nullptr, nullptr};
    if (keep) {
        a.z1 = n->z1;
        a.z2 = n->z2;
        a.yn = n->yn;
    }
    return a;
}

namespace kamx {
// used by the model's learned warm start
kamx_status mlp_forward_internal(kamx_mlp n, const float *x, int batch, float *y, hipStream_t s) {
    if (batch > n->cap) return mlp_fail(KAMX_EINVAL, "batch %d above the network's capacity %d", batch, n->cap);
    return mlp_forward_rows(n, own_acts(n, false), x, n->n_in, batch, y, n->n_out, s);
}
int mlp_n_in(kamx_mlp n) { return n->n_in; }
MlpView mlp_view(kamx_mlp n) {
    MlpView v;
    v.w1 = n->wb + n->L.bW1;
    v.w2 = n->wb + n->L.bW2;
    v.w3 = n->wb + n->L.bW3;
    v.b1 = n->w + n->L.ob1;
    v.b2 = n->w + n->L.ob2;
    v.b3 = n->w + n->L.ob3;
    v.mu_in = n->mu_in;
    v.s_in = n->s_in;
    v.mu_out = n->mu_out;
    v.sd_out = n->sd_out;
    v.n_in = n->n_in;
    v.fp = n->fp;
    v.H = n->H;
    v.n_out = n->n_out;
    v.op = n->op;
    return v;
}
int mlp_n_out(kamx_mlp n) { return n->n_out; }
int mlp_capacity(kamx_mlp n) { return n->cap; }
}  // namespace kamx

extern "C" kamx_status kamx_mlp_forward(kamx_mlp n, const float *x, int32_t batch, float *y, kamx_stream stream) {
    if (!n || !x || !y) return mlp_fail(KAMX_EINVAL, "NULL argument");
    if (batch < 1 || batch > n->cap) return mlp_fail(KAMX_EINVAL, "batch must be in [1, %d]", n->cap);
    return mlp_forward_rows(n, own_acts(n, false), x, n->n_in, batch, y, n->n_out,
                            reinterpret_cast<hipStream_t>(stream));
}

// ---- forward pass without allocation -------------------------------------
// The activations of kamx_mlp_forward_noalloc live in this fixed array: each
// GPU the library runs on holds its own copy until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kNoallocScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// device address of this GPU's scratch array (looked up once per device)
kamx_status scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return mlp_fail(KAMX_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return mlp_fail(KAMX_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return mlp_fail(KAMX_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return KAMX_OK;
}
}  // namespace

extern "C" kamx_status kamx_mlp_forward_noalloc(kamx_mlp n, const float *x, int32_t batch, float *y,
                                                kamx_stream stream) {
    if (!n || !x || !y) return mlp_fail(KAMX_EINVAL, "NULL argument");
    if (batch < 1 || batch > (1 << 24)) return mlp_fail(KAMX_EINVAL, "batch must be in [1, 2^24]");
    const size_t per_row = sizeof(__bf16) * ((size_t)n->fp + 2 * (size_t)n->H);
    const size_t rows_max = (kNoallocScratchBytes / per_row) / 64 * 64;
    if ((size_t)pad64(batch) > rows_max)
        return mlp_fail(KAMX_EINVAL, "batch %d above the %zu rows the fixed %zu-byte workspace holds for this network",
                        batch, rows_max, kNoallocScratchBytes);
    void *base = nullptr;
    kamx_status st = scratch_address(&base);
    if (st != KAMX_OK) return st;
    // every activation is written before it is read (padded rows included),
    // so nothing in the array has to start at zero
    const long R = pad64(batch);
    Acts a{};
    a.xh = reinterpret_cast<__bf16 *>(base);
    a.h1 = a.xh + R * n->fp;
    a.h2 = a.h1 + R * n->H;
    return mlp_forward_rows(n, a, x, n->n_in, batch, y, n->n_out, reinterpret_cast<hipStream_t>(stream));
}

extern "C" kamx_status kamx_mlp_train_step(kamx_mlp n, const float *x, const float *y_target, int32_t batch, float lr,
                                           float *loss_dev, kamx_stream stream) {
    if (!n || !x || !y_target) return mlp_fail(KAMX_EINVAL, "NULL argument");
    if (batch < 1 || batch > n->cap) return mlp_fail(KAMX_EINVAL, "batch must be in [1, %d]", n->cap);
    if (!(lr >= 0.f)) return mlp_fail(KAMX_EINVAL, "lr must be >= 0");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int R = pad64(batch), H = n->H, fp = n->fp, op = n->op;
    const Layout &L = n->L;
    kamx_status st = mlp_forward_rows(n, own_acts(n, true), x, n->n_in, batch, nullptr, 0, s);
    if (st != KAMX_OK) return st;
    const long cnt = (long)R * op;
    const int blocks = (int)((cnt + 255) / 256);
    hipLaunchKernelGGL(loss_grad_kernel, dim3(blocks), dim3(256), 0, s, n->yn, y_target, batch, n->n_out, op,
                       n->mu_out, n->sd_out, n->dy, n->dyb, R, n->partial);
    MLP_HIP(hipGetLastError());
    if (loss_dev) {
        hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, s, n->partial, blocks,
                           1.f / ((float)batch * (float)n->n_out), loss_dev);
        MLP_HIP(hipGetLastError());
    }
    EpiArgs e{};
    // layer 3: dW3 = dy^T h2, db3 = sum dy, dz2 = (dy W3) gelu'(z2)
    MLP_HIP(gemm_store(n, Operand{n->dyb, 1, op}, Operand{n->h2, 1, H}, op, H, R, n->g + L.oW3, s));
    MLP_HIP(colsum(n, n->dy, R, op, n->g + L.ob3, s));
    e = EpiArgs{};
    e.z = n->z2;
    e.f32 = n->dz2;
    e.b16 = n->dz2b;
    e.ld = H;
    MLP_HIP((gemm<kEpiBackward>(Operand{n->dyb, op, 1}, Operand{n->wb + L.bW3, 1, H}, R, H, op, e, s)));
    // layer 2
    MLP_HIP(gemm_store(n, Operand{n->dz2b, 1, H}, Operand{n->h1, 1, H}, H, H, R, n->g + L.oW2, s));
    MLP_HIP(colsum(n, n->dz2, R, H, n->g + L.ob2, s));
    e = EpiArgs{};
    e.z = n->z1;
    e.f32 = n->dz1;
    e.b16 = n->dz1b;
    e.ld = H;
    MLP_HIP((gemm<kEpiBackward>(Operand{n->dz2b, H, 1}, Operand{n->wb + L.bW2, 1, H}, R, H, H, e, s)));
    // layer 1
    MLP_HIP(gemm_store(n, Operand{n->dz1b, 1, H}, Operand{n->xh, 1, fp}, H, fp, R, n->g + L.oW1, s));
    MLP_HIP(colsum(n, n->dz1, R, H, n->g + L.ob1, s));
    // Adam
    n->t += 1;
    const float c1 = (float)(1.0 - pow(0.9, n->t)), c2 = (float)(1.0 - pow(0.999, n->t));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((L.total + 255) / 256)), dim3(256), 0, s, n->w, n->g, n->am,
                       n->av, L.total, lr, c1, c2, L, n->wb);
    MLP_HIP(hipGetLastError());
    return KAMX_OK;
}

extern "C" kamx_status kamx_mlp_weights(kamx_mlp n, float *buf, int32_t set, kamx_stream stream) {
    if (!n || !buf) return mlp_fail(KAMX_EINVAL, "NULL argument");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Layout &L = n->L;
    if (set) {
        MLP_HIP(hipMemcpyAsync(n->w, buf, sizeof(float) * L.total, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(refresh_bf16_kernel, dim3((unsigned)((L.total + 255) / 256)), dim3(256), 0, s, n->w, L,
                           n->wb);
        MLP_HIP(hipGetLastError());
        MLP_HIP(hipMemsetAsync(n->am, 0, sizeof(float) * L.total, s));
        MLP_HIP(hipMemsetAsync(n->av, 0, sizeof(float) * L.total, s));
        n->t = 0;
    } else {
        MLP_HIP(hipMemcpyAsync(buf, n->w, sizeof(float) * L.total, hipMemcpyDeviceToDevice, s));
    }
    return KAMX_OK;
}

extern "C" kamx_status kamx_mlp_gradients(kamx_mlp n, float *buf, kamx_stream stream) {
    if (!n || !buf) return mlp_fail(KAMX_EINVAL, "NULL argument");
    MLP_HIP(hipMemcpyAsync(buf, n->g, sizeof(float) * n->L.total, hipMemcpyDeviceToDevice,
                           reinterpret_cast<hipStream_t>(stream)));
    return KAMX_OK;
}
