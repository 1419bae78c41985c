// The surrogate network: a multilayer perceptron n_in -> width (depth hidden
// layers, exact GELU) -> n_out, trained by mean squared error with Adam.
//
// Matrix products run on the bf16 matrix cores with FP32 accumulation
// (v_mfma_f32_16x16x32_bf16): every layer input, weight and back-propagated
// gradient enters a product rounded to bf16; biases, pre-activations,
// gradients, the loss and the Adam state are FP32, and the FP32 master
// weights are what Adam updates (their bf16 copies are refreshed after each
// step).  The input layer, with at most kFp32In inputs, is no matrix product
// worth the matrix cores and runs in FP32 on the vector units: its inputs are
// the network's coordinates (time and parameters), whose bf16 rounding would
// cost 2^-9 of their range.  One strided GEMM kernel serves the forward product, the weight
// gradient (reduction over the batch, split over workgroups and summed in a
// fixed order) and the input gradient.
//
// Parameters, flat FP32: for each layer l, W_l [fan_in][fan_out] row-major,
// then b_l [fan_out].

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "../../include/quapi.h"
#include "../../include/quapi_mlp.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kGemmThreads = 256;             // 4 waves
constexpr int kTM = 64, kTN = 64, kTK = 32;   // workgroup tile; one MFMA's k per step
constexpr int kLdsK = kTK + 8;                // row pitch of the LDS tiles (bf16), breaks bank strides
constexpr int kVecThreads = 256;
constexpr int kMaxSplit = 64;
constexpr int kFp32In = 16;                   // input layers this narrow run in FP32

enum Epilogue : int {
    kStoreF32 = 0,     // outf = acc (+ bias)
    kGelu = 1,         // outf = acc + bias; outb = bf16(gelu(acc + bias))
    kGeluGrad = 2,     // outf = acc * gelu'(zprev); outb = bf16(outf)
};

__device__ __host__ inline uint16_t to_bf16(float f) {
    // round to nearest even (finite inputs)
    uint32_t u;
#ifdef __HIP_DEVICE_COMPILE__
    u = __builtin_bit_cast(uint32_t, f);
#else
    std::memcpy(&u, &f, 4);
#endif
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

__device__ inline float gelu_grad(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

struct GemmArgs {
    const uint16_t* A;            // A(m, k) = A[m * sam + k * sak]
    long long sam, sak;
    const uint16_t* B;            // B(k, n) = B[k * sbk + n * sbn]
    long long sbk, sbn;
    int M, N, K;
    int kslice;                   // reduction range of workgroup z: [z * kslice, min(K, (z + 1) * kslice))
    int epi;
    const float* bias;            // [N] or null
    const float* zprev;           // kGeluGrad: [M][N] pre-activations of the layer below
    float* outf;                  // [M][N] (+ z * M * N for split partials)
    uint16_t* outb;               // [M][N] or null
};

// One operand's 64 x 32 tile into the LDS as T[row][k] (row = m of A, n of
// B): element (row, k) of the operand is X[row * s_row + k * s_k].
__device__ inline void stage_tile(const uint16_t* X, long long s_row, long long s_k, int rows, int r0, int k0,
                                  int k_hi, int i, uint16_t (*T)[kLdsK]) {
    if (s_k == 1) {
        // 8 consecutive k of one row
        const int r = i >> 2, kq = (i & 3) * 8;
        const int row = r0 + r, k = k0 + kq;
        const long long o = (long long)row * s_row + k;
        if (row < rows && k + 8 <= k_hi && (o & 7) == 0) {
            *reinterpret_cast<uint4*>(&T[r][kq]) = *reinterpret_cast<const uint4*>(X + o);
            return;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
            T[r][kq + j] = (row < rows && k + j < k_hi) ? X[o + j] : (uint16_t)0;
        return;
    }
    if (s_row == 1) {
        // 8 consecutive rows at one k
        const int kk = i >> 3, rq = (i & 7) * 8;
        const int row = r0 + rq, k = k0 + kk;
        const long long o = (long long)k * s_k + row;
        if (k < k_hi && row + 8 <= rows && (o & 7) == 0) {
            const uint4 v = *reinterpret_cast<const uint4*>(X + o);
            const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
            for (int j = 0; j < 8; ++j) T[rq + j][kk] = e[j];
            return;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
            T[rq + j][kk] = (k < k_hi && row + j < rows) ? X[o + j] : (uint16_t)0;
        return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int idx = e * kGemmThreads + i;
        const int r = idx / kTK, kk = idx % kTK;
        const int row = r0 + r, k = k0 + kk;
        T[r][kk] = (row < rows && k < k_hi) ? X[(long long)row * s_row + (long long)k * s_k] : (uint16_t)0;
    }
}

// C = A B over one 64 x 64 tile; waves (wr, wc) take 32 x 32 quarters as 2 x 2
// MFMA tiles of 16 x 16.  MFMA operands: lane l holds row l % 16 of A and
// column l % 16 of B at k = (l / 16) * 8 .. + 8; the result holds rows
// (l / 16) * 4 .. + 4 of column l % 16.
__global__ __launch_bounds__(kGemmThreads) void gemm_bf16(const GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kTM][kLdsK];   // [m][k]
    __shared__ __attribute__((aligned(16))) uint16_t Bt[kTN][kLdsK];   // [n][k]
    const int i = threadIdx.x;
    const int wave = i >> 6, lane = i & 63;
    const int wr = wave >> 1, wc = wave & 1;
    const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
    const int k_lo = blockIdx.z * g.kslice;
    const int k_hi = min(g.K, k_lo + g.kslice);

    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    for (int k0 = k_lo; k0 < k_hi; k0 += kTK) {
        __syncthreads();
        // stage 64 x 32 of A and 32 x 64 of B, 8 elements per thread each: one
        // 16-byte load along the operand's contiguous dimension where the 8 lie
        // inside it and aligned, else element by element (zero outside)
        stage_tile(g.A, g.sam, g.sak, g.M, m0, k0, k_hi, i, As);
        stage_tile(g.B, g.sbn, g.sbk, g.N, n0, k0, k_hi, i, Bt);
        __syncthreads();
        bf16x8 af[2], bfr[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            af[t] = *reinterpret_cast<const bf16x8*>(&As[wr * 32 + t * 16 + (lane & 15)][(lane >> 4) * 8]);
            bfr[t] = *reinterpret_cast<const bf16x8*>(&Bt[wc * 32 + t * 16 + (lane & 15)][(lane >> 4) * 8]);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
    }

    float* const outf = g.outf + (size_t)blockIdx.z * g.M * g.N;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = m0 + wr * 32 + a * 16 + (lane >> 4) * 4 + v;
                const int n = n0 + wc * 32 + b * 16 + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                const size_t o = (size_t)m * g.N + n;
                float x = acc[a][b][v];
                if (g.bias) x += g.bias[n];
                if (g.epi == kGeluGrad) x *= gelu_grad(g.zprev[o]);
                outf[o] = x;
                if (g.epi == kGelu) g.outb[o] = to_bf16(gelu(x));
                else if (g.epi == kGeluGrad) g.outb[o] = to_bf16(x);
            }
}

// FP32 input layer: z[m][n] = b[n] + sum_k x[m][k] W[k][n]; a = bf16(gelu(z))
// (or z alone for a network without hidden layers)
__global__ void dense_in(const float* x, const float* W, const float* b, int M, int K, int N, float* z, uint16_t* a) {
    const long long idx = (long long)blockIdx.x * kVecThreads + threadIdx.x;
    if (idx >= (long long)M * N) return;
    const int m = (int)(idx / N), n = (int)(idx % N);
    float s = b[n];
    for (int k = 0; k < K; ++k) s = fmaf(x[(size_t)m * K + k], W[(size_t)k * N + n], s);
    z[idx] = s;
    if (a) a[idx] = to_bf16(gelu(s));
}

// its weight gradient, split over the batch: partial[z][k][n] = sum over the
// rows m of split z of x[m][k] dz[m][n].  Lanes take 64 columns n; the four
// waves take every fourth row of the split and add up in the LDS in wave order.
__global__ __launch_bounds__(kVecThreads) void dense_in_grad(const float* x, const float* dz, int M, int K, int N,
                                                              int rows, float* partial) {
    __shared__ float red[kVecThreads / 64][kFp32In][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = blockIdx.x * 64 + lane;
    const int m0 = blockIdx.y * rows, m1 = min(M, m0 + rows);
    float acc[kFp32In];
#pragma unroll
    for (int k = 0; k < kFp32In; ++k) acc[k] = 0.0f;
    if (n < N)
        for (int m = m0 + wave; m < m1; m += kVecThreads / 64) {
            const float d = dz[(size_t)m * N + n];
#pragma unroll
            for (int k = 0; k < kFp32In; ++k)
                if (k < K) acc[k] = fmaf(x[(size_t)m * K + k], d, acc[k]);
        }
#pragma unroll
    for (int k = 0; k < kFp32In; ++k) red[wave][k][lane] = acc[k];
    __syncthreads();
    if (wave == 0 && n < N)
        for (int k = 0; k < K; ++k) {
            float t = 0.0f;
            for (int w = 0; w < kVecThreads / 64; ++w) t += red[w][k][lane];
            partial[(size_t)blockIdx.y * K * N + (size_t)k * N + n] = t;
        }
}

__global__ void to_bf16_kernel(const float* x, uint16_t* y, long long n) {
    for (long long k = (long long)blockIdx.x * kVecThreads + threadIdx.x; k < n; k += (long long)gridDim.x * kVecThreads)
        y[k] = to_bf16(x[k]);
}

// Loss gradient dY = 2 (Y - T) / (B n_out) as FP32 and bf16, and per-workgroup
// partial sums of (Y - T)^2 (summed in workgroup order by loss_sum).
__global__ void loss_grad(const float* y, const float* t, long long n, float scale, float* dyf, uint16_t* dyb,
                          float* partial) {
    __shared__ float red[kVecThreads];
    float s = 0.0f;
    for (long long k = (long long)blockIdx.x * kVecThreads + threadIdx.x; k < n; k += (long long)gridDim.x * kVecThreads) {
        const float d = y[k] - t[k];
        s += d * d;
        const float gk = 2.0f * d * scale;
        dyf[k] = gk;
        dyb[k] = to_bf16(gk);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kVecThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void loss_sum(const float* partial, int n, float scale, float* loss) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float s = 0.0f;
        for (int k = 0; k < n; ++k) s += partial[k];
        *loss = s * scale;
    }
}

// grad[k] = sum over splits of partial[z][k], in split order
__global__ void sum_splits(const float* partial, int splits, long long n, float* grad) {
    for (long long k = (long long)blockIdx.x * kVecThreads + threadIdx.x; k < n; k += (long long)gridDim.x * kVecThreads) {
        float s = 0.0f;
        for (int z = 0; z < splits; ++z) s += partial[(size_t)z * n + k];
        grad[k] = s;
    }
}

// bias gradient, split over the batch: partial[z][c] = sum over the rows of
// split z of dZ[r][c] (summed over the splits in order by sum_splits).  Lanes
// take 64 columns; the four waves take every fourth row and add up in wave order.
__global__ __launch_bounds__(kVecThreads) void column_sums(const float* dz, int rows, int cols, int per,
                                                            float* partial) {
    __shared__ float red[kVecThreads / 64][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = blockIdx.x * 64 + lane;
    const int r0 = blockIdx.y * per, r1 = min(rows, r0 + per);
    float s = 0.0f;
    if (c < cols)
        for (int r = r0 + wave; r < r1; r += kVecThreads / 64) s += dz[(size_t)r * cols + c];
    red[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && c < cols) {
        float t = 0.0f;
        for (int w = 0; w < kVecThreads / 64; ++w) t += red[w][lane];
        partial[(size_t)blockIdx.y * cols + c] = t;
    }
}

// Adam (Kingma & Ba 2015) on the flat FP32 parameters; bias-corrected step sizes
// come in as arguments
__global__ void adam_kernel(float* w, float* m, float* v, const float* grad, long long n, float lr_t, float b1,
                            float b2, float eps_t) {
    for (long long k = (long long)blockIdx.x * kVecThreads + threadIdx.x; k < n; k += (long long)gridDim.x * kVecThreads) {
        const float gk = grad[k];
        const float mk = b1 * m[k] + (1.0f - b1) * gk;
        const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
        m[k] = mk;
        v[k] = vk;
        w[k] -= lr_t * mk / (sqrtf(vk) + eps_t);
    }
}

int blocks_for(long long n) { return (int)std::min<long long>((n + kVecThreads - 1) / kVecThreads, 2048); }

constexpr int kBiasRows = 256;  // rows per split of the bias gradient

}  // namespace

struct quapi_mlp {
    int n_in = 0, width = 0, depth = 0, n_out = 0, max_batch = 0;
    int n_layers = 0;
    std::vector<int> fin, fout;          // per layer
    std::vector<long long> w_off, b_off; // offsets in the flat parameters
    long long n_params = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    float *w = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    std::vector<uint16_t*> wb;           // bf16 weight copies per layer
    uint16_t* xb = nullptr;              // bf16 network input [max_batch][n_in]
    std::vector<float*> z;               // pre-activations per layer [max_batch][fout]
    std::vector<uint16_t*> ab;           // bf16 activations per hidden layer
    float* dzf = nullptr;                // FP32 gradient of a layer's pre-activation [max_batch][max width]
    float* dzf2 = nullptr;
    uint16_t* dzb = nullptr;             // its bf16 copy
    uint16_t* dzb2 = nullptr;
    float* partial = nullptr;            // split-reduction partials
    float* loss_part = nullptr;
    float* xf = nullptr;                 // FP32 network input [max_batch][n_in] (FP32 input layer)
    float* bias_part = nullptr;          // bias-gradient partials [<= 4096 splits][max width]
    bool fp32_in = false;
    int adam_t = 0;
    std::vector<void*> allocs;
};

namespace {

template <class T>
int mlp_alloc(quapi_mlp* c, T** p, size_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, (n ? n : 1) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return QUAPI_ENOMEM;
    }
    c->allocs.push_back(q);
    *p = (T*)q;
    return QUAPI_OK;
}

int launch_gemm(quapi_mlp* c, const GemmArgs& g, int splits) {
    dim3 grid((g.N + kTN - 1) / kTN, (g.M + kTM - 1) / kTM, splits);
    hipLaunchKernelGGL(gemm_bf16, grid, dim3(kGemmThreads), 0, c->stream, g);
    return hipGetLastError() == hipSuccess ? QUAPI_OK : QUAPI_EDEVICE;
}

int refresh_bf16(quapi_mlp* c) {
    for (int l = 0; l < c->n_layers; ++l) {
        const long long n = (long long)c->fin[l] * c->fout[l];
        hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(n)), dim3(kVecThreads), 0, c->stream, c->w + c->w_off[l],
                           c->wb[l], n);
    }
    return hipGetLastError() == hipSuccess ? QUAPI_OK : QUAPI_EDEVICE;
}

// forward of a batch already in c->xb (and c->xf); the output pre-activations land in z[last]
int forward(quapi_mlp* c, int batch) {
    for (int l = 0; l < c->n_layers; ++l) {
        const bool last = l == c->n_layers - 1;
        if (l == 0 && c->fp32_in) {
            const long long n = (long long)batch * c->fout[0];
            hipLaunchKernelGGL(dense_in, dim3((unsigned)((n + kVecThreads - 1) / kVecThreads)), dim3(kVecThreads), 0,
                               c->stream, c->xf, c->w + c->w_off[0], c->w + c->b_off[0], batch, c->fin[0],
                               c->fout[0], c->z[0], last ? nullptr : c->ab[0]);
            continue;
        }
        GemmArgs g{};
        g.A = l == 0 ? c->xb : c->ab[l - 1];
        g.sam = c->fin[l];
        g.sak = 1;
        g.B = c->wb[l];
        g.sbk = c->fout[l];
        g.sbn = 1;
        g.M = batch;
        g.N = c->fout[l];
        g.K = c->fin[l];
        g.kslice = g.K;
        g.epi = last ? kStoreF32 : kGelu;
        g.bias = c->w + c->b_off[l];
        g.outf = c->z[l];
        g.outb = last ? nullptr : c->ab[l];
        if (launch_gemm(c, g, 1)) return QUAPI_EDEVICE;
    }
    return QUAPI_OK;
}

int check_batch(quapi_mlp* c, int batch) { return (batch < 1 || batch > c->max_batch) ? QUAPI_EINVAL : QUAPI_OK; }

// bias gradient: column sums of dz [batch][cols] over splits of at least
// kBiasRows rows (at most 4096 splits), then summed over the splits in order
int bias_grad(quapi_mlp* c, const float* dz, int batch, int cols, float* out) {
    const int per = std::max(kBiasRows, (batch + 4095) / 4096);
    const int splits = (batch + per - 1) / per;
    float* part = c->bias_part;
    hipLaunchKernelGGL(column_sums, dim3((cols + 63) / 64, splits), dim3(kVecThreads), 0, c->stream, dz, batch, cols,
                       per, part);
    hipLaunchKernelGGL(sum_splits, dim3(blocks_for(cols)), dim3(kVecThreads), 0, c->stream, part, splits,
                       (long long)cols, out);
    return hipGetLastError() == hipSuccess ? QUAPI_OK : QUAPI_EDEVICE;
}

// the network input as the first layer reads it: FP32 copy, or bf16
int stage_input(quapi_mlp* c, const float* x, int batch) {
    const long long nx = (long long)batch * c->n_in;
    if (c->fp32_in) {
        if (hipMemcpyAsync(c->xf, x, (size_t)nx * sizeof(float), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
            return QUAPI_EDEVICE;
    } else {
        hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(nx)), dim3(kVecThreads), 0, c->stream, x, c->xb, nx);
    }
    return hipGetLastError() == hipSuccess ? QUAPI_OK : QUAPI_EDEVICE;
}

}  // namespace

extern "C" {

int quapi_mlp_create(int n_in, int width, int depth, int n_out, int max_batch, unsigned long long seed,
                     void* stream, quapi_mlp** out) {
    if (!out) return QUAPI_EINVAL;
    *out = nullptr;
    if (n_in < 1 || width < 1 || depth < 1 || n_out < 1 || max_batch < 1 || n_in > 4096 || width > 4096 ||
        n_out > 4096 || depth > 64 || max_batch > (1 << 22))
        return QUAPI_EINVAL;
    quapi_mlp* c = new (std::nothrow) quapi_mlp();
    if (!c) return QUAPI_ENOMEM;
    c->n_in = n_in;
    c->width = width;
    c->depth = depth;
    c->n_out = n_out;
    c->max_batch = max_batch;
    c->n_layers = depth + 1;
    for (int l = 0; l < c->n_layers; ++l) {
        c->fin.push_back(l == 0 ? n_in : width);
        c->fout.push_back(l == depth ? n_out : width);
        c->w_off.push_back(c->n_params);
        c->n_params += (long long)c->fin[l] * c->fout[l];
        c->b_off.push_back(c->n_params);
        c->n_params += c->fout[l];
    }
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return QUAPI_EDEVICE;
        }
        c->own_stream = true;
    }
    const int wmax = std::max(width, n_out);
    int rc = mlp_alloc(c, &c->w, c->n_params);
    if (!rc) rc = mlp_alloc(c, &c->grad, c->n_params);
    if (!rc) rc = mlp_alloc(c, &c->m, c->n_params);
    if (!rc) rc = mlp_alloc(c, &c->v, c->n_params);
    if (!rc) rc = mlp_alloc(c, &c->xb, (size_t)max_batch * n_in);
    c->fp32_in = n_in <= kFp32In;
    if (!rc && c->fp32_in) rc = mlp_alloc(c, &c->xf, (size_t)max_batch * n_in);
    c->wb.assign(c->n_layers, nullptr);
    c->z.assign(c->n_layers, nullptr);
    c->ab.assign(depth, nullptr);
    for (int l = 0; l < c->n_layers && !rc; ++l) {
        rc = mlp_alloc(c, &c->wb[l], (size_t)c->fin[l] * c->fout[l]);
        if (!rc) rc = mlp_alloc(c, &c->z[l], (size_t)max_batch * c->fout[l]);
        if (!rc && l < depth) rc = mlp_alloc(c, &c->ab[l], (size_t)max_batch * c->fout[l]);
    }
    if (!rc) rc = mlp_alloc(c, &c->dzf, (size_t)max_batch * wmax);
    if (!rc) rc = mlp_alloc(c, &c->dzf2, (size_t)max_batch * wmax);
    if (!rc) rc = mlp_alloc(c, &c->dzb, (size_t)max_batch * wmax);
    if (!rc) rc = mlp_alloc(c, &c->dzb2, (size_t)max_batch * wmax);
    const long long wmax_params = (long long)std::max(n_in, width) * wmax;
    if (!rc) rc = mlp_alloc(c, &c->partial, (size_t)kMaxSplit * wmax_params);
    if (!rc) rc = mlp_alloc(c, &c->loss_part, 2048);
    if (!rc) rc = mlp_alloc(c, &c->bias_part, (size_t)std::min(max_batch / kBiasRows + 1, 4096) * wmax);
    if (rc) {
        quapi_mlp_destroy(c);
        return rc;
    }
    // initial weights and biases uniform in +-1/sqrt(fan_in), from the SplitMix64
    // sequence of the seed (Steele, Lea, Flood 2014)
    std::vector<float> h((size_t)c->n_params);
    unsigned long long st = seed;
    auto next = [&st]() {
        unsigned long long z = (st += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    };
    for (int l = 0; l < c->n_layers; ++l) {
        const float s = 1.0f / std::sqrt((float)c->fin[l]);
        const long long n = (long long)c->fin[l] * c->fout[l] + c->fout[l];
        for (long long k = 0; k < n; ++k)
            h[c->w_off[l] + k] = s * (2.0f * (float)((next() >> 11) * (1.0 / 9007199254740992.0)) - 1.0f);
    }
    rc = quapi_mlp_set_params(c, h.data(), c->n_params);
    if (rc) {
        quapi_mlp_destroy(c);
        return rc;
    }
    *out = c;
    return QUAPI_OK;
}

int quapi_mlp_n_params(quapi_mlp* c, long long* n) {
    if (!c || !n) return QUAPI_EINVAL;
    *n = c->n_params;
    return QUAPI_OK;
}

int quapi_mlp_set_params(quapi_mlp* c, const float* host, long long n) {
    if (!c || !host || n != c->n_params) return QUAPI_EINVAL;
    hipError_t e = hipMemcpyAsync(c->w, host, (size_t)n * sizeof(float), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->m, 0, (size_t)n * sizeof(float), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->v, 0, (size_t)n * sizeof(float), c->stream);
    if (e != hipSuccess) return QUAPI_EDEVICE;
    c->adam_t = 0;
    if (refresh_bf16(c)) return QUAPI_EDEVICE;
    return hipStreamSynchronize(c->stream) == hipSuccess ? QUAPI_OK : QUAPI_EDEVICE;
}

int quapi_mlp_get_params(quapi_mlp* c, float* host, long long n) {
    if (!c || !host || n != c->n_params) return QUAPI_EINVAL;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return QUAPI_EDEVICE;
    return hipMemcpy(host, c->w, (size_t)n * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess ? QUAPI_OK
                                                                                                   : QUAPI_EDEVICE;
}

int quapi_mlp_get_grads(quapi_mlp* c, float* host, long long n) {
    if (!c || !host || n != c->n_params) return QUAPI_EINVAL;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return QUAPI_EDEVICE;
    return hipMemcpy(host, c->grad, (size_t)n * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess ? QUAPI_OK
                                                                                                      : QUAPI_EDEVICE;
}

int quapi_mlp_forward(quapi_mlp* c, const float* x, int batch, float* y) {
    if (!c || !x || !y) return QUAPI_EINVAL;
    if (check_batch(c, batch)) return QUAPI_EINVAL;
    if (stage_input(c, x, batch)) return QUAPI_EDEVICE;
    if (forward(c, batch)) return QUAPI_EDEVICE;
    const hipError_t e = hipMemcpyAsync(y, c->z[c->n_layers - 1], (size_t)batch * c->n_out * sizeof(float),
                                        hipMemcpyDeviceToDevice, c->stream);
    return e == hipSuccess ? QUAPI_OK : QUAPI_EDEVICE;
}

int quapi_mlp_backward(quapi_mlp* c, const float* x, const float* target, int batch, float* loss) {
    if (!c || !x || !target) return QUAPI_EINVAL;
    if (check_batch(c, batch)) return QUAPI_EINVAL;
    if (stage_input(c, x, batch)) return QUAPI_EDEVICE;
    if (forward(c, batch)) return QUAPI_EDEVICE;
    const int L = c->n_layers;
    // dL/dy of the mean over batch x n_out of (y - t)^2
    const long long ny = (long long)batch * c->n_out;
    const int lb = blocks_for(ny);
    const float scale = 1.0f / (float)ny;
    hipLaunchKernelGGL(loss_grad, dim3(lb), dim3(kVecThreads), 0, c->stream, c->z[L - 1], target, ny, scale, c->dzf,
                       c->dzb, c->loss_part);
    if (loss) hipLaunchKernelGGL(loss_sum, dim3(1), dim3(64), 0, c->stream, c->loss_part, lb, scale, loss);
    float* dzf = c->dzf;
    float* dzf_next = c->dzf2;
    uint16_t* dzb = c->dzb;
    uint16_t* dzb_next = c->dzb2;
    for (int l = L - 1; l >= 0; --l) {
        const int fin = c->fin[l], fout = c->fout[l];
        if (l == 0 && c->fp32_in) {
            // FP32 input layer: dW_0 = X^T dZ_0 in FP32, split over the batch
            const int splits = std::min(kMaxSplit, std::max(1, (batch + 255) / 256));
            const int rows = (batch + splits - 1) / splits;
            const int used = (batch + rows - 1) / rows;
            hipLaunchKernelGGL(dense_in_grad, dim3((fout + 63) / 64, used), dim3(kVecThreads), 0, c->stream, c->xf,
                               dzf, batch, fin, fout, rows, c->partial);
            const long long nw = (long long)fin * fout;
            hipLaunchKernelGGL(sum_splits, dim3(blocks_for(nw)), dim3(kVecThreads), 0, c->stream, c->partial, used,
                               nw, c->grad + c->w_off[0]);
            if (bias_grad(c, dzf, batch, fout, c->grad + c->b_off[0])) return QUAPI_EDEVICE;
            break;
        }
        // dW_l = A_{l-1}^T dZ_l: reduction over the batch, split over workgroups
        const int splits = std::min(kMaxSplit, std::max(1, (batch + 255) / 256));
        GemmArgs g{};
        g.A = l == 0 ? c->xb : c->ab[l - 1];   // A(m = input unit, k = sample)
        g.sam = 1;
        g.sak = fin;
        g.B = dzb;                             // B(k = sample, n = output unit)
        g.sbk = fout;
        g.sbn = 1;
        g.M = fin;
        g.N = fout;
        g.K = batch;
        g.kslice = ((batch + splits - 1) / splits + kTK - 1) / kTK * kTK;
        g.epi = kStoreF32;
        g.outf = c->partial;
        const int used = (batch + g.kslice - 1) / g.kslice;
        if (launch_gemm(c, g, used)) return QUAPI_EDEVICE;
        const long long nw = (long long)fin * fout;
        hipLaunchKernelGGL(sum_splits, dim3(blocks_for(nw)), dim3(kVecThreads), 0, c->stream, c->partial, used, nw,
                           c->grad + c->w_off[l]);
        if (bias_grad(c, dzf, batch, fout, c->grad + c->b_off[l])) return QUAPI_EDEVICE;
        if (l == 0) break;
        // dZ_{l-1} = (dZ_l W_l^T) * gelu'(Z_{l-1})
        GemmArgs h{};
        h.A = dzb;                             // A(m = sample, k = output unit)
        h.sam = fout;
        h.sak = 1;
        h.B = c->wb[l];                        // B(k = output unit, n = input unit) = W_l[n][k]
        h.sbk = 1;
        h.sbn = fout;
        h.M = batch;
        h.N = fin;
        h.K = fout;
        h.kslice = h.K;
        h.epi = kGeluGrad;
        h.zprev = c->z[l - 1];
        h.outf = dzf_next;
        h.outb = dzb_next;
        if (launch_gemm(c, h, 1)) return QUAPI_EDEVICE;
        std::swap(dzf, dzf_next);
        std::swap(dzb, dzb_next);
    }
    return hipGetLastError() == hipSuccess ? QUAPI_OK : QUAPI_EDEVICE;
}

int quapi_mlp_adam(quapi_mlp* c, float lr, float beta1, float beta2, float eps) {
    if (!c || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return QUAPI_EINVAL;
    ++c->adam_t;
    // bias corrections folded into the step size and epsilon
    const double c1 = 1.0 - std::pow((double)beta1, c->adam_t), c2 = 1.0 - std::pow((double)beta2, c->adam_t);
    const float lr_t = (float)(lr * std::sqrt(c2) / c1);
    const float eps_t = (float)(eps * std::sqrt(c2));
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(c->n_params)), dim3(kVecThreads), 0, c->stream, c->w, c->m, c->v,
                       c->grad, c->n_params, lr_t, beta1, beta2, eps_t);
    if (hipGetLastError() != hipSuccess) return QUAPI_EDEVICE;
    return refresh_bf16(c);
}

int quapi_mlp_sync(quapi_mlp* c) {
    if (!c) return QUAPI_EINVAL;
    return hipStreamSynchronize(c->stream) == hipSuccess ? QUAPI_OK : QUAPI_EDEVICE;
}

void quapi_mlp_destroy(quapi_mlp* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (void* p : c->allocs) (void)hipFree(p);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"
