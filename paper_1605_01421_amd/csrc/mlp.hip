// mlp.hip -- the surrogate network on gfx950: bfloat16 matrix products on
// the matrix cores (v_mfma_f32_16x16x32_bf16, float32 accumulation), fused
// bias / GELU / GELU' epilogues, pinball loss, bias gradients and AdamW.
//
// Layer l: Z_l = A_{l-1} W_l^T + b_l (float32), A_l = GELU(Z_l) stored as
// bfloat16 (hidden layers); the output layer keeps Z_L.  Backward:
//   dW_l = dZ_l^T A_{l-1},  db_l = sum_b dZ_l,  dZ_{l-1} = (dZ_l W_l) * GELU'(Z_{l-1})
// with dZ stored as bfloat16 before it enters a product.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "siminf.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TILE = 64;  // output tile per workgroup (M and N)
constexpr int KT = 32;    // K per matrix-core step
constexpr int LDS_K = 40; // padded row length of the LDS tiles (bf16 elements)

__host__ __device__ inline uint16_t f32_to_bf16(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);  // NaN
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf16_to_f32(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

__device__ inline float gelu(float z) { return 0.5f * z * erfcf(-z * 0.70710678118654752f); }
__device__ inline float gelu_grad(float z) {
    return 0.5f * erfcf(-z * 0.70710678118654752f) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

enum Epi { EPI_STORE = 0, EPI_GELU = 1, EPI_DGELU = 2 };

struct GemmArgs {
    int M, N, K;
    const uint16_t* A;
    int lda;  // AT ? A[k*lda + m] : A[m*lda + k]
    const uint16_t* B;
    int ldb;  // BT ? B[k*ldb + n] : B[n*ldb + k]
    const float* bias;  // [N] or null
    float* Cf;          // float32 result (EPI_STORE, EPI_GELU pre-activation)
    int ldc;
    uint16_t* Cb;  // bfloat16 result (EPI_GELU activation, EPI_DGELU gradient)
    int ldcb;
    const float* Zp;  // EPI_DGELU: pre-activations the gradient is multiplied by GELU' of
    int ldzp;
};

// C[M,N] = A[M,K] B[K,N] + bias, one 64x64 tile per workgroup of 256 threads.
// Wavefront w computes rows 32*(w/2).., columns 32*(w%2).. as 2x2 tiles of
// 16x16.  Operand tiles are staged in LDS as [row][k] so every lane reads its
// eight consecutive k values (lane l: row l%16, k 8*(l/16)..+7) in one load,
// whatever the orientation of the operand in global memory.
template <bool AT, bool BT, int EPI>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t As[TILE * LDS_K];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[TILE * LDS_K];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * TILE, n0 = blockIdx.x * TILE;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < g.K; k0 += KT) {
        // ---- stage A (64 rows x 32 k) and B (64 cols x 32 k) in LDS
        if (!AT) {
            const int r = tid >> 2, kc = (tid & 3) * 8;
            const int gm = m0 + r, gk = k0 + kc;
#pragma unroll
            for (int i = 0; i < 8; ++i)
                As[r * LDS_K + kc + i] = (gm < g.M && gk + i < g.K) ? g.A[(size_t)gm * g.lda + gk + i] : 0;
        } else {
            const int kk = tid >> 3, mc = (tid & 7) * 8;
            const int gk = k0 + kk;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int gm = m0 + mc + i;
                As[(mc + i) * LDS_K + kk] = (gm < g.M && gk < g.K) ? g.A[(size_t)gk * g.lda + gm] : 0;
            }
        }
        if (!BT) {
            const int r = tid >> 2, kc = (tid & 3) * 8;
            const int gn = n0 + r, gk = k0 + kc;
#pragma unroll
            for (int i = 0; i < 8; ++i)
                Bs[r * LDS_K + kc + i] = (gn < g.N && gk + i < g.K) ? g.B[(size_t)gn * g.ldb + gk + i] : 0;
        } else {
            const int kk = tid >> 3, nc = (tid & 7) * 8;
            const int gk = k0 + kk;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int gn = n0 + nc + i;
                Bs[(nc + i) * LDS_K + kk] = (gn < g.N && gk < g.K) ? g.B[(size_t)gk * g.ldb + gn] : 0;
            }
        }
        __syncthreads();
        // ---- 2x2 matrix-core products per wavefront
        bf16x8 a[2], b[2];
        const int kq = (lane >> 4) * 8, rl = lane & 15;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            a[i] = *reinterpret_cast<const bf16x8*>(&As[(wr + i * 16 + rl) * LDS_K + kq]);
            b[i] = *reinterpret_cast<const bf16x8*>(&Bs[(wc + i * 16 + rl) * LDS_K + kq]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // ---- epilogue: lane l holds rows 4*(l/16)+r, column l%16 of each 16x16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wr + i * 16 + (lane >> 4) * 4 + r;
                const int n = n0 + wc + j * 16 + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                float v = acc[i][j][r];
                if (g.bias) v += g.bias[n];
                if (EPI == EPI_STORE) {
                    g.Cf[(size_t)m * g.ldc + n] = v;
                } else if (EPI == EPI_GELU) {
                    g.Cf[(size_t)m * g.ldc + n] = v;
                    g.Cb[(size_t)m * g.ldcb + n] = f32_to_bf16(gelu(v));
                } else {
                    g.Cb[(size_t)m * g.ldcb + n] = f32_to_bf16(v * gelu_grad(g.Zp[(size_t)m * g.ldzp + n]));
                }
            }
}

template <bool AT, bool BT, int EPI>
hipError_t gemm(const GemmArgs& g, hipStream_t st) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    dim3 grid((g.N + TILE - 1) / TILE, (g.M + TILE - 1) / TILE);
    gemm_kernel<AT, BT, EPI><<<grid, 256, 0, st>>>(g);
    return hipGetLastError();
}

__global__ void to_bf16_kernel(const float* x, uint16_t* y, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        y[i] = f32_to_bf16(x[i]);
}

struct Levels {
    float q[8];
    int nq;
};

__global__ void zero_kernel(double* x) { *x = 0.0; }

// Pinball loss (sum accumulated in *loss) and its gradient dY / (B*N) as bf16.
__global__ void pinball_kernel(const float* Y, const float* T, int B, int N, Levels lv, uint16_t* dY,
                               double* loss) {
    const long long total = (long long)B * N;
    double part = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(i % N);
        const float q = lv.q[j % lv.nq];
        const float d = T[i] - Y[i];
        part += d > 0.f ? (double)q * d : (double)(q - 1.f) * d;
        dY[i] = f32_to_bf16((d > 0.f ? -q : 1.f - q) / (float)total);
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(loss, part);
}

// db[n] = sum_b dZ[b, n]
__global__ void colsum_kernel(const uint16_t* dZ, int B, int N, float* db) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += bf16_to_f32(dZ[(size_t)b * N + n]);
    db[n] = s;
}

// AdamW on float32 master weights; refreshes the bfloat16 copy.
__global__ void adamw_kernel(float* p, const float* g, float* m, float* v, uint16_t* pb, long long n, float lr,
                             float b1, float b2, float eps, float wd, float c1, float c2) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float mh = mi / c1, vh = vi / c2;
        const float w = p[i] - lr * (mh / (sqrtf(vh) + eps) + wd * p[i]);
        p[i] = w;
        if (pb) pb[i] = f32_to_bf16(w);
    }
}

int grid_for(long long n) { return (int)std::max<long long>(1, std::min<long long>((n + 255) / 256, 4096)); }

}  // namespace

struct siminf_mlp {
    int L = 0, max_batch = 0, t = 0;
    std::vector<int> dims;
    std::vector<void*> owned;
    std::vector<float*> W, b, gW, gb, mW, vW, mb, vb, Z;
    std::vector<uint16_t*> Wb, A, dZ;
    double* loss = nullptr;
    float* Y = nullptr;
};

namespace {
template <class T>
bool dalloc(siminf_mlp* m, size_t n, T** p) {
    *p = nullptr;
    if (hipMalloc((void**)p, sizeof(T) * std::max<size_t>(n, 1)) != hipSuccess) return false;
    m->owned.push_back(*p);
    return hipMemset(*p, 0, sizeof(T) * std::max<size_t>(n, 1)) == hipSuccess;
}

int mlp_forward(siminf_mlp* m, const float* X, int B, hipStream_t st) {
    const long long nin = (long long)B * m->dims[0];
    to_bf16_kernel<<<grid_for(nin), 256, 0, st>>>(X, m->A[0], nin);
    if (hipGetLastError() != hipSuccess) return SIMINF_E_DEVICE;
    for (int l = 0; l < m->L; ++l) {
        GemmArgs g{};
        g.M = B;
        g.N = m->dims[l + 1];
        g.K = m->dims[l];
        g.A = m->A[l];
        g.lda = m->dims[l];
        g.B = m->Wb[l];
        g.ldb = m->dims[l];
        g.bias = m->b[l];
        g.Cf = m->Z[l];
        g.ldc = g.N;
        hipError_t e;
        if (l + 1 < m->L) {
            g.Cb = m->A[l + 1];
            g.ldcb = g.N;
            e = gemm<false, false, EPI_GELU>(g, st);
        } else {
            e = gemm<false, false, EPI_STORE>(g, st);
        }
        if (e != hipSuccess) return SIMINF_E_DEVICE;
    }
    return SIMINF_OK;
}
}  // namespace

extern "C" {

int siminf_mlp_create(int32_t nlayers, const int32_t* dims, int32_t max_batch, siminf_mlp** out) {
    if (!out || !dims || nlayers < 1 || nlayers > 64 || max_batch < 1) return SIMINF_E_ARG;
    for (int i = 0; i <= nlayers; ++i)
        if (dims[i] < 1 || dims[i] > 65536) return SIMINF_E_ARG;
    siminf_mlp* m = new (std::nothrow) siminf_mlp();
    if (!m) return SIMINF_E_ALLOC;
    *out = m;
    m->L = nlayers;
    m->max_batch = max_batch;
    m->dims.assign(dims, dims + nlayers + 1);
    m->W.resize(nlayers);
    m->b.resize(nlayers);
    m->gW.resize(nlayers);
    m->gb.resize(nlayers);
    m->mW.resize(nlayers);
    m->vW.resize(nlayers);
    m->mb.resize(nlayers);
    m->vb.resize(nlayers);
    m->Z.resize(nlayers);
    m->Wb.resize(nlayers);
    m->dZ.resize(nlayers);
    m->A.resize(nlayers);
    bool ok = true;
    for (int l = 0; l < nlayers; ++l) {
        const size_t nw = (size_t)dims[l + 1] * dims[l], nb = dims[l + 1], nz = (size_t)max_batch * dims[l + 1];
        ok = ok && dalloc(m, nw, &m->W[l]) && dalloc(m, nb, &m->b[l]) && dalloc(m, nw, &m->gW[l]) &&
             dalloc(m, nb, &m->gb[l]) && dalloc(m, nw, &m->mW[l]) && dalloc(m, nw, &m->vW[l]) &&
             dalloc(m, nb, &m->mb[l]) && dalloc(m, nb, &m->vb[l]) && dalloc(m, nz, &m->Z[l]) &&
             dalloc(m, nw, &m->Wb[l]) && dalloc(m, nz, &m->dZ[l]) &&
             dalloc(m, (size_t)max_batch * dims[l], &m->A[l]);
    }
    ok = ok && dalloc(m, 1, &m->loss);
    if (!ok) return SIMINF_E_ALLOC;
    return SIMINF_OK;
}

int siminf_mlp_set_params(siminf_mlp* m, int32_t layer, const float* W, const float* b) {
    if (!m || layer < 0 || layer >= m->L || !W || !b) return SIMINF_E_ARG;
    const size_t nw = (size_t)m->dims[layer + 1] * m->dims[layer], nb = m->dims[layer + 1];
    std::vector<uint16_t> wb(nw);
    for (size_t i = 0; i < nw; ++i) wb[i] = f32_to_bf16(W[i]);
    if (hipMemcpy(m->W[layer], W, nw * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->b[layer], b, nb * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->Wb[layer], wb.data(), nw * 2, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(m->mW[layer], 0, nw * 4) != hipSuccess || hipMemset(m->vW[layer], 0, nw * 4) != hipSuccess ||
        hipMemset(m->mb[layer], 0, nb * 4) != hipSuccess || hipMemset(m->vb[layer], 0, nb * 4) != hipSuccess)
        return SIMINF_E_DEVICE;
    m->t = 0;
    return SIMINF_OK;
}

int siminf_mlp_get_params(const siminf_mlp* m, int32_t layer, float* W, float* b) {
    if (!m || layer < 0 || layer >= m->L) return SIMINF_E_ARG;
    const size_t nw = (size_t)m->dims[layer + 1] * m->dims[layer], nb = m->dims[layer + 1];
    if ((W && hipMemcpy(W, m->W[layer], nw * 4, hipMemcpyDeviceToHost) != hipSuccess) ||
        (b && hipMemcpy(b, m->b[layer], nb * 4, hipMemcpyDeviceToHost) != hipSuccess))
        return SIMINF_E_DEVICE;
    return SIMINF_OK;
}

int siminf_mlp_get_grads(const siminf_mlp* m, int32_t layer, float* dW, float* db) {
    if (!m || layer < 0 || layer >= m->L) return SIMINF_E_ARG;
    const size_t nw = (size_t)m->dims[layer + 1] * m->dims[layer], nb = m->dims[layer + 1];
    if (hipDeviceSynchronize() != hipSuccess ||
        (dW && hipMemcpy(dW, m->gW[layer], nw * 4, hipMemcpyDeviceToHost) != hipSuccess) ||
        (db && hipMemcpy(db, m->gb[layer], nb * 4, hipMemcpyDeviceToHost) != hipSuccess))
        return SIMINF_E_DEVICE;
    return SIMINF_OK;
}

int siminf_mlp_forward(siminf_mlp* m, const float* X, int32_t B, float* Y, void* hip_stream) {
    if (!m || !X || !Y || B < 1 || B > m->max_batch) return SIMINF_E_ARG;
    hipStream_t st = (hipStream_t)hip_stream;
    const int rc = mlp_forward(m, X, B, st);
    if (rc) return rc;
    const size_t ny = (size_t)B * m->dims[m->L];
    return hipMemcpyAsync(Y, m->Z[m->L - 1], ny * 4, hipMemcpyDeviceToDevice, st) == hipSuccess ? SIMINF_OK
                                                                                                 : SIMINF_E_DEVICE;
}

int siminf_mlp_backward(siminf_mlp* m, const float* X, const float* T, int32_t B, const double* probs, int32_t nq,
                        double* loss, void* hip_stream) {
    if (!m || !X || !T || !probs || B < 1 || B > m->max_batch || nq < 1 || nq > 8) return SIMINF_E_ARG;
    hipStream_t st = (hipStream_t)hip_stream;
    Levels lv{};
    lv.nq = nq;
    for (int i = 0; i < nq; ++i) lv.q[i] = (float)probs[i];
    zero_kernel<<<1, 1, 0, st>>>(m->loss);
    int rc = mlp_forward(m, X, B, st);
    if (rc) return rc;
    const int L = m->L, Nout = m->dims[L];
    pinball_kernel<<<grid_for((long long)B * Nout), 256, 0, st>>>(m->Z[L - 1], T, B, Nout, lv, m->dZ[L - 1],
                                                                 m->loss);
    if (hipGetLastError() != hipSuccess) return SIMINF_E_DEVICE;
    for (int l = L - 1; l >= 0; --l) {
        const int N = m->dims[l + 1], K = m->dims[l];
        // dW_l[N,K] = dZ_l^T A_{l-1}: reduction over the batch
        GemmArgs g{};
        g.M = N;
        g.N = K;
        g.K = B;
        g.A = m->dZ[l];
        g.lda = N;
        g.B = m->A[l];
        g.ldb = K;
        g.Cf = m->gW[l];
        g.ldc = K;
        if (gemm<true, true, EPI_STORE>(g, st) != hipSuccess) return SIMINF_E_DEVICE;
        colsum_kernel<<<(N + 255) / 256, 256, 0, st>>>(m->dZ[l], B, N, m->gb[l]);
        if (hipGetLastError() != hipSuccess) return SIMINF_E_DEVICE;
        if (l > 0) {
            // dZ_{l-1}[B,K] = (dZ_l W_l) * GELU'(Z_{l-1})
            GemmArgs d{};
            d.M = B;
            d.N = K;
            d.K = N;
            d.A = m->dZ[l];
            d.lda = N;
            d.B = m->Wb[l];
            d.ldb = K;
            d.Cb = m->dZ[l - 1];
            d.ldcb = K;
            d.Zp = m->Z[l - 1];
            d.ldzp = K;
            if (gemm<false, true, EPI_DGELU>(d, st) != hipSuccess) return SIMINF_E_DEVICE;
        }
    }
    if (loss) {
        double s = 0.0;
        if (hipMemcpyAsync(&s, m->loss, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return SIMINF_E_DEVICE;
        *loss = s / ((double)B * Nout);
    }
    return SIMINF_OK;
}

int siminf_mlp_adamw(siminf_mlp* m, float lr, float beta1, float beta2, float eps, float weight_decay,
                     void* hip_stream) {
    if (!m) return SIMINF_E_ARG;
    hipStream_t st = (hipStream_t)hip_stream;
    m->t += 1;
    const float c1 = 1.f - powf(beta1, (float)m->t), c2 = 1.f - powf(beta2, (float)m->t);
    for (int l = 0; l < m->L; ++l) {
        const long long nw = (long long)m->dims[l + 1] * m->dims[l], nb = m->dims[l + 1];
        adamw_kernel<<<grid_for(nw), 256, 0, st>>>(m->W[l], m->gW[l], m->mW[l], m->vW[l], m->Wb[l], nw, lr, beta1,
                                                  beta2, eps, weight_decay, c1, c2);
        adamw_kernel<<<grid_for(nb), 256, 0, st>>>(m->b[l], m->gb[l], m->mb[l], m->vb[l], nullptr, nb, lr, beta1,
                                                  beta2, eps, weight_decay, c1, c2);
        if (hipGetLastError() != hipSuccess) return SIMINF_E_DEVICE;
    }
    return SIMINF_OK;
}

void siminf_mlp_destroy(siminf_mlp* m) {
    if (!m) return;
    (void)hipDeviceSynchronize();
    for (void* p : m->owned) (void)hipFree(p);
    delete m;
}

int siminf_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t* A, int32_t lda, int32_t a_trans,
                     const uint16_t* B, int32_t ldb, int32_t b_trans, float* C, int32_t ldc, void* hip_stream) {
    if (M < 0 || N < 0 || K < 0 || !A || !B || !C) return SIMINF_E_ARG;
    GemmArgs g{};
    g.M = M;
    g.N = N;
    g.K = K;
    g.A = A;
    g.lda = lda;
    g.B = B;
    g.ldb = ldb;
    g.Cf = C;
    g.ldc = ldc;
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e;
    if (!a_trans && !b_trans) e = gemm<false, false, EPI_STORE>(g, st);
    else if (!a_trans && b_trans) e = gemm<false, true, EPI_STORE>(g, st);
    else if (a_trans && !b_trans) e = gemm<true, false, EPI_STORE>(g, st);
    else e = gemm<true, true, EPI_STORE>(g, st);
    return e == hipSuccess ? SIMINF_OK : SIMINF_E_DEVICE;
}

}  // extern "C"
