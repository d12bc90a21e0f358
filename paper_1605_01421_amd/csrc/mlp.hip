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
#include <mutex>
#include <new>
#include <vector>

#include "siminf.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128;  // output tile per workgroup of 256 threads
constexpr int KT = 32;             // K per matrix-core step
constexpr int LDS_K = 40;          // padded LDS row (bf16 elements): 80 B, 16-byte aligned

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

// Epilogues: float32 result (+ bias); GELU with the pre-activation kept
// (training) or not (inference); gradient times GELU'; split-K partial.
enum Epi { EPI_STORE = 0, EPI_GELU = 1, EPI_DGELU = 2, EPI_GELU_ACT = 3, EPI_PART = 4 };

struct GemmArgs {
    int M, N, K;
    const uint16_t* A;
    int lda;  // AT ? A[k*lda + m] : A[m*lda + k]
    const uint16_t* B;
    int ldb;  // BT ? B[k*ldb + n] : B[n*ldb + k]
    const float* bias;  // [N] or null
    float* Cf;          // float32 result (EPI_STORE, EPI_GELU pre-activation, EPI_PART partials)
    int ldc;
    uint16_t* Cb;  // bfloat16 result (EPI_GELU / EPI_GELU_ACT activation, EPI_DGELU gradient)
    int ldcb;
    const float* Zp;  // EPI_DGELU: pre-activations the gradient is multiplied by GELU' of
    int ldzp;
    int kslice;  // K range of one blockIdx.z (a multiple of KT)
};

// Global -> register staging of one operand tile of R rows x KT k values.
// The operand is stored [row][k] (TRANS false, rows ld apart) or [k][row]
// (TRANS true); either way the LDS tile is [row][k], so that every lane
// reads the eight consecutive k values of its matrix-core operand in one
// 16-byte load.  VEC elements move per global load (8, 4 or 1): whole
// vectors inside the matrix, element by element at its ragged edges.
template <bool TRANS, int VEC, int R>
struct Stage {
    static constexpr int NV = R * KT / VEC / 256;
    static constexpr int NW = VEC > 1 ? VEC / 2 : 1;  // 32-bit words per vector
    static_assert(NV * VEC * 256 == R * KT, "tile does not split evenly over the workgroup");
    uint32_t w[NV][NW];

    __device__ __forceinline__ static void where(int i, int& row, int& k) {
        if (!TRANS) {
            row = i / (KT / VEC);
            k = (i % (KT / VEC)) * VEC;
        } else {
            k = i / (R / VEC);
            row = (i % (R / VEC)) * VEC;
        }
    }

    __device__ __forceinline__ static uint16_t half(const uint32_t (&x)[NW], int e) {
        if constexpr (VEC == 1) return (uint16_t)x[0];
        else return (uint16_t)(x[e >> 1] >> (16 * (e & 1)));
    }

    __device__ __forceinline__ void load(const uint16_t* P, int ld, int rows, int kend, int r0, int k0, int tid) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            int row, k;
            where(tid + j * 256, row, k);
            const int gr = r0 + row, gk = k0 + k;
            const bool full = !TRANS ? (gr < rows && gk + VEC <= kend) : (gk < kend && gr + VEC <= rows);
            const uint16_t* q = P + (!TRANS ? (size_t)gr * ld + gk : (size_t)gk * ld + gr);
            if (full) {
                if constexpr (VEC == 8) {
                    const uint4 x = *reinterpret_cast<const uint4*>(q);
                    w[j][0] = x.x;
                    w[j][1] = x.y;
                    w[j][2] = x.z;
                    w[j][3] = x.w;
                } else if constexpr (VEC == 4) {
                    const uint2 x = *reinterpret_cast<const uint2*>(q);
                    w[j][0] = x.x;
                    w[j][1] = x.y;
                } else {
                    w[j][0] = q[0];
                }
            } else {
#pragma unroll
                for (int e = 0; e < NW; ++e) w[j][e] = 0u;
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const bool in = !TRANS ? (gr < rows && gk + e < kend) : (gk < kend && gr + e < rows);
                    const uint32_t h = in ? (uint32_t)q[e] : 0u;
                    if constexpr (VEC == 1) w[j][0] = h;
                    else w[j][e >> 1] |= h << (16 * (e & 1));
                }
            }
        }
    }

    __device__ __forceinline__ void store(uint16_t* S, int tid) const {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            int row, k;
            where(tid + j * 256, row, k);
            if (!TRANS) {
                if constexpr (VEC == 8) {
                    *reinterpret_cast<uint4*>(&S[row * LDS_K + k]) = uint4{w[j][0], w[j][1], w[j][2], w[j][3]};
                } else if constexpr (VEC == 4) {
                    *reinterpret_cast<uint2*>(&S[row * LDS_K + k]) = uint2{w[j][0], w[j][1]};
                } else {
                    S[row * LDS_K + k] = (uint16_t)w[j][0];
                }
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) S[(row + e) * LDS_K + k] = half(w[j], e);
            }
        }
    }
};

// C[M,N] = A[M,K] B[K,N] (+ bias): a 128x128 tile per workgroup of four
// wavefronts, each computing 64x64 as 4x4 matrix-core tiles of 16x16 with
// K = 32 per step.  The next K step's operands are loaded from global memory
// into registers while the current step runs on the matrix cores.  With
// EPI_PART, blockIdx.z computes the partial product over its K slice.
template <bool AT, bool BT, int EPI, int VEC>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t As[BM * LDS_K];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * LDS_K];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    const int kbeg = blockIdx.z * g.kslice;
    const int kend = min(g.K, kbeg + g.kslice);
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    Stage<AT, VEC, BM> sa;
    Stage<BT, VEC, BN> sb;
    if (kbeg < kend) {
        sa.load(g.A, g.lda, g.M, kend, m0, kbeg, tid);
        sb.load(g.B, g.ldb, g.N, kend, n0, kbeg, tid);
    }
    const int kq = (lane >> 4) * 8, rl = lane & 15;
    for (int k0 = kbeg; k0 < kend; k0 += KT) {
        sa.store(As, tid);
        sb.store(Bs, tid);
        __syncthreads();
        if (k0 + KT < kend) {
            sa.load(g.A, g.lda, g.M, kend, m0, k0 + KT, tid);
            sb.load(g.B, g.ldb, g.N, kend, n0, k0 + KT, tid);
        }
        bf16x8 a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a[i] = *reinterpret_cast<const bf16x8*>(&As[(wr + i * 16 + rl) * LDS_K + kq]);
            b[i] = *reinterpret_cast<const bf16x8*>(&Bs[(wc + i * 16 + rl) * LDS_K + kq]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // ---- epilogue: lane l holds rows 4*(l/16)+r, column l%16 of each 16x16 tile
    float* part = EPI == EPI_PART ? g.Cf + (size_t)blockIdx.z * g.M * g.N : nullptr;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wr + i * 16 + (lane >> 4) * 4 + r;
                const int n = n0 + wc + j * 16 + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                float v = acc[i][j][r];
                if (EPI == EPI_PART) {
                    part[(size_t)m * g.N + n] = v;
                    continue;
                }
                if (g.bias) v += g.bias[n];
                if (EPI == EPI_STORE) {
                    g.Cf[(size_t)m * g.ldc + n] = v;
                } else if (EPI == EPI_GELU) {
                    g.Cf[(size_t)m * g.ldc + n] = v;
                    g.Cb[(size_t)m * g.ldcb + n] = f32_to_bf16(gelu(v));
                } else if (EPI == EPI_GELU_ACT) {
                    g.Cb[(size_t)m * g.ldcb + n] = f32_to_bf16(gelu(v));
                } else {
                    g.Cb[(size_t)m * g.ldcb + n] = f32_to_bf16(v * gelu_grad(g.Zp[(size_t)m * g.ldzp + n]));
                }
            }
}

// C[m,n] = sum over s of the split-K partials P[s][m][n], in slice order.
__global__ void splitk_reduce_kernel(const float* P, int S, int M, int N, float* C, int ldc) {
    const long long total = (long long)M * N;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int z = 0; z < S; ++z) s += P[(size_t)z * total + i];
        C[(i / N) * ldc + (i % N)] = s;
    }
}

// Widest vector both operands allow: row stride and base address aligned.
inline int vec_width(const GemmArgs& g) {
    auto ok = [&](int v) {
        return g.lda % v == 0 && g.ldb % v == 0 && ((uintptr_t)g.A % (2 * v)) == 0 && ((uintptr_t)g.B % (2 * v)) == 0;
    };
    return ok(8) ? 8 : ok(4) ? 4 : 1;
}

template <bool AT, bool BT, int EPI>
hipError_t gemm(GemmArgs g, hipStream_t st, float* work = nullptr, int max_slices = 1) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    const int tiles = ((g.N + BN - 1) / BN) * ((g.M + BM - 1) / BM);
    // split K when the output has few tiles and K is long (weight gradients)
    int S = 1;
    if (EPI == EPI_STORE && work && g.bias == nullptr)
        S = std::max(1, std::min({max_slices, (g.K + 255) / 256, std::max(1, 256 / std::max(tiles, 1))}));
    const int steps = (g.K + KT - 1) / KT;
    g.kslice = ((steps + S - 1) / S) * KT;
    if (g.kslice <= 0) g.kslice = KT;
    S = std::max(1, (g.K + g.kslice - 1) / g.kslice);
    dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, S);
    const int vec = vec_width(g);
    GemmArgs pg = g;
    if (S > 1) pg.Cf = work;
#define SIMINF_GEMM_LAUNCH(E)                                                              \
    do {                                                                                   \
        if (vec == 8) gemm_kernel<AT, BT, E, 8><<<grid, 256, 0, st>>>(pg);                 \
        else if (vec == 4) gemm_kernel<AT, BT, E, 4><<<grid, 256, 0, st>>>(pg);            \
        else gemm_kernel<AT, BT, E, 1><<<grid, 256, 0, st>>>(pg);                          \
    } while (0)
    if (S > 1) {
        SIMINF_GEMM_LAUNCH(EPI_PART);
        if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
        const long long total = (long long)g.M * g.N;
        const int blocks = (int)std::max<long long>(1, std::min<long long>((total + 255) / 256, 4096));
        splitk_reduce_kernel<<<blocks, 256, 0, st>>>(work, S, g.M, g.N, g.Cf, g.ldc);
    } else {
        SIMINF_GEMM_LAUNCH(EPI);
    }
#undef SIMINF_GEMM_LAUNCH
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
__global__ void __launch_bounds__(256) pinball_kernel(const float* Y, const float* T, int B, int N, Levels lv,
                                                      uint16_t* dY, double* loss) {
    __shared__ double red[4];
    const int total = B * N;
    double part = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int r = (i % N) % lv.nq;
        float q = lv.q[0];
#pragma unroll
        for (int c = 1; c < 8; ++c) q = r == c ? lv.q[c] : q;  // selects: no indexed private array
        const float d = T[i] - Y[i];
        part += d > 0.f ? (double)q * d : (double)(q - 1.f) * d;
        dY[i] = f32_to_bf16((d > 0.f ? -q : 1.f - q) / (float)total);
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, ((red[0] + red[1]) + red[2]) + red[3]);
}

// Column sums db[n] = sum_b dZ[b, n] in two deterministic passes: block
// (x, y) sums rows 256y.. of columns 64x.. (64 columns x 4 row lanes, then
// an LDS reduction) into part[y][n]; colsum_finish adds the parts in order.
__global__ void colsum_kernel(const uint16_t* dZ, int B, int N, int ld, float* part) {
    __shared__ float red[4][64];
    const int c = threadIdx.x & 63, rlane = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + c;
    const int r0 = blockIdx.y * 256;
    float s = 0.f;
    if (n < N)
        for (int r = r0 + rlane; r < min(B, r0 + 256); r += 4) s += bf16_to_f32(dZ[(size_t)r * ld + n]);
    red[rlane][c] = s;
    __syncthreads();
    if (rlane == 0 && n < N) part[(size_t)blockIdx.y * N + n] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

__global__ void colsum_finish(const float* part, int chunks, int N, float* db) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int y = 0; y < chunks; ++y) s += part[(size_t)y * N + n];
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

// The ensemble's answer for sample b (one workgroup per sample): every
// member's standardised output p is mapped back, y = p * y_std + y_mean
// (binary64), Y = the members' mean, and the disagreement is the mean over
// the outputs of the members' sample standard deviation (divisor K - 1; 0
// for a single member).  The sums run in a fixed order.
__global__ void __launch_bounds__(256) ensemble_combine_kernel(const float* P, int K, int B, int N,
                                                               const float* ymean, const float* ystd, float* Y,
                                                               float* dis) {
    __shared__ double red[256];
    const int b = blockIdx.x;
    double ssum = 0.0;
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
        const double sd = ystd[j], mu = ymean[j];
        double mean = 0.0;
        for (int k = 0; k < K; ++k) mean += (double)P[((size_t)k * B + b) * N + j] * sd + mu;
        mean /= (double)K;
        double m2 = 0.0;
        for (int k = 0; k < K; ++k) {
            const double d = ((double)P[((size_t)k * B + b) * N + j] * sd + mu) - mean;
            m2 += d * d;
        }
        Y[(size_t)b * N + j] = (float)mean;
        ssum += K > 1 ? sqrt(m2 / (double)(K - 1)) : 0.0;
    }
    red[threadIdx.x] = ssum;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) dis[b] = (float)(red[0] / (double)N);
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
    float* work = nullptr;   // split-K partial products of the weight gradients
    float* cpart = nullptr;  // column-sum partials of the bias gradients
};

constexpr int MAX_SLICES = 16;  // split-K slices of a weight-gradient product

namespace {
template <class T>
bool dalloc(siminf_mlp* m, size_t n, T** p) {
    *p = nullptr;
    if (hipMalloc((void**)p, sizeof(T) * std::max<size_t>(n, 1)) != hipSuccess) return false;
    m->owned.push_back(*p);
    return hipMemset(*p, 0, sizeof(T) * std::max<size_t>(n, 1)) == hipSuccess;
}

// train: keep the float32 pre-activations that the backward pass needs.
int mlp_forward(siminf_mlp* m, const float* X, int B, hipStream_t st, bool train) {
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
            e = train ? gemm<false, false, EPI_GELU>(g, st) : gemm<false, false, EPI_GELU_ACT>(g, st);
        } else {
            e = gemm<false, false, EPI_STORE>(g, st);
        }
        if (e != hipSuccess) return SIMINF_E_DEVICE;
    }
    return SIMINF_OK;
}
// The ensemble prediction into the workspace `work` (members x B x N
// floats): each member's forward pass in slices of its largest batch, its
// outputs copied into its part of the workspace, then the combination.
int ensemble_predict(siminf_mlp* const* nets, int K, const float* X, int B, const float* ymean, const float* ystd,
                     float* Y, float* dis, hipStream_t st, float* work) {
    const int din = nets[0]->dims[0], N = nets[0]->dims[nets[0]->L];
    for (int k = 0; k < K; ++k) {
        siminf_mlp* m = nets[k];
        for (int b0 = 0; b0 < B; b0 += m->max_batch) {
            const int bs = std::min(m->max_batch, B - b0);
            const int rc = mlp_forward(m, X + (size_t)b0 * din, bs, st, false);
            if (rc) return rc;
            if (hipMemcpyAsync(work + ((size_t)k * B + b0) * N, m->Z[m->L - 1], sizeof(float) * (size_t)bs * N,
                               hipMemcpyDeviceToDevice, st) != hipSuccess)
                return SIMINF_E_DEVICE;
        }
    }
    ensemble_combine_kernel<<<B, 256, 0, st>>>(work, K, B, N, ymean, ystd, Y, dis);
    return hipGetLastError() == hipSuccess ? SIMINF_OK : SIMINF_E_DEVICE;
}

int ensemble_check(siminf_mlp* const* nets, int K, const float* X, int B, const float* ymean, const float* ystd,
                   const float* Y, const float* dis) {
    if (!nets || K < 1 || K > 64 || !X || B < 1 || !ymean || !ystd || !Y || !dis) return SIMINF_E_ARG;
    for (int k = 0; k < K; ++k) {
        if (!nets[k]) return SIMINF_E_ARG;
        if (nets[k]->dims[0] != nets[0]->dims[0] || nets[k]->dims[nets[k]->L] != nets[0]->dims[nets[0]->L])
            return SIMINF_E_ARG;
    }
    return SIMINF_OK;
}
// The workspace of siminf_mlp_ensemble_predict_static, for callers that
// cannot allocate: a fixed array in device memory, one per device (each GPU
// the library runs on holds it until the process ends).  In host code the
// array's name is not a device address: its address on the current device
// comes from hipGetSymbolAddress, taken once per device.
constexpr size_t SCRATCH_FLOATS = (size_t)1 << 22;  // 16 MiB
__device__ __align__(256) float scratch[SCRATCH_FLOATS];

constexpr int SCRATCH_DEVICES = 64;
std::mutex scratch_mutex;
float* scratch_ptr[SCRATCH_DEVICES] = {};

// The current device's copy of `scratch`, or nullptr (and *rc set).
float* scratch_on_current_device(int* rc) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SCRATCH_DEVICES) {
        *rc = SIMINF_E_DEVICE;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            *rc = SIMINF_E_DEVICE;
            return nullptr;
        }
        scratch_ptr[dev] = (float*)ptr;
    }
    return scratch_ptr[dev];
}
}  // namespace

extern "C" {

int siminf_mlp_create(int32_t nlayers, const int32_t* dims, int32_t max_batch, siminf_mlp** out) {
    if (!out || !dims || nlayers < 1 || nlayers > 64 || max_batch < 1) return SIMINF_E_ARG;
    for (int i = 0; i <= nlayers; ++i)
        if (dims[i] < 1 || dims[i] > 65536 || (long long)dims[i] * max_batch > 0x7FFFFFFFLL) return SIMINF_E_ARG;
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
    size_t wmax = 1, nmax = 1;
    for (int l = 0; l < nlayers; ++l) {
        wmax = std::max(wmax, (size_t)dims[l + 1] * dims[l]);
        nmax = std::max(nmax, (size_t)dims[l + 1]);
    }
    ok = ok && dalloc(m, 1, &m->loss) && dalloc(m, (size_t)MAX_SLICES * wmax, &m->work) &&
         dalloc(m, (size_t)((max_batch + 255) / 256) * nmax, &m->cpart);
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
    const int rc = mlp_forward(m, X, B, st, false);
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
    int rc = mlp_forward(m, X, B, st, true);
    if (rc) return rc;
    const int L = m->L, Nout = m->dims[L];
    pinball_kernel<<<std::min(grid_for((long long)B * Nout), 512), 256, 0, st>>>(m->Z[L - 1], T, B, Nout, lv, m->dZ[L - 1],
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
        if (gemm<true, true, EPI_STORE>(g, st, m->work, MAX_SLICES) != hipSuccess) return SIMINF_E_DEVICE;
        const int chunks = (B + 255) / 256;
        colsum_kernel<<<dim3((N + 63) / 64, chunks), 256, 0, st>>>(m->dZ[l], B, N, N, m->cpart);
        colsum_finish<<<(N + 255) / 256, 256, 0, st>>>(m->cpart, chunks, N, m->gb[l]);
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

int siminf_mlp_ensemble_predict(siminf_mlp* const* nets, int32_t members, const float* X, int32_t B,
                                const float* y_mean, const float* y_std, float* Y, float* disagreement,
                                void* hip_stream) {
    int rc = ensemble_check(nets, members, X, B, y_mean, y_std, Y, disagreement);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t n = (size_t)members * B * nets[0]->dims[nets[0]->L];
    float* work = nullptr;
    if (hipMallocAsync((void**)&work, sizeof(float) * n, st) != hipSuccess) return SIMINF_E_ALLOC;
    rc = ensemble_predict(nets, members, X, B, y_mean, y_std, Y, disagreement, st, work);
    if (hipFreeAsync(work, st) != hipSuccess && rc == SIMINF_OK) rc = SIMINF_E_DEVICE;
    return rc;
}

int siminf_mlp_ensemble_predict_static(siminf_mlp* const* nets, int32_t members, const float* X, int32_t B,
                                       const float* y_mean, const float* y_std, float* Y, float* disagreement,
                                       void* hip_stream) {
    int rc = ensemble_check(nets, members, X, B, y_mean, y_std, Y, disagreement);
    if (rc) return rc;
    const size_t n = (size_t)members * B * nets[0]->dims[nets[0]->L];
    if (n > SCRATCH_FLOATS) return SIMINF_E_UNSUPPORTED;
    float* work = scratch_on_current_device(&rc);
    if (!work) return rc;
    return ensemble_predict(nets, members, X, B, y_mean, y_std, Y, disagreement, (hipStream_t)hip_stream, work);
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
