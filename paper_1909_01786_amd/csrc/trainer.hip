// trainer.hip -- training kernels of the learned Decision's scorer (gfx950).
//
// The scorer of the score-driven Decision (a message-passing network over
// the bipartite graph of variables and static nogoods; the integer form in
// scorer.hip) is trained in its float form: activations a in [0, 1]
// (integer code / 256), matrices w in [-127/128, 127/128] (code / 128),
// biases b = code / 2^17, so that a layer
//     a' = clamp(u / 4 + b, 0, 1),   u = a S + norm(sum over edges of a_src P|N)
// is the integer layer act(z) = min(255, (z + 256) >> 9) divided by 256 up
// to its roundings.  Every dense product runs on the matrix cores with
// bfloat16 operands and float32 accumulation (32x32x16 blocks); edge sums
// are segment sums over the two CSR orders of the literals (by nogood and by
// variable), so each direction of the message passing -- and its gradient,
// which runs the other way -- is a gather, never a scattered atomic.
//
// Row arrays are [rows][64] float32, row-major.  Matrices are [in][out].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "trainer.h"

namespace asp {
namespace {

#define DEV __device__ __forceinline__

constexpr int H = 64;
constexpr int NT = 256;          // threads per workgroup (four waves)
constexpr int LDT = H + 8;       // LDS row stride of bf16 tiles (16-byte rows, bank offset)

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

DEV __bf16 tobf(float x) { return (__bf16)x; }

// Element r of a 32x32 block held by `lane`: row, column inside the block.
DEV int blk_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// One 32x32 output block over K = 64: A rows (stride LDT, row i at A + i*LDT,
// k contiguous) times B given as rows of its transpose (BT row j holds
// column j of B, k contiguous).  Lane l supplies row / column l % 32 and
// k = 8 (l / 32) + 0..7 of each 16-wide k step.
DEV v16f mma64(const __bf16* A, const __bf16* BT, int lane) {
    v16f acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    const int i = lane & 31, kh = (lane >> 5) * 8;
#pragma unroll
    for (int k0 = 0; k0 < H; k0 += 16) {
        const v8bf x = *(const v8bf*)(A + i * LDT + k0 + kh);
        const v8bf y = *(const v8bf*)(BT + i * LDT + k0 + kh);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, acc, 0, 0, 0);
    }
    return acc;
}

// Stage rows [r0, r0+64) of a [rows][64] float array into a bf16 tile
// (zero past `rows`).
DEV void stage_rows(__bf16* T, const float* X, int64_t r0, int64_t rows, int tid) {
    for (int idx = tid; idx < 64 * 16; idx += NT) {
        const int r = idx >> 4, c4 = (idx & 15) * 4;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (r0 + r < rows) v = *(const float4*)(X + (r0 + r) * H + c4);
        __bf16* d = T + r * LDT + c4;
        d[0] = tobf(v.x); d[1] = tobf(v.y); d[2] = tobf(v.z); d[3] = tobf(v.w);
    }
}

// Stage the transpose of rows [r0, r0+64) (tile row c holds column c of the
// rows, k = row index), zero past `rows`.
DEV void stage_rows_t(__bf16* T, const float* X, int64_t r0, int64_t rows, int tid) {
    for (int idx = tid; idx < 64 * 64; idx += NT) {
        const int r = idx >> 6, c = idx & 63;
        const float v = r0 + r < rows ? X[(r0 + r) * H + c] : 0.f;
        T[c * LDT + r] = tobf(v);
    }
}

// ------------------------------------------------------------ kernels
// Y[r] = alpha * X[r] W (trans = 0) or alpha * X[r] W^T (trans = 1), plus
// Y[r] when acc; one 64-row tile per workgroup, grid-stride.
__global__ __launch_bounds__(NT) void k_mm(const float* X, const float* W, int trans, float* Y,
                                           int64_t rows, float alpha, int acc) {
    __shared__ __attribute__((aligned(16))) __bf16 sA[64 * LDT];
    __shared__ __attribute__((aligned(16))) __bf16 sBT[64 * LDT];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    // BT[j][k] = B[k][j] with B = W (trans 0) or W^T (trans 1)
    for (int idx = tid; idx < H * H; idx += NT) {
        const int k = idx >> 6, j = idx & 63;
        sBT[j * LDT + k] = tobf(trans ? W[j * H + k] : W[k * H + j]);
    }
    const int rb = w & 1, cb = w >> 1;
    const int64_t ntile = (rows + 63) / 64;
    for (int64_t t = blockIdx.x; t < ntile; t += gridDim.x) {
        __syncthreads();
        stage_rows(sA, X, t * 64, rows, tid);
        __syncthreads();
        const v16f o = mma64(sA + 32 * rb * LDT, sBT + 32 * cb * LDT, lane);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t row = t * 64 + 32 * rb + blk_row(r, lane);
            const int col = 32 * cb + (lane & 31);
            if (row < rows) {
                float* y = Y + row * H + col;
                *y = acc ? *y + alpha * o[r] : alpha * o[r];
            }
        }
    }
}

// dW[64][64] += X^T D over `rows` rows (K = rows): each workgroup sums its
// row chunks on the matrix cores, then adds its partial with atomics.
__global__ __launch_bounds__(NT) void k_mm_tn(const float* X, const float* D, float* dW,
                                              int64_t rows, int64_t rows_per_wg) {
    __shared__ __attribute__((aligned(16))) __bf16 sXT[64 * LDT];
    __shared__ __attribute__((aligned(16))) __bf16 sDT[64 * LDT];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int rb = w & 1, cb = w >> 1;
    v16f acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
    const int64_t r1 = r0 + rows_per_wg < rows ? r0 + rows_per_wg : rows;
    for (int64_t c = r0; c < r1; c += 64) {
        __syncthreads();
        stage_rows_t(sXT, X, c, r1, tid);
        stage_rows_t(sDT, D, c, r1, tid);
        __syncthreads();
        // out[i][j] = sum_k XT[i][k] DT[j][k]
        const int i = lane & 31, kh = (lane >> 5) * 8;
#pragma unroll
        for (int k0 = 0; k0 < 64; k0 += 16) {
            const v8bf x = *(const v8bf*)(sXT + (32 * rb + i) * LDT + k0 + kh);
            const v8bf y = *(const v8bf*)(sDT + (32 * cb + i) * LDT + k0 + kh);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = 32 * rb + blk_row(r, lane), col = 32 * cb + (lane & 31);
        if (acc[r] != 0.f) atomicAdd(&dW[row * H + col], acc[r]);
    }
}

// out[r] (+)= oscale[r] * sum over edges e of row r of
//     sscale[src] * (neg(e) ? SN : SP)[src],   src = idx[e] >> 1, neg = idx[e] & 1;
// a null SP or SN skips that sign, null scales are 1.  One wave per row,
// one column per lane.
__global__ __launch_bounds__(NT) void k_segsum(const int64_t* off, const int32_t* idx,
                                               const float* SP, const float* SN,
                                               const float* sscale, const float* oscale,
                                               float* out, int64_t rows, int acc) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (NT / 64);
    for (int64_t r = (int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6); r < rows; r += waves) {
        const int64_t e0 = off[r], e1 = off[r + 1];
        float s = 0.f;
        for (int64_t e = e0; e < e1; ++e) {
            const int32_t x = idx[e];
            const float* src = (x & 1) ? SN : SP;
            if (!src) continue;
            const int64_t q = (int64_t)(x >> 1);
            const float f = sscale ? sscale[q] : 1.f;
            s += f * src[q * H + lane];
        }
        if (oscale) s *= oscale[r];
        float* o = out + r * H + lane;
        *o = acc ? *o + s : s;
    }
}

// A = clamp(U / 4 + b, 0, 1).
__global__ __launch_bounds__(NT) void k_act_fwd(const float* U, const float* b, float* A,
                                                int64_t rows) {
    const int64_t n = rows * H;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const float z = 0.25f * U[i] + b[i & 63];
        A[i] = z <= 0.f ? 0.f : (z >= 1.f ? 1.f : z);
    }
}

// G = dA / 4 where 0 < A < 1 (else 0); db[j] += sum over rows of dA where
// 0 < A < 1.  Column sums: per-wave partials, then atomics.
__global__ __launch_bounds__(NT) void k_act_bwd(const float* dA, const float* A, float* G,
                                                float* db, int64_t rows) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (NT / 64);
    float cs = 0.f;
    for (int64_t r = (int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6); r < rows; r += waves) {
        const int64_t i = r * H + lane;
        const float a = A[i];
        const float g = (a > 0.f && a < 1.f) ? dA[i] : 0.f;
        G[i] = 0.25f * g;
        cs += g;
    }
    if (cs != 0.f) atomicAdd(&db[lane], cs);
}

// Embedding: A[r] = clamp(X8[r] E / 4 + e, 0, 1) with 8 input features.
__global__ __launch_bounds__(NT) void k_embed_fwd(const float* X8, const float* E, const float* e,
                                                  float* A, int64_t rows) {
    __shared__ float sE[8 * H];
    for (int i = threadIdx.x; i < 8 * H; i += NT) sE[i] = E[i];
    __syncthreads();
    const int64_t n = rows * H;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const int64_t r = i >> 6;
        const int j = (int)(i & 63);
        float z = 0.f;
#pragma unroll
        for (int f = 0; f < 8; ++f) z += X8[r * 8 + f] * sE[f * H + j];
        z = 0.25f * z + e[j];
        A[i] = z <= 0.f ? 0.f : (z >= 1.f ? 1.f : z);
    }
}

// dE[f][j] += sum over rows of X8[r][f] G[r][j].
__global__ __launch_bounds__(NT) void k_embed_bwd(const float* X8, const float* G, float* dE,
                                                  int64_t rows) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (NT / 64);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int64_t r = (int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6); r < rows; r += waves) {
        const float g = G[r * H + lane];
#pragma unroll
        for (int f = 0; f < 8; ++f) s[f] += X8[r * 8 + f] * g;
    }
#pragma unroll
    for (int f = 0; f < 8; ++f)
        if (s[f] != 0.f) atomicAdd(&dE[f * H + lane], s[f]);
}

// Readout and loss: for each labelled row (y >= 0), z = A wo + bo; the loss
// adds softplus(z) - y z (binary cross-entropy with logits) / n_lab; dA =
// (sigmoid(z) - y) / n_lab * wo, and dwo, dbo accumulate.  One wave per row.
__global__ __launch_bounds__(NT) void k_readout(const float* A, const float* y, const float* wo,
                                                const float* bo, float* dA, float* dwo,
                                                float* dbo, float* loss, int64_t rows,
                                                float inv_n) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (NT / 64);
    float gw = 0.f, gb = 0.f, ls = 0.f;
    const float w = wo[lane];
    for (int64_t r = (int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6); r < rows; r += waves) {
        const float lab = y[r];
        const float a = A[r * H + lane];
        if (lab < 0.f) {
            dA[r * H + lane] = 0.f;
            continue;
        }
        float z = a * w;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) z += __shfl_xor(z, d, 64);
        z += bo[0];
        const float p = 1.f / (1.f + __expf(-z));
        const float g = (p - lab) * inv_n;
        dA[r * H + lane] = g * w;
        gw += g * a;
        if (lane == 0) {
            gb += g;
            ls += (fmaxf(z, 0.f) - z * lab + log1pf(__expf(-fabsf(z)))) * inv_n;
        }
    }
    if (gw != 0.f) atomicAdd(&dwo[lane], gw);
    if (lane == 0) {
        if (gb != 0.f) atomicAdd(dbo, gb);
        if (ls != 0.f) atomicAdd(loss, ls);
    }
}

// Adam (beta1 0.9, beta2 0.999, eps 1e-8) on n parameters at step t (1-based);
// then each parameter is clipped to [-lim[k], lim[k]] of its range k
// (matrices: the weight codes' range; biases: the bias codes' range).
__global__ __launch_bounds__(NT) void k_adam(float* p, const float* g, float* m, float* v,
                                             int64_t n, float lr, float bc1, float bc2,
                                             const uint8_t* range, const float* lim) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const float gi = g[i];
        const float mi = 0.9f * m[i] + 0.1f * gi;
        const float vi = 0.999f * v[i] + 0.001f * gi * gi;
        m[i] = mi;
        v[i] = vi;
        float x = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
        const float L = lim[range[i]];
        p[i] = x < -L ? -L : (x > L ? L : x);
    }
}

}  // namespace

// ------------------------------------------------------------ launchers
static int grid_for(int64_t work, int per_wg) {
    int64_t g = (work + per_wg - 1) / per_wg;
    if (g < 1) g = 1;
    return g > 65536 ? 65536 : (int)g;
}

hipError_t tr_mm(const float* X, const float* W, int trans, float* Y, int64_t rows, float alpha,
                 int acc, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mm, dim3(grid_for((rows + 63) / 64, 1)), dim3(NT), 0, s, X, W, trans, Y,
                       rows, alpha, acc);
    return hipGetLastError();
}

hipError_t tr_mm_tn(const float* X, const float* D, float* dW, int64_t rows, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    const int64_t per = 2048;
    const int64_t g = (rows + per - 1) / per;
    hipLaunchKernelGGL(k_mm_tn, dim3((unsigned)g), dim3(NT), 0, s, X, D, dW, rows, per);
    return hipGetLastError();
}

hipError_t tr_segsum(const int64_t* off, const int32_t* idx, const float* SP, const float* SN,
                     const float* sscale, const float* oscale, float* out, int64_t rows, int acc,
                     hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_segsum, dim3(grid_for(rows, NT / 64)), dim3(NT), 0, s, off, idx, SP, SN,
                       sscale, oscale, out, rows, acc);
    return hipGetLastError();
}

hipError_t tr_act_fwd(const float* U, const float* b, float* A, int64_t rows, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_act_fwd, dim3(grid_for(rows * H, NT * 8)), dim3(NT), 0, s, U, b, A, rows);
    return hipGetLastError();
}

hipError_t tr_act_bwd(const float* dA, const float* A, float* G, float* db, int64_t rows,
                      hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_act_bwd, dim3(grid_for(rows, (NT / 64) * 16)), dim3(NT), 0, s, dA, A, G,
                       db, rows);
    return hipGetLastError();
}

hipError_t tr_embed_fwd(const float* X8, const float* E, const float* e, float* A, int64_t rows,
                        hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_embed_fwd, dim3(grid_for(rows * H, NT * 8)), dim3(NT), 0, s, X8, E, e, A,
                       rows);
    return hipGetLastError();
}

hipError_t tr_embed_bwd(const float* X8, const float* G, float* dE, int64_t rows, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_embed_bwd, dim3(grid_for(rows, (NT / 64) * 16)), dim3(NT), 0, s, X8, G,
                       dE, rows);
    return hipGetLastError();
}

hipError_t tr_readout(const float* A, const float* y, const float* wo, const float* bo, float* dA,
                      float* dwo, float* dbo, float* loss, int64_t rows, float inv_n,
                      hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_readout, dim3(grid_for(rows, (NT / 64) * 16)), dim3(NT), 0, s, A, y, wo,
                       bo, dA, dwo, dbo, loss, rows, inv_n);
    return hipGetLastError();
}

hipError_t tr_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, int t,
                   const uint8_t* range, const float* lim, hipStream_t s) {
    const float bc1 = 1.f - powf(0.9f, (float)t), bc2 = 1.f - powf(0.999f, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n, NT)), dim3(NT), 0, s, p, g, m, v, n, lr, bc1, bc2,
                       range, lim);
    return hipGetLastError();
}

}  // namespace asp
