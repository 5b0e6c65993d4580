// scorer.hip -- the learned Decision's atom scorer for gfx950 (CDNA4, wave64).
//
// The Decision of Sect. 2 picks an applicable rule by a score of its head.
// The learned form scores atoms with a message-passing network over the
// bipartite graph of variables and static nogoods (edges: nogood literals,
// with their sign).  The network is quantisation-aware so that it is exact:
// activations are integer codes 0..255 and weights integer codes -127..127,
// both held as bfloat16; a 64-term product of them is an integer below 2^21,
// exact in the float32 accumulator of the matrix cores whatever the order of
// its sums.  Edge terms are integer too (below), and the requantisation
// act(z) = min(255, (z + 256) >> 9) for z > 0 is integer.
//
// Work is cut into tiles of 64 rows of one instance (variables, or static
// nogoods), one workgroup of four waves per tile, tiles taken grid-stride so
// each workgroup stages the layer's weights into LDS once.  Each row's edge
// sources are summed first (four threads per row, 16 columns each, the
// positive and the negative edges apart), and the sums are multiplied once
// by both sign matrices stacked along K on the matrix cores (32x32x16 bf16
// blocks), in base-256 limbs so that every operand is exact in bfloat16 --
// by linearity the same integer as summing every edge's product, with no
// per-edge products and no atomics.  The epilogue multiplies the tile's own
// rows by the self matrix, adds the normalised edge term and the bias,
// requantises, and stores the 64 codes per row.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/asp.h"
#include "scorer.h"

namespace asp {
namespace {

#define DEV __device__ __forceinline__

constexpr int H = ASP_SCORER_H;   // hidden width
constexpr int F = ASP_SCORER_F;   // input features
constexpr int TR = 64;            // rows per tile
constexpr int NT = 256;           // threads per workgroup
constexpr int LD = H + 8;         // LDS row stride of bf16 operand tiles (16-byte rows)

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

DEV const uint16_t* wmat(const ScorerArgs& a, size_t off) { return (const uint16_t*)(a.w + off); }
DEV const int32_t* wvec(const ScorerArgs& a, size_t off) { return (const int32_t*)(a.w + off); }

// An integer-valued bfloat16 as int (exact for the codes used here).
DEV int bf16_int(uint16_t b) { return (int)__uint_as_float((uint32_t)b << 16); }
// Activation code 0..255 as bfloat16 bits (exact).
DEV uint16_t code_bf16(uint32_t code) { return (uint16_t)(__float_as_uint((float)code) >> 16); }

DEV int act(long long z) { return z <= 0 ? 0 : (int)(((z + 256) >> 9) < 255 ? ((z + 256) >> 9) : 255); }

// s / 2^k rounded half up (arithmetic shift), k = ceil(log2 n); n <= 1: s.
DEV long long norm_sum(long long s, int n) {
    if (n <= 1) return s;
    const int k = 32 - __clz(n - 1);
    return (s + (1LL << (k - 1))) >> k;
}

// One 32x32 block: 32 rows of an operand tile (stride LD) times 32 output
// columns given as rows of a transposed weight tile (stride LD), K = 64, in
// four 32x32x16 steps; lane l supplies row / column l % 32 and k = 8 (l / 32)
// + 0..7 of each step.
DEV v16f mma_block(const uint16_t* A, const uint16_t* BT, int lane) {
    v16f acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    const int i = lane & 31, kh = (lane >> 5) * 8;
#pragma unroll
    for (int k0 = 0; k0 < H; k0 += 16) {
        const v8bf x = *(const v8bf*)(A + i * LD + k0 + kh);
        const v8bf y = *(const v8bf*)(BT + i * LD + k0 + kh);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, acc, 0, 0, 0);
    }
    return acc;
}

// Row of output element r of a 32x32 block (its column is lane % 32).
DEV int blk_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// BT[j][k] = M[k][j] for a [64][64] matrix M held in global memory.
DEV void stage_t(uint16_t* BT, const uint16_t* M, int tid) {
    for (int idx = tid; idx < H * H; idx += NT) {
        const int k = idx >> 6, j = idx & 63;
        BT[j * LD + k] = M[k * H + j];
    }
}

// Both sign matrices side by side along K: operand rows of 2H values (the
// positive-edge sums, then the negative-edge sums) times [M+; M-].
constexpr int K2 = 2 * H;
constexpr int LD2 = K2 + 8;       // LDS row stride of the 2H-wide tiles (16-byte rows)

// One 32x32 block of a 2H-wide operand tile (stride LD2) times 32 output
// columns given as rows of the transposed stacked weights (stride LD2).
DEV v16f mma_block2(const uint16_t* A, const uint16_t* BT, int lane) {
    v16f acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    const int i = lane & 31, kh = (lane >> 5) * 8;
#pragma unroll
    for (int k0 = 0; k0 < K2; k0 += 16) {
        const v8bf x = *(const v8bf*)(A + i * LD2 + k0 + kh);
        const v8bf y = *(const v8bf*)(BT + i * LD2 + k0 + kh);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, acc, 0, 0, 0);
    }
    return acc;
}

// BT[j][m H + k] = M_m[k][j] for the [64][64] matrices M_0 (positive edges)
// and M_1 (negative edges) held in global memory.
DEV void stage_t2(uint16_t* BT, const uint16_t* M0, const uint16_t* M1, int tid) {
    for (int idx = tid; idx < 2 * H * H; idx += NT) {
        const int m = idx >= H * H ? 1 : 0, r = idx - m * H * H;
        const int k = r >> 6, j = r & 63;
        BT[j * LD2 + m * H + k] = (m ? M1 : M0)[k * H + j];
    }
}

// 16 activation codes from global memory as bfloat16 into an operand row.
DEV void load_codes16(uint16_t* dst, const uint8_t* src) {
    const uint4 q = *(const uint4*)src;
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int t = 0; t < 4; ++t) dst[4 * b + t] = code_bf16((w[b] >> (8 * t)) & 255u);
}

DEV void zero16(uint16_t* dst) {
#pragma unroll
    for (int t = 0; t < 16; ++t) dst[t] = 0;
}

// 16 codes (bytes of a row quarter) added into 16 integer sums.
DEV void add_codes16(int* s, const uint4 q) {
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int t = 0; t < 4; ++t) s[4 * b + t] += (int)((w[b] >> (8 * t)) & 255u);
}

// LDS of the layer kernels (dynamic, 16-byte aligned base).
struct LayerLds {
    uint16_t* wt;              // [H][LD2] both sign matrices, stacked along K, transposed
    uint16_t* st;              // [H][LD] self matrix, transposed
    uint16_t* opa;             // [TR][LD2] operand tile: sum limbs, then (stride LD) the
                               // tile's own rows; the output codes alias it
    int32_t* start;            // [2TR+1] segment starts
    int32_t* bias;             // [H]
    int32_t* smax;             // [1] largest edge sum of the tile
};

constexpr size_t kLayerLds = sizeof(uint16_t) * H * LD2 + sizeof(uint16_t) * H * LD +
                             sizeof(uint16_t) * TR * LD2 + sizeof(int32_t) * (2 * TR + 1 + H + 1) + 16;

DEV LayerLds carve(unsigned char* p) {
    LayerLds L;
    L.wt = (uint16_t*)p; p += sizeof(uint16_t) * H * LD2;
    L.st = (uint16_t*)p; p += sizeof(uint16_t) * H * LD;
    L.opa = (uint16_t*)p; p += sizeof(uint16_t) * TR * LD2;
    L.start = (int32_t*)p; p += sizeof(int32_t) * (2 * TR + 1);
    L.bias = (int32_t*)p; p += sizeof(int32_t) * H;
    L.smax = (int32_t*)p;
    return L;
}

// The edge term of a tile: for each row, the sums of its neighbours' code
// rows over its positive and over its negative edges (thread: one row, one
// quarter of the columns), times [M+; M-] on the matrix cores.  A product
// is linear, so this equals the sum of every edge's own product.  The sums
// (up to 255 per edge) are split into base-256 limbs, each exact in
// bfloat16; a limb's product (|.| <= 255 * 127 * 2H < 2^24) is exact in the
// float32 accumulator, and the limbs recombine in 64-bit integers.  Returns
// this lane's 16 elements of its wave's 32x32 output block.
template <class Edges>
DEV void edge_term(const LayerLds& L, int rows, Edges edges, int tid, long long* tot) {
    const int w = tid >> 6, lane = tid & 63;
    const int r = 16 * w + (lane >> 2), q = lane & 3;
    int sp[16], sn[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) sp[t] = sn[t] = 0;
    if (r < rows) edges(r, q, sp, sn);
    int mx = 0;
#pragma unroll
    for (int t = 0; t < 16; ++t) mx = max(mx, max(sp[t], sn[t]));
    if (tid == 0) *L.smax = 0;
    __syncthreads();
    atomicMax(L.smax, mx);
    __syncthreads();
    const int top = *L.smax;
    const int nl = top < (1 << 8) ? 1 : top < (1 << 16) ? 2 : top < (1 << 24) ? 3 : 4;
    const int rb = w & 1, cb = w >> 1;
#pragma unroll
    for (int t = 0; t < 16; ++t) tot[t] = 0;
    for (int li = 0; li < nl; ++li) {
        uint16_t* row = L.opa + r * LD2 + 16 * q;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            row[t] = code_bf16(((uint32_t)sp[t] >> (8 * li)) & 255u);
            row[H + t] = code_bf16(((uint32_t)sn[t] >> (8 * li)) & 255u);
        }
        __syncthreads();
        const v16f o = mma_block2(L.opa + 32 * rb * LD2, L.wt + 32 * cb * LD2, lane);
#pragma unroll
        for (int t = 0; t < 16; ++t) tot[t] += (long long)(int)o[t] * (1LL << (8 * li));
        __syncthreads();
    }
}

// Epilogue: own rows (loaded into the operand tile at stride LD) times the
// self matrix, plus the normalised edge term and the bias, requantised into
// `out` rows.  seg_len(row) gives the normaliser; rows >= rows_n are not
// written.
template <class Len>
DEV void finish_tile(const LayerLds& L, int rows_n, Len seg_len, int zero_row, const long long* tot,
                     uint8_t* out, int tid) {
    const int w = tid >> 6, lane = tid & 63;
    const int rb = w & 1, cb = w >> 1;
    const v16f o = mma_block(L.opa + 32 * rb * LD, L.st + 32 * cb * LD, lane);
    __syncthreads();                               // operand tile is read; codes may alias it
    uint8_t* codes = (uint8_t*)L.opa;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = 32 * rb + blk_row(r, lane), col = 32 * cb + (lane & 31);
        if (row < rows_n) {
            const long long z = (long long)(int)o[r] + norm_sum(tot[r], seg_len(row)) + L.bias[col];
            codes[row * H + col] = row == zero_row ? (uint8_t)0 : (uint8_t)act(z);
        }
    }
    __syncthreads();
    const int row = tid >> 2, part = tid & 3;
    if (row < rows_n) *(uint4*)(out + (size_t)row * H + part * 16) = *(const uint4*)(codes + row * H + part * 16);
}

// ------------------------------------------------------------------ kernels
__global__ __launch_bounds__(NT) void k_embed(ScorerArgs a) {
    __shared__ int sE[F * H];
    __shared__ int sB[H];
    __shared__ int sX[TR][F];
    const int tid = threadIdx.x;
    const int total = a.n_vtiles + a.n_ctiles;
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const bool var = t < a.n_vtiles;
        const ScorerTile tl = var ? a.vtiles[t] : a.ctiles[t - a.n_vtiles];
        const InstDesc& d = a.inst[tl.inst];
        const uint16_t* E = wmat(a, var ? offsetof(asp_scorer_weights, Ev) : offsetof(asp_scorer_weights, Ec));
        const int32_t* eb = wvec(a, var ? offsetof(asp_scorer_weights, ev) : offsetof(asp_scorer_weights, ec));
        for (int i = tid; i < F * H; i += NT) sE[i] = bf16_int(E[i]);
        for (int i = tid; i < H; i += NT) sB[i] = eb[i];
        const int nrows = var ? min(TR, d.V + 1 - tl.row0) : min(TR, d.n_static - tl.row0);
        if (tid < TR) {
            int x[F];
#pragma unroll
            for (int f = 0; f < F; ++f) x[f] = 0;
            const int r = tl.row0 + tid;
            if (tid < nrows && var && r >= 1) {
                const int32_t* MO = a.map_off + d.map_off;
                const int dp = MO[2 * r + 1] - MO[2 * r], dn = MO[2 * r + 2] - MO[2 * r + 1];
                x[0] = 32;
                x[1] = r <= d.A ? 32 : 0;
                if (r > d.A) x[2 + (r - d.A - 1) % 3] = 32;
                // degrees as saturating log codes: 16 * bit length
                auto logc = [](int v) { return min(255, 16 * (v > 0 ? 32 - __clz(v) : 0)); };
                x[5] = logc(dp);
                x[6] = logc(dn);
                x[7] = logc(dp + dn);
            } else if (tid < nrows && !var) {
                const int32_t* NO = a.ng_off + d.ng_off;
                const int32_t* NL = a.ng_lits + d.ng_lits;
                const int b = NO[r], len = NO[r + 1] - b;
                int np = 0;
                for (int q = 0; q < len; ++q) np += NL[b + q] > 0 ? 1 : 0;
                x[0] = 32;
                x[1] = len > 0 ? (32 + len / 2) / len : 0;
                x[2] = len == 1 ? 32 : 0;
                x[3] = len == 2 ? 32 : 0;
                x[4] = len == 3 ? 32 : 0;
                x[5] = len >= 4 ? 32 : 0;
                x[6] = len > 0 ? (32 * np + len / 2) / len : 0;
            }
#pragma unroll
            for (int f = 0; f < F; ++f) sX[tid][f] = x[f];
        }
        __syncthreads();
        const int row = tid >> 2, c0 = (tid & 3) * 16;
        if (row < nrows) {
            uint8_t* out = a.ws + (var ? a.hv_off[tl.inst] : a.hc_off[tl.inst]) +
                           (size_t)(tl.row0 + row) * H + c0;
            const bool zero = var && tl.row0 + row == 0;
            uint32_t pk[4] = {0u, 0u, 0u, 0u};
            for (int j = 0; j < 16; ++j) {
                long long z = sB[c0 + j];
#pragma unroll
                for (int f = 0; f < F; ++f) z += (long long)sX[row][f] * sE[f * H + c0 + j];
                const uint32_t code = zero ? 0u : (uint32_t)act(z);
                pk[j >> 2] |= code << (8 * (j & 3));
            }
            *(uint4*)out = make_uint4(pk[0], pk[1], pk[2], pk[3]);
        }
        __syncthreads();
    }
}

// Nogood update of layer l: hc = act(hc S + norm(sum hv P | hv N, |c|) + bc).
__global__ __launch_bounds__(NT) void k_nogoods(ScorerArgs a, int l) {
    HIP_DYNAMIC_SHARED(uint4, smem16);   // 16-byte aligned base for the bf16 operand rows
    const LayerLds L = carve((unsigned char*)smem16);
    const int tid = threadIdx.x;
    const size_t HH = (size_t)H * H;
    stage_t2(L.wt, wmat(a, offsetof(asp_scorer_weights, P)) + l * HH,
             wmat(a, offsetof(asp_scorer_weights, N)) + l * HH, tid);
    stage_t(L.st, wmat(a, offsetof(asp_scorer_weights, S)) + l * HH, tid);
    for (int i = tid; i < H; i += NT) L.bias[i] = wvec(a, offsetof(asp_scorer_weights, bc))[l * H + i];
    for (int t = blockIdx.x; t < a.n_ctiles; t += gridDim.x) {
        const ScorerTile tl = a.ctiles[t];
        const InstDesc& d = a.inst[tl.inst];
        const int rows = min(TR, d.n_static - tl.row0);
        const int32_t* NO = a.ng_off + d.ng_off + tl.row0;
        const int32_t* NL = a.ng_lits + d.ng_lits;
        const uint8_t* hv = a.ws + a.hv_off[tl.inst];
        uint8_t* hc = a.ws + a.hc_off[tl.inst] + (size_t)tl.row0 * H;
        for (int i = tid; i <= rows; i += NT) L.start[i] = NO[i];
        __syncthreads();
        long long tot[16];
        edge_term(L, rows, [&](int r, int q, int* sp, int* sn) {
            const int e1 = L.start[r + 1];
            for (int e = L.start[r]; e < e1; e += 2) {
                const bool two = e + 1 < e1;
                const int l0 = NL[e], l1 = two ? NL[e + 1] : 0;
                const uint4 c0 = *(const uint4*)(hv + (size_t)(l0 < 0 ? -l0 : l0) * H + 16 * q);
                const uint4 c1 = two ? *(const uint4*)(hv + (size_t)(l1 < 0 ? -l1 : l1) * H + 16 * q)
                                     : make_uint4(0u, 0u, 0u, 0u);
                if (l0 > 0) add_codes16(sp, c0); else add_codes16(sn, c0);
                if (l1 > 0) add_codes16(sp, c1); else add_codes16(sn, c1);
            }
        }, tid, tot);
        const int er = tid >> 2, part = tid & 3;
        if (er < rows) load_codes16(L.opa + er * LD + part * 16, hc + (size_t)er * H + part * 16);
        else zero16(L.opa + er * LD + part * 16);
        __syncthreads();
        finish_tile(L, rows, [&](int row) { return L.start[row + 1] - L.start[row]; }, -1, tot, hc, tid);
        __syncthreads();
    }
}

// Variable update of layer l: hv = act(hv T + norm(sum hc Q | hc R, deg v) + bv);
// the last layer also writes each atom's score hv . wo + bo.
__global__ __launch_bounds__(NT) void k_vars(ScorerArgs a, int l, int last) {
    HIP_DYNAMIC_SHARED(uint4, smem16);   // 16-byte aligned base for the bf16 operand rows
    const LayerLds L = carve((unsigned char*)smem16);
    __shared__ int sWo[H];
    const int tid = threadIdx.x;
    const size_t HH = (size_t)H * H;
    stage_t2(L.wt, wmat(a, offsetof(asp_scorer_weights, Q)) + l * HH,
             wmat(a, offsetof(asp_scorer_weights, R)) + l * HH, tid);
    stage_t(L.st, wmat(a, offsetof(asp_scorer_weights, T)) + l * HH, tid);
    for (int i = tid; i < H; i += NT) {
        L.bias[i] = wvec(a, offsetof(asp_scorer_weights, bv))[l * H + i];
        sWo[i] = wvec(a, offsetof(asp_scorer_weights, wo))[i];
    }
    const int bo = *wvec(a, offsetof(asp_scorer_weights, bo));
    for (int t = blockIdx.x; t < a.n_vtiles; t += gridDim.x) {
        const ScorerTile tl = a.vtiles[t];
        const InstDesc& d = a.inst[tl.inst];
        const int rows = min(TR, d.V + 1 - tl.row0);
        const int32_t* MO = a.map_off + d.map_off + 2 * tl.row0;
        const MapEntry* ME = a.map_ent + d.map_ids;
        const uint8_t* hc = a.ws + a.hc_off[tl.inst];
        uint8_t* hv = a.ws + a.hv_off[tl.inst] + (size_t)tl.row0 * H;
        const int nseg = 2 * rows;
        for (int i = tid; i <= nseg; i += NT) L.start[i] = MO[i];
        __syncthreads();
        long long tot[16];
        // a variable's positive literal's occurrences, then its negative's
        edge_term(L, rows, [&](int r, int q, int* sp, int* sn) {
            const int e1 = L.start[2 * r + 2], em = L.start[2 * r + 1];
            for (int e = L.start[2 * r]; e < e1; e += 2) {
                const bool two = e + 1 < e1;
                const int c0 = ME[e].id, c1 = two ? ME[e + 1].id : 0;
                const uint4 x0 = *(const uint4*)(hc + (size_t)c0 * H + 16 * q);
                const uint4 x1 = two ? *(const uint4*)(hc + (size_t)c1 * H + 16 * q)
                                     : make_uint4(0u, 0u, 0u, 0u);
                if (e < em) add_codes16(sp, x0); else add_codes16(sn, x0);
                if (e + 1 < em) add_codes16(sp, x1); else add_codes16(sn, x1);
            }
        }, tid, tot);
        const int er = tid >> 2, part = tid & 3;
        if (er < rows) load_codes16(L.opa + er * LD + part * 16, hv + (size_t)er * H + part * 16);
        else zero16(L.opa + er * LD + part * 16);
        __syncthreads();
        finish_tile(L, rows, [&](int row) { return L.start[2 * row + 2] - L.start[2 * row]; },
                    tl.row0 == 0 ? 0 : -1, tot, hv, tid);
        if (last && tid < rows) {
            const int v = tl.row0 + tid;
            if (v <= d.A) {
                const uint8_t* codes = (const uint8_t*)L.opa + tid * H;
                int s = bo;
                for (int j = 0; j < H; ++j) s += (int)codes[j] * sWo[j];
                a.atom_score[d.ascore + v] = v == 0 ? 0 : s;
            }
        }
        __syncthreads();
    }
}

// The Decision's order of an instance's rules under these scores: rule
// score descending, then rule ascending, as one ascending 64-bit key
// (complemented biased score, rule).
DEV unsigned long long score_key(int score, int j) {
    return ((unsigned long long)(~((uint32_t)score ^ 0x80000000u)) << 32) | (uint32_t)j;
}

constexpr int kSortChunk = 1024;

// rule_score[r] = atom_score[head(r)] for every headed rule of the listed
// instances, and rule_ord_sc = the (rule, head) pairs in the Decision's
// order under these scores: chunks of kSortChunk keys sorted in LDS by a
// bitonic network, then merged pairwise in global memory (each key's place
// in the merged run is its index in its own run plus the number of keys
// below it in the other run, found by binary search; keys are distinct),
// alternating between the output array and the sort buffer.
__global__ __launch_bounds__(NT) void k_rule_scores(ScorerArgs a) {
    __shared__ unsigned long long sk[kSortChunk];
    const int tid = threadIdx.x;
    const int n = a.inst_list ? a.n_inst : 1;
    for (int b = blockIdx.x; b < n; b += gridDim.x) {
        const InstDesc& d = a.inst[a.inst_list ? a.inst_list[b] : a.single];
        const int Rh = d.Rh;
        unsigned long long* A = (unsigned long long*)(a.rule_ord_sc + 2 * d.rules);
        unsigned long long* B = a.sort_tmp + d.rules;
        for (int j = tid; j < Rh; j += NT) {
            const int sc = a.atom_score[d.ascore + a.rule_head[d.rules + j]];
            a.rule_score[d.rules + j] = sc;
            A[j] = score_key(sc, j);
        }
        __syncthreads();
        for (int c0 = 0; c0 < Rh; c0 += kSortChunk) {
            const int m = min(kSortChunk, Rh - c0);
            for (int i = tid; i < kSortChunk; i += NT) sk[i] = i < m ? A[c0 + i] : ~0ull;
            __syncthreads();
            for (int k = 2; k <= kSortChunk; k <<= 1) {
                for (int jj = k >> 1; jj > 0; jj >>= 1) {
                    for (int t = tid; t < kSortChunk / 2; t += NT) {
                        const int i = 2 * jj * (t / jj) + (t % jj), p = i + jj;
                        const unsigned long long x = sk[i], y = sk[p];
                        if ((x > y) == ((i & k) == 0)) {
                            sk[i] = y;
                            sk[p] = x;
                        }
                    }
                    __syncthreads();
                }
            }
            for (int i = tid; i < m; i += NT) A[c0 + i] = sk[i];
            __syncthreads();
        }
        unsigned long long *src = A, *dst = B;
        for (int w = kSortChunk; w < Rh; w *= 2) {
            for (int i = tid; i < Rh; i += NT) {
                const int run = i / w, r0 = run * w, ps = (run & ~1) * w;
                const int o0 = (run & 1) ? r0 - w : r0 + w;          // the other run
                const int o1 = (run & 1) ? r0 : min(r0 + 2 * w, Rh);
                const unsigned long long x = src[i];
                int lo = o0, hi = o0 < o1 ? o1 : o0;                 // first key >= x in [o0, o1)
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (src[mid] < x) lo = mid + 1; else hi = mid;
                }
                dst[ps + (i - r0) + (lo - o0)] = x;
            }
            __syncthreads();
            unsigned long long* t = src;
            src = dst;
            dst = t;
        }
        // (rule, head) pairs in place of the keys
        for (int p = tid; p < Rh; p += NT) {
            const int j = (int)(uint32_t)(src[p] & 0xffffffffull);
            A[p] = ((unsigned long long)(uint32_t)a.rule_head[d.rules + j] << 32) | (uint32_t)j;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------- readout training
// Logistic regression of the readout on the last layer's codes: for every
// labelled atom v (label 1: true in the answer set found, 0: false),
// logit = sum_j (hv_j / 256) w_j + b, and the gradient of the mean binary
// cross-entropy is (sigmoid(logit) - y) (hv_j / 256, 1).  Sums go through
// float atomics in LDS, then one global atomic per workgroup and element.
__global__ __launch_bounds__(NT) void k_readout_grad(ScorerArgs a, TrainArgs t) {
    __shared__ float sg[H + 2];
    __shared__ float sw[H + 1];
    const int tid = threadIdx.x;
    if (tid < H + 2) sg[tid] = 0.f;
    if (tid < H + 1) sw[tid] = t.wb[tid];
    __syncthreads();
    for (int ti = blockIdx.x; ti < a.n_vtiles; ti += gridDim.x) {
        const ScorerTile tl = a.vtiles[ti];
        const InstDesc& d = a.inst[tl.inst];
        const int v = tl.row0 + (tid & 63);
        // four row groups of 16 columns: lanes of one row share its logit
        const int part = tid >> 6;
        float lg = 0.f, y = -1.f;
        const uint8_t* hv = a.ws + a.hv_off[tl.inst] + (size_t)v * H;
        if (v >= 1 && v <= d.A && v <= d.V) {
            const int8_t lab = t.labels[d.model + v - 1];
            if (lab >= 0) {
                y = (float)lab;
                for (int j = 0; j < H; ++j) lg += (float)hv[j] * (1.f / 256.f) * sw[j];
                lg += sw[H];
            }
        }
        if (y >= 0.f) {
            const float p = 1.f / (1.f + __expf(-lg));
            const float g = (p - y) * t.inv_n;
            for (int j = part * 16; j < part * 16 + 16; ++j)
                atomicAdd(&sg[j], g * (float)hv[j] * (1.f / 256.f));
            if (part == 0) {
                atomicAdd(&sg[H], g);
                // binary cross-entropy, stable form
                const float ce = fmaxf(lg, 0.f) - lg * y + __logf(1.f + __expf(-fabsf(lg)));
                atomicAdd(&sg[H + 1], ce * t.inv_n);
            }
        }
    }
    __syncthreads();
    if (tid < H + 2) atomicAdd(&t.grad[tid], sg[tid]);
}

// Adam step on (w, b) from the summed gradient; clears the gradient and
// records the loss of this step.
__global__ void k_readout_adam(TrainArgs t, int step) {
    const int i = threadIdx.x;
    if (i < H + 1) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float g = t.grad[i];
        t.m[i] = b1 * t.m[i] + (1.f - b1) * g;
        t.v[i] = b2 * t.v[i] + (1.f - b2) * g * g;
        const float mh = t.m[i] / (1.f - __powf(b1, (float)(step + 1)));
        const float vh = t.v[i] / (1.f - __powf(b2, (float)(step + 1)));
        t.wb[i] -= t.lr * mh / (sqrtf(vh) + eps);
    }
    __syncthreads();
    if (i == 0) t.loss[step] = t.grad[H + 1];
    __syncthreads();
    if (i < H + 2) t.grad[i] = 0.f;
}

}  // namespace

// ----------------------------------------------------------------- launchers
hipError_t launch_scorer_embed(const ScorerArgs& a, int grid, hipStream_t s) {
    if (a.n_vtiles + a.n_ctiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_embed, dim3(grid), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_scorer_nogoods(const ScorerArgs& a, int layer, int grid, hipStream_t s) {
    if (a.n_ctiles == 0) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)k_nogoods,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLayerLds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_nogoods, dim3(grid), dim3(NT), kLayerLds, s, a, layer);
    return hipGetLastError();
}

hipError_t launch_scorer_vars(const ScorerArgs& a, int layer, int grid, hipStream_t s) {
    if (a.n_vtiles == 0) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)k_vars,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLayerLds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_vars, dim3(grid), dim3(NT), kLayerLds, s, a, layer,
                       layer == ASP_SCORER_L - 1 ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_readout_train(const ScorerArgs& a, const TrainArgs& t, int steps, int grid,
                                hipStream_t s) {
    for (int k = 0; k < steps; ++k) {
        hipLaunchKernelGGL(k_readout_grad, dim3(grid), dim3(NT), 0, s, a, t);
        hipLaunchKernelGGL(k_readout_adam, dim3(1), dim3(128), 0, s, t, k);
    }
    return hipGetLastError();
}

hipError_t launch_rule_scores(const ScorerArgs& a, hipStream_t s) {
    const int n = a.inst_list ? a.n_inst : 1;
    if (n == 0) return hipSuccess;
    const int grid = n < 4096 ? n : 4096;
    hipLaunchKernelGGL(k_rule_scores, dim3(grid), dim3(NT), 0, s, a);
    return hipGetLastError();
}

}  // namespace asp
