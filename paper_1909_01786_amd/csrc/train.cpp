// train.cpp -- host side of the scorer's training (internal to libasp).
//
// Lays the training programs out as one graph (variable rows, static nogood
// rows, the literals as edges in both CSR orders), with the scorer's input
// features and the per-atom labels, in a caller-owned device workspace; then
// runs full-batch forward / backward passes and Adam steps with the kernels
// of trainer.hip.  Parameters are the float form of asp_scorer_weights
// (layout in asp.h, ASP_SCORER_NPARAM floats).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/asp.h"
#include "encode.h"
#include "train.h"
#include "trainer.h"

namespace asp {
namespace {

constexpr int H = ASP_SCORER_H, F = ASP_SCORER_F, L = ASP_SCORER_L;
constexpr int64_t HH = (int64_t)H * H;

// Offsets (floats) of each parameter group in the flat vector.
struct ParamLayout {
    int64_t Ev = 0, Ec, ev, ec, P, N, S, Q, R, T, bc, bv, wo, bo, n;
    ParamLayout() {
        int64_t o = 0;
        Ev = o; o += F * H;
        Ec = o; o += F * H;
        ev = o; o += H;
        ec = o; o += H;
        P = o; o += L * HH;
        N = o; o += L * HH;
        S = o; o += L * HH;
        Q = o; o += L * HH;
        R = o; o += L * HH;
        T = o; o += L * HH;
        bc = o; o += L * H;
        bv = o; o += L * H;
        wo = o; o += H;
        bo = o; o += 1;
        n = o;
    }
};

// Scales between integer codes and float parameters.
constexpr double kW = 128.0;       // matrix and readout codes
constexpr double kB = 131072.0;    // layer and embedding biases (2^17)
constexpr double kBo = 32768.0;    // readout bias (2^15)
constexpr float kLim[3] = {127.0f / 128.0f, 128.0f, 512.0f};   // clip per range kind

uint64_t al(uint64_t x) { return (x + 255) / 256 * 256; }

int log2ceil(int64_t n) {
    int k = 0;
    while (((int64_t)1 << k) < n) ++k;
    return k;
}

int code_L(int64_t d) {   // saturating log code of a degree: 16 * bit length
    int b = 0;
    while (d > 0) {
        ++b;
        d >>= 1;
    }
    return std::min(255, 16 * b);
}

struct Sizes {
    int64_t nv = 0, nc = 0, ne = 0, atoms = 0;
};

Sizes sizes_of(const std::vector<const HostProgram*>& progs) {
    Sizes z;
    for (auto* h : progs) {
        z.nv += h->V;
        z.nc += h->n_nogoods();
        z.ne += (int64_t)h->ng_lits.size();
        z.atoms += h->A;
    }
    return z;
}

struct WsLayout {
    uint64_t P, G, M, V, range, lim, loss, Xv, Xc, coff, cidx, voff, vidx, cscale, vscale, y;
    uint64_t Av[L + 1], Ac[L + 1], tv[3], tc[3], dv[2], dc[2];
    uint64_t total;
};

WsLayout ws_layout(const Sizes& z) {
    const ParamLayout PL;
    WsLayout W;
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t at = o;
        o = al(o + bytes);
        return at;
    };
    W.P = take(4 * PL.n);
    W.G = take(4 * PL.n);
    W.M = take(4 * PL.n);
    W.V = take(4 * PL.n);
    W.range = take(PL.n);
    W.lim = take(4 * 4);
    W.loss = take(4 * 4);
    W.Xv = take(4 * F * z.nv);
    W.Xc = take(4 * F * z.nc);
    W.coff = take(8 * (z.nc + 1));
    W.cidx = take(4 * z.ne);
    W.voff = take(8 * (z.nv + 1));
    W.vidx = take(4 * z.ne);
    W.cscale = take(4 * z.nc);
    W.vscale = take(4 * z.nv);
    W.y = take(4 * z.nv);
    for (int l = 0; l <= L; ++l) W.Av[l] = take(4 * H * z.nv);
    for (int l = 0; l <= L; ++l) W.Ac[l] = take(4 * H * z.nc);
    for (int i = 0; i < 3; ++i) W.tv[i] = take(4 * H * z.nv);
    for (int i = 0; i < 3; ++i) W.tc[i] = take(4 * H * z.nc);
    for (int i = 0; i < 2; ++i) W.dv[i] = take(4 * H * z.nv);
    for (int i = 0; i < 2; ++i) W.dc[i] = take(4 * H * z.nc);
    W.total = o;
    return W;
}

#define TRCHK(expr)                                                               \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) {                                                   \
            *err = std::string(#expr) + ": " + hipGetErrorString(e_);             \
            return ASP_E_DEVICE;                                                  \
        }                                                                         \
    } while (0)

}  // namespace

int64_t train_nparam() { return ParamLayout().n; }

int32_t train_workspace(const std::vector<const HostProgram*>& progs, uint64_t* bytes) {
    *bytes = ws_layout(sizes_of(progs)).total;
    return ASP_OK;
}

void train_quantize(const float* p, asp_scorer_weights* w) {
    const ParamLayout PL;
    auto bf = [](int code) {      // integer code as bfloat16 bits (exact for |code| <= 256)
        float f = (float)code;
        uint32_t u;
        memcpy(&u, &f, 4);
        return (uint16_t)(u >> 16);
    };
    auto q = [](double x, double scale, double lim) {
        double c = std::nearbyint(x * scale);
        return (int)std::max(-lim, std::min(lim, c));
    };
    memset(w, 0, sizeof(*w));
    for (int i = 0; i < F * H; ++i) {
        w->Ev[i] = bf(q(p[PL.Ev + i], kW, 127));
        w->Ec[i] = bf(q(p[PL.Ec + i], kW, 127));
    }
    for (int64_t i = 0; i < L * HH; ++i) {
        w->P[i] = bf(q(p[PL.P + i], kW, 127));
        w->N[i] = bf(q(p[PL.N + i], kW, 127));
        w->S[i] = bf(q(p[PL.S + i], kW, 127));
        w->Q[i] = bf(q(p[PL.Q + i], kW, 127));
        w->R[i] = bf(q(p[PL.R + i], kW, 127));
        w->T[i] = bf(q(p[PL.T + i], kW, 127));
    }
    for (int i = 0; i < H; ++i) {
        w->ev[i] = q(p[PL.ev + i], kB, 1 << 24);
        w->ec[i] = q(p[PL.ec + i], kB, 1 << 24);
        w->wo[i] = q(p[PL.wo + i], kW, 127);
    }
    for (int i = 0; i < L * H; ++i) {
        w->bc[i] = q(p[PL.bc + i], kB, 1 << 24);
        w->bv[i] = q(p[PL.bv + i], kB, 1 << 24);
    }
    w->bo = q(p[PL.bo], kBo, 1 << 24);
}

void train_dequantize(const asp_scorer_weights* w, float* p) {
    const ParamLayout PL;
    auto val = [](uint16_t b) {
        uint32_t u = (uint32_t)b << 16;
        float f;
        memcpy(&f, &u, 4);
        return f;
    };
    for (int i = 0; i < F * H; ++i) {
        p[PL.Ev + i] = (float)(val(w->Ev[i]) / kW);
        p[PL.Ec + i] = (float)(val(w->Ec[i]) / kW);
    }
    for (int64_t i = 0; i < L * HH; ++i) {
        p[PL.P + i] = (float)(val(w->P[i]) / kW);
        p[PL.N + i] = (float)(val(w->N[i]) / kW);
        p[PL.S + i] = (float)(val(w->S[i]) / kW);
        p[PL.Q + i] = (float)(val(w->Q[i]) / kW);
        p[PL.R + i] = (float)(val(w->R[i]) / kW);
        p[PL.T + i] = (float)(val(w->T[i]) / kW);
    }
    for (int i = 0; i < H; ++i) {
        p[PL.ev + i] = (float)(w->ev[i] / kB);
        p[PL.ec + i] = (float)(w->ec[i] / kB);
        p[PL.wo + i] = (float)(w->wo[i] / kW);
    }
    for (int i = 0; i < L * H; ++i) {
        p[PL.bc + i] = (float)(w->bc[i] / kB);
        p[PL.bv + i] = (float)(w->bv[i] / kB);
    }
    p[PL.bo] = (float)(w->bo / kBo);
}

int32_t train_run(const std::vector<const HostProgram*>& progs, const float* labels, float* params,
                  int32_t steps, float lr, uint8_t* ws, uint64_t ws_bytes, float* loss_out,
                  float* grad_out, hipStream_t s, std::string* err) {
    const ParamLayout PL;
    const Sizes z = sizes_of(progs);
    const WsLayout W = ws_layout(z);
    if (ws_bytes < W.total) {
        *err = "training workspace of " + std::to_string(ws_bytes) + " bytes, need " +
               std::to_string(W.total);
        return ASP_E_CAPACITY;
    }
    // ---- the graph, features, scales and labels (host, then uploaded)
    std::vector<float> Xv((size_t)(F * z.nv), 0.f), Xc((size_t)(F * z.nc), 0.f);
    std::vector<int64_t> coff((size_t)z.nc + 1), voff((size_t)z.nv + 1);
    std::vector<int32_t> cidx((size_t)z.ne), vidx((size_t)z.ne);
    std::vector<float> cscale((size_t)z.nc), vscale((size_t)z.nv), y((size_t)z.nv, -1.f);
    int64_t vb = 0, cb = 0, eb_c = 0, eb_v = 0, ab = 0, n_lab = 0;
    for (auto* h : progs) {
        const int64_t V = h->V, A = h->A, nS = h->n_nogoods();
        if ((vb + V) * 2 + 1 > INT32_MAX || (cb + nS) * 2 + 1 > INT32_MAX) {
            *err = "training graph beyond 2^30 rows";
            return ASP_E_CAPACITY;
        }
        // nogood rows: CSR by nogood, edges (variable row, sign)
        for (int64_t c = 0; c < nS; ++c) {
            const int32_t b = h->ng_off[c], e = h->ng_off[c + 1], len = e - b;
            coff[cb + c] = eb_c;
            int np = 0;
            for (int32_t q = b; q < e; ++q) {
                const int32_t l = h->ng_lits[q];
                const int64_t v = l < 0 ? -l : l;
                cidx[eb_c++] = (int32_t)(((vb + v - 1) << 1) | (l < 0 ? 1 : 0));
                np += l > 0 ? 1 : 0;
            }
            float* x = &Xc[(size_t)(cb + c) * F];
            x[0] = 32.f;
            x[1] = len > 0 ? (float)((32 + len / 2) / len) : 0.f;
            x[2] = len == 1 ? 32.f : 0.f;
            x[3] = len == 2 ? 32.f : 0.f;
            x[4] = len == 3 ? 32.f : 0.f;
            x[5] = len >= 4 ? 32.f : 0.f;
            x[6] = len > 0 ? (float)((32 * np + len / 2) / len) : 0.f;
            for (int f = 0; f < F; ++f) x[f] /= 256.f;
            cscale[cb + c] = ldexpf(1.f, -log2ceil(std::max<int64_t>(len, 1)));
        }
        // variable rows 1..V: CSR by variable from the literal map, edges
        // (nogood row, sign of the literal)
        for (int64_t v = 1; v <= V; ++v) {
            const int64_t r = vb + v - 1;
            voff[r] = eb_v;
            const int32_t p0 = h->map_off[2 * v], p1 = h->map_off[2 * v + 1],
                          p2 = h->map_off[2 * v + 2];
            for (int32_t q = p0; q < p1; ++q) vidx[eb_v++] = (int32_t)((cb + h->map_ent[q].id) << 1);
            for (int32_t q = p1; q < p2; ++q)
                vidx[eb_v++] = (int32_t)(((cb + h->map_ent[q].id) << 1) | 1);
            const int64_t dp = p1 - p0, dn = p2 - p1;
            float* x = &Xv[(size_t)r * F];
            x[0] = 32.f;
            x[1] = v <= A ? 32.f : 0.f;
            if (v > A) x[2 + (v - A - 1) % 3] = 32.f;
            x[5] = (float)code_L(dp);
            x[6] = (float)code_L(dn);
            x[7] = (float)code_L(dp + dn);
            for (int f = 0; f < F; ++f) x[f] /= 256.f;
            vscale[r] = ldexpf(1.f, -log2ceil(std::max<int64_t>(dp + dn, 1)));
            if (v <= A && labels) {
                const float lab = labels[ab + v - 1];
                if (lab >= 0.f) {
                    y[r] = lab > 1.f ? 1.f : lab;
                    ++n_lab;
                }
            }
        }
        vb += V;
        cb += nS;
        ab += A;
    }
    coff[z.nc] = eb_c;
    voff[z.nv] = eb_v;
    if (eb_c != z.ne || eb_v != z.ne) {
        *err = "literal map and nogood lists disagree";
        return ASP_E_INTERNAL;
    }
    if (n_lab == 0) {
        *err = "no labelled atom";
        return ASP_E_INVALID;
    }
    std::vector<uint8_t> range((size_t)PL.n, 0);
    for (int64_t i = PL.ev; i < PL.ev + 2 * H; ++i) range[i] = 1;
    for (int64_t i = PL.bc; i < PL.bc + 2 * L * H; ++i) range[i] = 1;
    range[PL.bo] = 2;
    auto put = [&](uint64_t off, const void* src, size_t bytes) -> hipError_t {
        if (bytes == 0) return hipSuccess;
        return hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, s);
    };
    TRCHK(put(W.P, params, 4 * PL.n));
    TRCHK(hipMemsetAsync(ws + W.M, 0, 4 * PL.n, s));
    TRCHK(hipMemsetAsync(ws + W.V, 0, 4 * PL.n, s));
    TRCHK(put(W.range, range.data(), range.size()));
    TRCHK(put(W.lim, kLim, sizeof(kLim)));
    TRCHK(put(W.Xv, Xv.data(), 4 * Xv.size()));
    TRCHK(put(W.Xc, Xc.data(), 4 * Xc.size()));
    TRCHK(put(W.coff, coff.data(), 8 * coff.size()));
    TRCHK(put(W.cidx, cidx.data(), 4 * cidx.size()));
    TRCHK(put(W.voff, voff.data(), 8 * voff.size()));
    TRCHK(put(W.vidx, vidx.data(), 4 * vidx.size()));
    TRCHK(put(W.cscale, cscale.data(), 4 * cscale.size()));
    TRCHK(put(W.vscale, vscale.data(), 4 * vscale.size()));
    TRCHK(put(W.y, y.data(), 4 * y.size()));
    TRCHK(hipStreamSynchronize(s));   // host staging vectors die here

    auto F32 = [&](uint64_t off) { return (float*)(ws + off); };
    float* Pp = F32(W.P);
    float* Gp = F32(W.G);
    const int64_t* c_off = (const int64_t*)(ws + W.coff);
    const int64_t* v_off = (const int64_t*)(ws + W.voff);
    const int32_t* c_idx = (const int32_t*)(ws + W.cidx);
    const int32_t* v_idx = (const int32_t*)(ws + W.vidx);
    const float* c_sc = F32(W.cscale);
    const float* v_sc = F32(W.vscale);
    const int64_t nv = z.nv, nc = z.nc;

    // one forward and backward pass: loss into ws loss[0], gradient into G
    auto pass = [&]() -> int32_t {
        TRCHK(hipMemsetAsync(Gp, 0, 4 * PL.n, s));
        TRCHK(hipMemsetAsync(ws + W.loss, 0, 16, s));
        TRCHK(tr_embed_fwd(F32(W.Xv), Pp + PL.Ev, Pp + PL.ev, F32(W.Av[0]), nv, s));
        TRCHK(tr_embed_fwd(F32(W.Xc), Pp + PL.Ec, Pp + PL.ec, F32(W.Ac[0]), nc, s));
        for (int l = 0; l < L; ++l) {
            float *MP = F32(W.tv[0]), *MN = F32(W.tv[1]), *Uv = F32(W.tv[2]);
            float *MQ = F32(W.tc[0]), *MR = F32(W.tc[1]), *Uc = F32(W.tc[2]);
            TRCHK(tr_mm(F32(W.Av[l]), Pp + PL.P + l * HH, 0, MP, nv, 1.f, 0, s));
            TRCHK(tr_mm(F32(W.Av[l]), Pp + PL.N + l * HH, 0, MN, nv, 1.f, 0, s));
            TRCHK(tr_mm(F32(W.Ac[l]), Pp + PL.S + l * HH, 0, Uc, nc, 1.f, 0, s));
            TRCHK(tr_segsum(c_off, c_idx, MP, MN, nullptr, c_sc, Uc, nc, 1, s));
            TRCHK(tr_act_fwd(Uc, Pp + PL.bc + l * H, F32(W.Ac[l + 1]), nc, s));
            TRCHK(tr_mm(F32(W.Ac[l + 1]), Pp + PL.Q + l * HH, 0, MQ, nc, 1.f, 0, s));
            TRCHK(tr_mm(F32(W.Ac[l + 1]), Pp + PL.R + l * HH, 0, MR, nc, 1.f, 0, s));
            TRCHK(tr_mm(F32(W.Av[l]), Pp + PL.T + l * HH, 0, Uv, nv, 1.f, 0, s));
            TRCHK(tr_segsum(v_off, v_idx, MQ, MR, nullptr, v_sc, Uv, nv, 1, s));
            TRCHK(tr_act_fwd(Uv, Pp + PL.bv + l * H, F32(W.Av[l + 1]), nv, s));
        }
        int cur = 0;
        TRCHK(tr_readout(F32(W.Av[L]), F32(W.y), Pp + PL.wo, Pp + PL.bo, F32(W.dv[cur]),
                         Gp + PL.wo, Gp + PL.bo, F32(W.loss), nv, 1.f / (float)n_lab, s));
        TRCHK(hipMemsetAsync(ws + W.dc[cur], 0, 4 * (size_t)H * nc, s));
        for (int l = L - 1; l >= 0; --l) {
            const int nxt = 1 - cur;
            float *dAv1 = F32(W.dv[cur]), *dAc1 = F32(W.dc[cur]);
            float *dAv0 = F32(W.dv[nxt]), *dAc0 = F32(W.dc[nxt]);
            float *GP = F32(W.tv[0]), *GN = F32(W.tv[1]), *gv = F32(W.tv[2]);
            float *GQ = F32(W.tc[0]), *GR = F32(W.tc[1]), *gc = F32(W.tc[2]);
            // variable update of layer l
            TRCHK(tr_act_bwd(dAv1, F32(W.Av[l + 1]), gv, Gp + PL.bv + l * H, nv, s));
            TRCHK(tr_mm_tn(F32(W.Av[l]), gv, Gp + PL.T + l * HH, nv, s));
            TRCHK(tr_mm(gv, Pp + PL.T + l * HH, 1, dAv0, nv, 1.f, 0, s));
            TRCHK(tr_segsum(c_off, c_idx, gv, nullptr, v_sc, nullptr, GQ, nc, 0, s));
            TRCHK(tr_segsum(c_off, c_idx, nullptr, gv, v_sc, nullptr, GR, nc, 0, s));
            TRCHK(tr_mm_tn(F32(W.Ac[l + 1]), GQ, Gp + PL.Q + l * HH, nc, s));
            TRCHK(tr_mm_tn(F32(W.Ac[l + 1]), GR, Gp + PL.R + l * HH, nc, s));
            TRCHK(tr_mm(GQ, Pp + PL.Q + l * HH, 1, dAc1, nc, 1.f, 1, s));
            TRCHK(tr_mm(GR, Pp + PL.R + l * HH, 1, dAc1, nc, 1.f, 1, s));
            // nogood update of layer l
            TRCHK(tr_act_bwd(dAc1, F32(W.Ac[l + 1]), gc, Gp + PL.bc + l * H, nc, s));
            TRCHK(tr_mm_tn(F32(W.Ac[l]), gc, Gp + PL.S + l * HH, nc, s));
            TRCHK(tr_mm(gc, Pp + PL.S + l * HH, 1, dAc0, nc, 1.f, 0, s));
            TRCHK(tr_segsum(v_off, v_idx, gc, nullptr, c_sc, nullptr, GP, nv, 0, s));
            TRCHK(tr_segsum(v_off, v_idx, nullptr, gc, c_sc, nullptr, GN, nv, 0, s));
            TRCHK(tr_mm_tn(F32(W.Av[l]), GP, Gp + PL.P + l * HH, nv, s));
            TRCHK(tr_mm_tn(F32(W.Av[l]), GN, Gp + PL.N + l * HH, nv, s));
            TRCHK(tr_mm(GP, Pp + PL.P + l * HH, 1, dAv0, nv, 1.f, 1, s));
            TRCHK(tr_mm(GN, Pp + PL.N + l * HH, 1, dAv0, nv, 1.f, 1, s));
            cur = nxt;
        }
        // embeddings
        float *gv = F32(W.tv[2]), *gc = F32(W.tc[2]);
        TRCHK(tr_act_bwd(F32(W.dv[cur]), F32(W.Av[0]), gv, Gp + PL.ev, nv, s));
        TRCHK(tr_embed_bwd(F32(W.Xv), gv, Gp + PL.Ev, nv, s));
        TRCHK(tr_act_bwd(F32(W.dc[cur]), F32(W.Ac[0]), gc, Gp + PL.ec, nc, s));
        TRCHK(tr_embed_bwd(F32(W.Xc), gc, Gp + PL.Ec, nc, s));
        return ASP_OK;
    };

    if (steps == 0) {
        int32_t rc = pass();
        if (rc) return rc;
        float loss = 0.f;
        TRCHK(hipMemcpyAsync(&loss, ws + W.loss, 4, hipMemcpyDeviceToHost, s));
        if (grad_out) TRCHK(hipMemcpyAsync(grad_out, Gp, 4 * PL.n, hipMemcpyDeviceToHost, s));
        TRCHK(hipStreamSynchronize(s));
        if (loss_out) loss_out[0] = loss;
        return ASP_OK;
    }
    for (int32_t t = 1; t <= steps; ++t) {
        int32_t rc = pass();
        if (rc) return rc;
        if (loss_out)
            TRCHK(hipMemcpyAsync(loss_out + (t - 1), ws + W.loss, 4, hipMemcpyDeviceToHost, s));
        TRCHK(tr_adam(Pp, Gp, F32(W.M), F32(W.V), PL.n, lr, t, ws + W.range, F32(W.lim), s));
    }
    TRCHK(hipMemcpyAsync(params, Pp, 4 * PL.n, hipMemcpyDeviceToHost, s));
    if (grad_out) TRCHK(hipMemcpyAsync(grad_out, Gp, 4 * PL.n, hipMemcpyDeviceToHost, s));
    TRCHK(hipStreamSynchronize(s));
    return ASP_OK;
}

}  // namespace asp
