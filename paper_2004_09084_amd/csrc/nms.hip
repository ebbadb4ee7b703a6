// Learned decoder of libqcmet (not in the paper): normalized/offset min-sum
// over the same layered schedule as the sum-product decoder, with weights
// alpha, beta per (iteration, base row, target edge type).  Forward layer
// update, early-termination bookkeeping, binary cross-entropy loss, reverse
// layer sweep and the optimizer step, all on the GPU.
//
// Min-sum check update (per check m of base row i in sweep t, target edge e):
//   mu_e = min_{e' != e} |q_e'|           (ties: the lowest column wins)
//   r_e  = (-1)^{s ^ xor_{e'!=e}[q_e' < 0]} * alpha[t][i][tau_e] * max(mu_e - beta[t][i][tau_e], 0)
// tau_e = 0 for an edge in a column of degree >= 2, 1 for the degree-1 edge.
// The minimum saturates at 30, the sum-product clip level (iterated min-sum
// messages otherwise grow without bound and overflow); a check with a single
// edge sees an empty minimum, read as 30.
// The degree-1 edge's q is its channel LLR at every visit (its variable has
// this check only), so |LLR_d| and s ^ [LLR_d < 0] sit in K; its own message
// only reaches the output APP_d = LLR_d + r_d, formed when requested.
#include "device_common.h"
#include "qcmet_internal.h"

namespace {

using namespace qmdev;

// bound of the reverse-sweep adjoints (dLoss/dAPP, dLoss/dr)
constexpr float kAdjointMax = 1e30f;

constexpr float kInf = __builtin_inff();

typedef const __attribute__((address_space(4))) float ConstF;

// two smallest (value, position) pairs in lexicographic order
struct Min2 {
    float m1, m2;
    int p1, p2;
    __device__ __forceinline__ void init() {
        m1 = m2 = kInf;
        p1 = p2 = -1;
    }
    // branch-free (selects), so that loads after an insertion are not held
    // behind a divergent branch on the inserted value
    __device__ __forceinline__ void insert(float v, int p) {
        const bool lt1 = (v < m1) | ((v == m1) & (p < p1));
        const bool lt2 = (v < m2) | ((v == m2) & (p < p2));
        const float nm2 = lt1 ? m1 : (lt2 ? v : m2);
        const int np2 = lt1 ? p1 : (lt2 ? p : p2);
        m1 = lt1 ? v : m1;
        p1 = lt1 ? p : p1;
        m2 = nm2;
        p2 = np2;
    }
    // exclusive minimum for the edge at position p, saturated at 30 (also
    // when p is the only edge)
    __device__ __forceinline__ float excl(int p) const {
        const float mu = (p == p1) ? m2 : m1;
        return fminf(mu, QM_X_HI);
    }
    // the position that attains the exclusive minimum for p, or -1 if the
    // set is empty or the saturation is active (no gradient flows then)
    __device__ __forceinline__ int excl_arg(int p) const {
        const float mu = (p == p1) ? m2 : m1;
        return mu > QM_X_HI ? -1 : ((p == p1) ? p2 : p1);
    }
};

__device__ __forceinline__ float nms_msg(bool neg, float alpha, float beta, float mu) {
    const float mag = alpha * fmaxf(mu - beta, 0.0f);
    return neg ? -mag : mag;
}

__device__ __forceinline__ float dabs(float q) { return q > 0.0f ? 1.0f : (q < 0.0f ? -1.0f : 0.0f); }

// device-side buffer resources of the min-sum kernels
struct NmsDev {
    __amdgpu_buffer_rsrc_t rAd, rQ, rgA, rgR, rgAd;
    bool q_on;
};

// --------------------------------------------------------------- forward --
template <int D, int FPL>
__device__ __forceinline__ void check_nms(const LaneCtx &c, ConstRowDesc *rd, const NmsLayerArgs &na,
                                          const NmsDev &nd, int tile) {
    const uint32_t col_bytes = c.colw * 4u;
    const uint32_t vo4 = c.node * 4u;
    const int row = rd->row;
    const uint32_t row_so = (uint32_t)row * col_bytes;
    const int d1col = rd->d1col, d1shift = rd->d1shift, d1pos = rd->d1pos;
    const bool has_d1 = d1col >= 0;
    int sh[D > 0 ? D : 1], pos[D > 0 ? D : 1];
    uint32_t col_so[D > 0 ? D : 1], ent_so[D > 0 ? D : 1];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        sh[j] = rd->shift[j];
        col_so[j] = (uint32_t)rd->col[j] * col_bytes;
        ent_so[j] = (uint32_t)rd->ent[j] * col_bytes;
        pos[j] = j + ((has_d1 && j >= d1pos) ? 1 : 0);
    }
    ConstF *w = (ConstF *)na.W + row * 4;
    const float a1 = w[0], b1 = w[1], a2 = w[2], b2 = w[3];

    // frames still decoding: the tile's mask (one scalar load; a tile with
    // none exits as a whole), so no per-lane flag load is waited for before
    // the first data load
    bool live[FPL];
    const uint64_t tm = na.tmask ? ((const __attribute__((address_space(4))) uint64_t *)na.tmask)[tile] : ~0ull;
    if (tm == 0ull) return;
    const int fl0 = (int)(c.node & ((1u << c.ftl) - 1u));
#pragma unroll
    for (int f = 0; f < FPL; ++f) live[f] = ((tm >> (fl0 + f)) & 1ull) != 0ull;

    float kap[FPL];
    bload_f32<FPL>(c.rK, vo4, row_so, kap);
    // the degree-1 APP inputs, loaded here so they are not a round trip of
    // their own at the end
    const bool form_d1 = c.last && has_d1;
    float lam[FPL];
    if (form_d1) bload_f32<FPL>(c.rA, shifted_off(c, d1shift), (uint32_t)d1col * col_bytes, lam);
    float q[D > 0 ? D : 1][FPL], av[D > 0 ? D : 1][FPL], rv[D > 0 ? D : 1][FPL];
    uint32_t aoff[D > 0 ? D : 1];
    // every load of the check first, then the arithmetic (the two smallest
    // (value, position) pairs do not depend on the insertion order)
#pragma unroll
    for (int j = 0; j < D; ++j) {
        aoff[j] = shifted_off(c, sh[j]);
        bload_f32<FPL>(c.rA, aoff[j], col_so[j], av[j]);
        bload_f32<FPL>(c.rR, vo4, ent_so[j], rv[j]);
    }
    bool neg[FPL];
    Min2 mn[FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) {
        neg[f] = (int32_t)__float_as_uint(kap[f]) < 0;
        mn[f].init();
        if (has_d1) mn[f].insert(fabsf(kap[f]), d1pos);
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            q[j][f] = av[j][f] - rv[j][f];
            neg[f] = neg[f] != (q[j][f] < 0.0f);
            mn[f].insert(fabsf(q[j][f]), pos[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
        float rm[FPL], an[FPL];
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            const float r = nms_msg(neg[f] != (q[j][f] < 0.0f), a1, b1, mn[f].excl(pos[j]));
            rm[f] = live[f] ? r : rv[j][f];
            an[f] = live[f] ? q[j][f] + r : av[j][f];
        }
        if (nd.q_on) bstore_f32<FPL>(nd.rQ, vo4, ent_so[j], q[j]);
        bstore_f32<FPL>(c.rR, vo4, ent_so[j], rm);
        bstore_f32<FPL>(c.rA, aoff[j], col_so[j], an);
    }
    if (form_d1) {
        float out[FPL];
        bool all = true;
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            // sign: s ^ xor over the degree>=2 edges = neg ^ [lam < 0]
            const float r = nms_msg(neg[f] != (lam[f] < 0.0f), a2, b2, mn[f].excl(d1pos));
            out[f] = lam[f] + r;
            all = all && live[f];
        }
        // a stopped frame keeps its degree-1 APPs: only live frames store
        if (all) {
            bstore_f32<FPL>(nd.rAd, vo4, row_so, out);
        } else {
#pragma unroll
            for (int f = 0; f < FPL; ++f)
                if (live[f]) {
                    const float one[1] = {out[f]};
                    bstore_f32<1>(nd.rAd, vo4 + 4u * (uint32_t)f, row_so, one);
                }
        }
    }
}

template <int D, int FPL>
__device__ __forceinline__ void dispatch_nms(int d, const LaneCtx &c, ConstRowDesc *rd, const NmsLayerArgs &na,
                                             const NmsDev &nd, int tile) {
    if constexpr (D >= 0) {
        if (d == D) {
            check_nms<D, FPL>(c, rd, na, nd, tile);
            return;
        }
        dispatch_nms<D - 1, FPL>(d, c, rd, na, nd, tile);
    }
}

__device__ __forceinline__ bool lane_setup(const LayerArgs &a, int b, int fpll, LaneCtx &c, int &tile, int &rs,
                                           int &chunk) {
    tile = b % a.ntiles;
    const int rest = b / a.ntiles;
    chunk = rest % a.chunks;
    rs = rest / a.chunks;
    c.Z = a.Z;
    c.ftl = a.ft_log2;
    c.last = a.last;
    const int lpl = c.ftl - fpll;
    const int idx = chunk * (int)blockDim.x + (int)threadIdx.x;
    const bool valid = idx < (c.Z << lpl);
    const int id = valid ? idx : 0;
    c.k = id >> lpl;
    c.node = ((uint32_t)c.k << c.ftl) + ((uint32_t)(id & ((1 << lpl) - 1)) << fpll);
    c.colw = (uint32_t)c.Z << c.ftl;
    c.rA = make_rsrc(a.A + (int64_t)tile * a.strideA, (uint32_t)(a.strideA * 4));
    c.rR = make_rsrc(static_cast<char *>(a.R) + (int64_t)tile * a.strideR * 4, (uint32_t)(a.strideR * 4));
    c.rK = make_rsrc(a.K + (int64_t)tile * a.strideK, (uint32_t)(a.strideK * 4));
    return valid;
}

template <int MAXD, int FPL>
__global__ void __launch_bounds__(256) k_nms_layer(const NmsLayerArgs na) {
    LaneCtx c;
    int tile, rs, chunk;
    if (!lane_setup(na.L, (int)blockIdx.x, LogOf<FPL>::v, c, tile, rs, chunk)) return;
    NmsDev nd;
    nd.rAd = make_rsrc(na.Ad + (int64_t)tile * na.L.strideK, (uint32_t)(na.L.strideK * 4));
    nd.q_on = na.Q != nullptr;
    nd.rQ = make_rsrc(na.Q ? na.Q + (int64_t)tile * na.L.strideR : na.Ad, nd.q_on ? (uint32_t)(na.L.strideR * 4) : 0u);
    ConstRowDesc *rd = as_const(na.L.rows + rs);
    dispatch_nms<MAXD, FPL>(rd->d, c, rd, na, nd, tile);
}

// K for min-sum: |LLR_d| with sign s ^ [LLR_d < 0] (rows without a degree-1
// column: +inf magnitude, never a minimum; sign s)
__global__ void __launch_bounds__(256) k_nms_kappa(const float *__restrict__ A, const uint8_t *__restrict__ Sil,
                                                   float *__restrict__ K, const RowDesc *rows, int Z, int ftl,
                                                   int ntiles, int chunks, int64_t strideA, int64_t strideM) {
    const int b = blockIdx.x;
    const int tile = b % ntiles;
    const int rest = b / ntiles;
    const int chunk = rest % chunks;
    const int rs = rest / chunks;
    const int idx = chunk * (int)blockDim.x + (int)threadIdx.x;
    if (idx >= (Z << ftl)) return;
    const int k = idx >> ftl;
    const int fl = idx & ((1 << ftl) - 1);
    ConstRowDesc *rd = as_const(rows + rs);
    const int moff = ((rd->row * Z + k) << ftl) + fl;
    uint32_t neg = Sil[(int64_t)tile * strideM + moff] & 1u;
    float mag = kInf;
    if (rd->d1col >= 0) {
        int v = k + rd->d1shift;
        v = v >= Z ? v - Z : v;
        const float lam = A[(int64_t)tile * strideA + (((rd->d1col * Z + v) << ftl) + fl)];
        mag = fabsf(lam);
        neg ^= (uint32_t)(lam < 0.0f);
    }
    K[(int64_t)tile * strideM + moff] = with_sign(mag, neg);
}

// to_A: A[d1col][(k + a) mod Z] = Ad[row][k] (the degree-1 APPs enter the
// variable array for the final outputs); else Ad = the channel LLRs.  A lane
// moves V adjacent frames of one check (V divides FT).
template <int V>
__global__ void __launch_bounds__(256) k_commit_d1(float *__restrict__ A, float *__restrict__ Ad, int to_A,
                                                   const RowDesc *rows, int Z, int ftl, int ntiles, int chunks,
                                                   int64_t strideA, int64_t strideM) {
    typedef float vec __attribute__((ext_vector_type(V)));
    const int b = blockIdx.x;
    const int tile = b % ntiles;
    const int rest = b / ntiles;
    const int chunk = rest % chunks;
    const int rs = rest / chunks;
    const int idx = (chunk * (int)blockDim.x + (int)threadIdx.x) * V;
    if (idx >= (Z << ftl)) return;
    ConstRowDesc *rd = as_const(rows + rs);
    if (rd->d1col < 0) return;
    const int k = idx >> ftl;
    const int fl = idx & ((1 << ftl) - 1);
    int v = k + rd->d1shift;
    v = v >= Z ? v - Z : v;
    vec *pa = reinterpret_cast<vec *>(A + (int64_t)tile * strideA + (((rd->d1col * Z + v) << ftl) + fl));
    vec *pd = reinterpret_cast<vec *>(Ad + (int64_t)tile * strideM + (((rd->row * Z + k) << ftl) + fl));
    if (to_A)
        *pa = *pd;
    else
        *pd = *pa;
}

// per-tile live masks from the per-frame flags: one ballot per wave, the
// first lane of each tile's frames stores (FT <= 64 divides the wave)
__device__ __forceinline__ void store_tile_masks(bool live, int f, int Fpad, int ftl, uint64_t *tmask) {
    const uint64_t b = __ballot(live);
    const int FT = 1 << ftl;
    const int lane = (int)(threadIdx.x & 63u);
    const uint64_t mask = FT >= 64 ? ~0ull : (1ull << FT) - 1ull;
    if (f < Fpad && (f & (FT - 1)) == 0) tmask[f >> ftl] = (b >> (lane & ~(FT - 1))) & mask;
}

__global__ void k_tile_masks(const uint32_t *act, uint64_t *tmask, int Fpad, int ftl) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    store_tile_masks(f < Fpad && act[f] != 0u, f, Fpad, ftl, tmask);
}

// after a syndrome pass: frames that became valid stop (iterations = done)
__global__ void k_et_update(uint32_t *fail, uint32_t *act, uint64_t *tmask, int32_t *iters, int Fpad, int ftl,
                            int done) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    bool live = false;
    if (f < Fpad) {
        live = act[f] != 0u;
        if (live && fail[f] == 0u) {
            live = false;
            act[f] = 0u;
            iters[f] = done;
        }
        fail[f] = 0u;
    }
    store_tile_masks(live, f, Fpad, ftl, tmask);
}

__global__ void k_et_final(const uint32_t *act, int32_t *iters, int Fpad, int T) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < Fpad && act[f]) iters[f] = T;
}

// ------------------------------------------------------------------ loss --
// deterministic block sum of one float (wave shuffles, then LDS in wave order)
__device__ __forceinline__ float block_sum(float v, float *lds) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    float s = 0.0f;
    if (threadIdx.x == 0)
        for (int i = 0; i < nw; ++i) s += lds[i];
    __syncthreads();
    return s;
}

// binary cross-entropy of the current APPs: loss = sum softplus(-(1-2x) APP)
// (scaled by inv_norm at the end: 1/(F n), divided by T for one term of a
// loss over T sweeps); dL/dAPP = -(1-2x) sigmoid(-(1-2x) APP) * inv_norm.
// Items: (tile, unit, chunk of 256 lanes), unit < ncols a column whose APPs
// are in A, else a row whose degree-1 APPs are in Ad; a lane takes V
// adjacent frames of one node.  A bounded grid strides over the items in a
// fixed assignment and each workgroup leaves one partial sum, so the loss
// is run-to-run identical.
// softplus(u) = max(u, 0) + log1p(e) and sigmoid(u) share e = e^-|u| (the
// hardware base-2 exponential); log1p(e) is its series below 2^-6 (error
// under e^5 / 5) and the hardware logarithm of 1 + e above.
__device__ __forceinline__ void bce_term(float app, bool bit, float inv, float &l, float &g) {
    constexpr float kLog2e = 1.44269504088896341f, kLn2 = 0.693147180559945309f;
    const float u = bit ? app : -app;  // -(1 - 2x) APP
    const float e = __builtin_amdgcn_exp2f(-fabsf(u) * kLog2e);
    const float ser = e * (1.0f - e * (0.5f - e * (0.33333333f - 0.25f * e)));
    const float lp = e < 0x1p-6f ? ser : __builtin_amdgcn_logf(1.0f + e) * kLn2;
    l = fmaxf(u, 0.0f) + lp;  // softplus(u)
    const float r = __builtin_amdgcn_rcpf(1.0f + e);
    const float sg = u >= 0.0f ? r : e * r;  // sigmoid(u)
    g = (bit ? sg : -sg) * inv;              // d softplus(u) / d APP
}

template <int V>
__device__ __forceinline__ void bce_lanes(const float *__restrict__ src, const uint8_t *__restrict__ xs,
                                          float *__restrict__ dst, bool (&real)[V], float inv, float &l) {
    float a[V], g[V];
    bool bit[V];
    if constexpr (V == 4) {
        const float4 av = *reinterpret_cast<const float4 *>(src);
        const uchar4 xv = *reinterpret_cast<const uchar4 *>(xs);
        a[0] = av.x; a[1] = av.y; a[2] = av.z; a[3] = av.w;
        bit[0] = xv.x != 0; bit[1] = xv.y != 0; bit[2] = xv.z != 0; bit[3] = xv.w != 0;
    } else {
        a[0] = src[0];
        bit[0] = xs[0] != 0;
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
        float li, gi;
        bce_term(a[v], bit[v], inv, li, gi);
        g[v] = real[v] ? gi : 0.0f;
        if (real[v]) l += li;
    }
    if constexpr (V == 4) *reinterpret_cast<float4 *>(dst) = make_float4(g[0], g[1], g[2], g[3]);
    else dst[0] = g[0];
}

template <int V>
__global__ void __launch_bounds__(256) k_bce(const float *__restrict__ A, const float *__restrict__ Ad,
                                             const uint8_t *__restrict__ X, float *__restrict__ gA,
                                             float *__restrict__ gAd, float *__restrict__ part,
                                             const int32_t *cols, int ncols, const RowDesc *rows, int mb, int Z,
                                             int ftl, int ntiles, int chunks, int64_t strideA, int64_t strideM,
                                             int F, float inv_norm) {
    __shared__ float lds[8];
    const int FT = 1 << ftl;
    // item arithmetic in 32 bits (the launcher checks the item count)
    const uint32_t items = (uint32_t)ntiles * (uint32_t)chunks * (uint32_t)(ncols + mb);
    const int lanes = (Z << ftl) / V;  // lanes of one item
    float l = 0.0f;
#pragma unroll 2
    for (uint32_t b = blockIdx.x; b < items; b += gridDim.x) {
        const int tile = (int)(b % (uint32_t)ntiles);
        const uint32_t rest = b / (uint32_t)ntiles;
        const int chunk = (int)(rest % (uint32_t)chunks);
        const int unit = (int)(rest / (uint32_t)chunks);
        const int idx = chunk * (int)blockDim.x + (int)threadIdx.x;
        if (idx >= lanes) continue;
        const int e0 = idx * V;  // k * FT + first frame of the lane
        const int k = e0 >> ftl;
        const int fl = e0 & (FT - 1);
        bool real[V];
#pragma unroll
        for (int v = 0; v < V; ++v) real[v] = tile * FT + fl + v < F;
        if (unit < ncols) {
            const int64_t o = (int64_t)tile * strideA + (((int64_t)cols[unit] * Z) << ftl) + e0;
            bce_lanes<V>(A + o, X + o, gA + o, real, inv_norm, l);
        } else {
            ConstRowDesc *rd = as_const(rows + (unit - ncols));
            if (rd->d1col < 0) continue;
            int v = k + rd->d1shift;
            v = v >= Z ? v - Z : v;
            const int64_t od = (int64_t)tile * strideM + (((int64_t)rd->row * Z) << ftl) + e0;
            const int64_t ox = (int64_t)tile * strideA + ((((int64_t)rd->d1col * Z + v) << ftl) + fl);
            bce_lanes<V>(Ad + od, X + ox, gAd + od, real, inv_norm, l);
        }
    }
    const float s = block_sum(l, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// *out = sum(part) * scale, or *out += that (accumulate: a loss with one term
// per sweep, added in sweep order)
__global__ void k_sum_parts(const float *part, int n, float scale, int accumulate, float *out) {
    __shared__ float lds[8];
    float v = 0.0f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
    const float s = block_sum(v, lds);
    if (threadIdx.x == 0) *out = (accumulate ? *out : 0.0f) + s * scale;
}

// -------------------------------------------------------------- backward --
// Reverse of one layer of sweep t.  With q recorded by the recompute pass,
// per check: APP_new = q + r_new gives dq = dAPP and dr = dAPP + dR (what r's
// later use as r_old sent back); r = sg alpha relu(mu - beta) gives
// dalpha += dr sg relu(.), and where mu > beta: dbeta -= dr sg alpha and
// dq[argmin] += dr sg alpha sign(q[argmin]); then dAPP_old = dq, dR_old = -dq.
// The degree-1 edge is a target only in the last sweep (its message reaches
// the loss there); gradients into its q stop at the channel LLR.
template <int D, int FPL>
__device__ __forceinline__ void check_nms_bwd(const LaneCtx &c, ConstRowDesc *rd, const NmsBwdArgs &ba,
                                              const NmsDev &nd, bool valid, float acc[4], int &clamped) {
    if (!valid) return;
    const uint32_t col_bytes = c.colw * 4u;
    const uint32_t vo4 = c.node * 4u;
    const int row = rd->row;
    const uint32_t row_so = (uint32_t)row * col_bytes;
    const int d1col = rd->d1col, d1pos = rd->d1pos, d1shift = rd->d1shift;
    const bool has_d1 = d1col >= 0;
    int sh[D > 0 ? D : 1], pos[D > 0 ? D : 1];
    uint32_t col_so[D > 0 ? D : 1], ent_so[D > 0 ? D : 1];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        sh[j] = rd->shift[j];
        col_so[j] = (uint32_t)rd->col[j] * col_bytes;
        ent_so[j] = (uint32_t)rd->ent[j] * col_bytes;
        pos[j] = j + ((has_d1 && j >= d1pos) ? 1 : 0);
    }
    ConstF *w = (ConstF *)ba.W + row * 4;
    const float a1 = w[0], b1 = w[1], a2 = w[2], b2 = w[3];

    float kap[FPL];
    bload_f32<FPL>(c.rK, vo4, row_so, kap);
    bool neg[FPL];
    Min2 mn[FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) {
        neg[f] = (int32_t)__float_as_uint(kap[f]) < 0;
        mn[f].init();
        if (has_d1) mn[f].insert(fabsf(kap[f]), d1pos);
    }
    float q[D > 0 ? D : 1][FPL], gq[D > 0 ? D : 1][FPL], gr[D > 0 ? D : 1][FPL];
    uint32_t aoff[D > 0 ? D : 1];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        aoff[j] = shifted_off(c, sh[j]);
        float ga[FPL], gro[FPL];
        bload_f32<FPL>(nd.rQ, vo4, ent_so[j], q[j]);
        bload_f32<FPL>(nd.rgA, aoff[j], col_so[j], ga);
        // a term's own sweep is the first reverse sweep of its window: no
        // later sweep has sent anything back through these messages yet
        if (c.last) {
#pragma unroll
            for (int f = 0; f < FPL; ++f) gro[f] = 0.0f;
        } else {
            bload_f32<FPL>(nd.rgR, vo4, ent_so[j], gro);
        }
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            neg[f] = neg[f] != (q[j][f] < 0.0f);
            mn[f].insert(fabsf(q[j][f]), pos[j]);
            gq[j][f] = ga[f];
            gr[j][f] = ga[f] + gro[f];
        }
    }
    float G1[FPL], G2[FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) G1[f] = G2[f] = 0.0f;
    // type-1 targets
#pragma unroll
    for (int j = 0; j < D; ++j) {
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            const float sg = (neg[f] != (q[j][f] < 0.0f)) ? -1.0f : 1.0f;
            const int arg = mn[f].excl_arg(pos[j]);
            const float z = mn[f].excl(pos[j]) - b1;
            acc[0] += gr[j][f] * sg * fmaxf(z, 0.0f);
            if (z > 0.0f) {
                const float gz = gr[j][f] * sg * a1;
                acc[1] -= gz;
                if (arg >= 0) {
                    if (arg == mn[f].p1) G1[f] += gz;
                    else G2[f] += gz;
                }
            }
        }
    }
    // degree-1 target (last sweep only)
    if (c.last && has_d1) {
        const uint32_t off = shifted_off(c, d1shift);
        float lam[FPL], gd[FPL];
        bload_f32<FPL>(c.rA, off, (uint32_t)d1col * col_bytes, lam);
        bload_f32<FPL>(nd.rgAd, vo4, row_so, gd);
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            const float sg = (neg[f] != (lam[f] < 0.0f)) ? -1.0f : 1.0f;
            const int arg = mn[f].excl_arg(d1pos);
            const float z = mn[f].excl(d1pos) - b2;
            acc[2] += gd[f] * sg * fmaxf(z, 0.0f);
            if (z > 0.0f) {
                const float gz = gd[f] * sg * a2;
                acc[3] -= gz;
                if (arg >= 0) {
                    if (arg == mn[f].p1) G1[f] += gz;
                    else G2[f] += gz;
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
        float ga[FPL], gro[FPL];
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            float g = gq[j][f];
            if (pos[j] == mn[f].p1) g += G1[f] * dabs(q[j][f]);
            if (pos[j] == mn[f].p2) g += G2[f] * dabs(q[j][f]);
            // adjoints can grow geometrically over many reverse sweeps; bound
            // them well inside float32 so that no inf (and no inf - inf)
            // arises, and count every component the bound changes
            clamped += (fabsf(g) > kAdjointMax) ? 1 : 0;
            g = fminf(fmaxf(g, -kAdjointMax), kAdjointMax);
            ga[f] = g;
            gro[f] = -g;
        }
        bstore_f32<FPL>(nd.rgA, aoff[j], col_so[j], ga);
        bstore_f32<FPL>(nd.rgR, vo4, ent_so[j], gro);
    }
}

template <int D, int FPL>
__device__ __forceinline__ void dispatch_nms_bwd(int d, const LaneCtx &c, ConstRowDesc *rd, const NmsBwdArgs &ba,
                                                 const NmsDev &nd, bool valid, float acc[4], int &clamped) {
    if constexpr (D >= 0) {
        if (d == D) {
            check_nms_bwd<D, FPL>(c, rd, ba, nd, valid, acc, clamped);
            return;
        }
        dispatch_nms_bwd<D - 1, FPL>(d, c, rd, ba, nd, valid, acc, clamped);
    }
}

template <int MAXD, int FPL>
__global__ void __launch_bounds__(256) k_nms_bwd(const NmsBwdArgs ba) {
    __shared__ float lds[8];
    LaneCtx c;
    int tile, rs, chunk;
    const bool valid = lane_setup(ba.L, (int)blockIdx.x, LogOf<FPL>::v, c, tile, rs, chunk);
    const int64_t sA = ba.L.strideA, sR = ba.L.strideR, sM = ba.L.strideK;
    NmsDev nd;
    nd.q_on = true;
    nd.rAd = make_rsrc(ba.gAd, 0u);
    nd.rQ = make_rsrc(ba.Q + (int64_t)tile * sR, (uint32_t)(sR * 4));
    nd.rgA = make_rsrc(ba.gA + (int64_t)tile * sA, (uint32_t)(sA * 4));
    nd.rgR = make_rsrc(ba.gR + (int64_t)tile * sR, (uint32_t)(sR * 4));
    nd.rgAd = make_rsrc(ba.gAd + (int64_t)tile * sM, (uint32_t)(sM * 4));
    ConstRowDesc *rd = as_const(ba.L.rows + rs);
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    int clamped = 0;
    dispatch_nms_bwd<MAXD, FPL>(rd->d, c, rd, ba, nd, valid, acc, clamped);
    // clamped adjoints (rare: long unrolls only): one atomic per wave that has any
    if (__ballot(clamped != 0) != 0ull) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) clamped += __shfl_xor(clamped, o, 64);
        if ((threadIdx.x & 63u) == 0u) atomicAdd(ba.clamps, clamped);
    }
    float out[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) out[i] = block_sum(acc[i], lds);
    if (threadIdx.x == 0) {
        // a sweep's weights take one partial per loss term whose window
        // reaches them; the launches run in a fixed order, so the sums do too
        float *p = ba.part + ((((int64_t)ba.t * ba.mb + rd->row) * ba.L.ntiles + tile) * ba.L.chunks + chunk) * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) p[i] += out[i];
    }
}

// grad[t][i][tau][alpha|beta] = sum over the workgroups of (t, i), fixed
// order.  The sum is taken in double: with adjoints at their bound (long
// unrolls) the partials are finite but their float32 sum can overflow; the
// result saturates at the largest float32 instead of becoming infinite, so
// it keeps its sign for the optimiser.
__global__ void __launch_bounds__(256) k_grad_reduce(const float *part, float *grad, int T, int mb, int per_row,
                                                     int nsets, int64_t set_stride) {
    // one workgroup per (sweep, row): each lane sums a fixed stride of the
    // partials in double, then a fixed tree in LDS, so the sums are run-to-run
    // identical
    __shared__ double lds[4][256];
    const int ti = (int)blockIdx.x;  // t * mb + i
    const int tid = (int)threadIdx.x;
    if (ti >= T * mb) return;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < nsets; ++k) {
        const float4 *p = reinterpret_cast<const float4 *>(part + k * set_stride + (int64_t)ti * per_row * 4);
        for (int r = tid; r < per_row; r += 256) {
            const float4 v = p[r];
            s[0] += (double)v.x;
            s[1] += (double)v.y;
            s[2] += (double)v.z;
            s[3] += (double)v.w;
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) lds[c][tid] = s[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
#pragma unroll
            for (int c = 0; c < 4; ++c) lds[c][tid] += lds[c][tid + w];
        }
        __syncthreads();
    }
    if (tid < 4) {
        constexpr double kMax = 3.4028234663852886e38;  // largest float32
        double v = lds[tid][0];
        v = v > kMax ? kMax : v < -kMax ? -kMax : v;
        // components: 0 dalpha(type 1), 1 dbeta(type 1), 2 dalpha(degree 1), 3 dbeta(degree 1)
        grad[(int64_t)ti * 4 + tid] = (float)v;
    }
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// w -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
// A non-finite gradient component counts as 0 and |g| is capped at 1e15 so
// that g^2 stays finite (Adam's step depends on g only through m / sqrt(v)).
__global__ void k_adam(float *w, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    gi = __builtin_isfinite(gi) ? fminf(fmaxf(gi, -1e15f), 1e15f) : 0.0f;
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

hipError_t qm_launch_nms_kappa(const float *A, const uint8_t *Sil, float *K, const RowDesc *rows, int mb,
                               const TileGeom &g, hipStream_t s) {
    const int chunks = ((g.Z << g.ft_log2) + 255) / 256;
    const int64_t blocks = (int64_t)g.ntiles * mb * chunks;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_nms_kappa, dim3((unsigned)blocks), dim3(256), 0, s, A, Sil, K, rows, g.Z, g.ft_log2,
                       g.ntiles, chunks, (int64_t)g.n << g.ft_log2, (int64_t)g.m << g.ft_log2);
    return hipGetLastError();
}

hipError_t qm_launch_nms_layer(const NmsLayerArgs &na, int maxd, int fpl, int block, hipStream_t s) {
    const LayerArgs &a = na.L;
    const int64_t blocks = (int64_t)a.ntiles * a.nrows * a.chunks;
    if (blocks == 0) return hipSuccess;
    if (block < 64 || block > 256 || (fpl != 1 && fpl != 2) || (1 << a.ft_log2) < fpl)
        return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)blocks), tb((unsigned)block);
#define QM_N(D, P) hipLaunchKernelGGL((k_nms_layer<D, P>), grid, tb, 0, s, na)
#define QM_NP(D)                  \
    if (fpl == 2) QM_N(D, 2);     \
    else QM_N(D, 1);              \
    break;
    switch (maxd) {
        case 2: { QM_NP(2) }
        case 3: { QM_NP(3) }
        case 4: { QM_NP(4) }
        case 5: { QM_NP(5) }
        case 6: { QM_NP(6) }
        case 8: { QM_NP(8) }
        default: { QM_NP(16) }
    }
#undef QM_NP
#undef QM_N
    return hipGetLastError();
}

hipError_t qm_launch_nms_bwd(const NmsBwdArgs &ba, int maxd, int fpl, int block, hipStream_t s) {
    const LayerArgs &a = ba.L;
    const int64_t blocks = (int64_t)a.ntiles * a.nrows * a.chunks;
    if (blocks == 0) return hipSuccess;
    if (block < 64 || block > 256 || (fpl != 1 && fpl != 2) || (1 << a.ft_log2) < fpl)
        return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)blocks), tb((unsigned)block);
#define QM_B(D, P) hipLaunchKernelGGL((k_nms_bwd<D, P>), grid, tb, 0, s, ba)
#define QM_BP(D)                  \
    if (fpl == 2) QM_B(D, 2);     \
    else QM_B(D, 1);              \
    break;
    switch (maxd) {
        case 2: { QM_BP(2) }
        case 3: { QM_BP(3) }
        case 4: { QM_BP(4) }
        case 5: { QM_BP(5) }
        case 6: { QM_BP(6) }
        case 8: { QM_BP(8) }
        default: { QM_BP(16) }
    }
#undef QM_BP
#undef QM_B
    return hipGetLastError();
}

hipError_t qm_launch_commit_d1(float *A, float *Ad, int to_A, const RowDesc *rows, int mb, const TileGeom &g,
                               hipStream_t s) {
    const int V = g.ft_log2 >= 2 ? 4 : 1;  // 16-byte moves when a node holds >= 4 frames
    const int chunks = ((g.Z << g.ft_log2) / V + 255) / 256;
    const int64_t blocks = (int64_t)g.ntiles * mb * chunks;
    if (blocks == 0) return hipSuccess;
    const int64_t sA = (int64_t)g.n << g.ft_log2, sM = (int64_t)g.m << g.ft_log2;
    if (V == 4)
        hipLaunchKernelGGL(k_commit_d1<4>, dim3((unsigned)blocks), dim3(256), 0, s, A, Ad, to_A, rows, g.Z, g.ft_log2,
                           g.ntiles, chunks, sA, sM);
    else
        hipLaunchKernelGGL(k_commit_d1<1>, dim3((unsigned)blocks), dim3(256), 0, s, A, Ad, to_A, rows, g.Z, g.ft_log2,
                           g.ntiles, chunks, sA, sM);
    return hipGetLastError();
}

hipError_t qm_launch_et_update(uint32_t *fail, uint32_t *act, uint64_t *tmask, int32_t *iters, int Fpad, int ft_log2,
                               int done, hipStream_t s) {
    if (ft_log2 < 0 || ft_log2 > 6 || (Fpad & ((1 << ft_log2) - 1))) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_et_update, dim3((unsigned)((Fpad + 255) / 256)), dim3(256), 0, s, fail, act, tmask, iters,
                       Fpad, ft_log2, done);
    return hipGetLastError();
}

hipError_t qm_launch_tile_masks(const uint32_t *act, uint64_t *tmask, int Fpad, int ft_log2, hipStream_t s) {
    if (ft_log2 < 0 || ft_log2 > 6 || (Fpad & ((1 << ft_log2) - 1))) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_tile_masks, dim3((unsigned)((Fpad + 255) / 256)), dim3(256), 0, s, act, tmask, Fpad, ft_log2);
    return hipGetLastError();
}

hipError_t qm_launch_et_final(const uint32_t *act, int32_t *iters, int Fpad, int T, hipStream_t s) {
    hipLaunchKernelGGL(k_et_final, dim3((unsigned)((Fpad + 255) / 256)), dim3(256), 0, s, act, iters, Fpad, T);
    return hipGetLastError();
}

// frames per lane of the loss kernel: 4 (16-byte accesses) when a tile
// holds at least 4 frames
static int bce_frames_per_lane(const TileGeom &g) { return g.ft_log2 >= 2 ? 4 : 1; }
static int bce_chunks(const TileGeom &g) {
    return (((g.Z << g.ft_log2) / bce_frames_per_lane(g)) + 255) / 256;
}

// workgroups of the loss kernel (its grid strides over the items)
int qm_bce_blocks(int ncols, int mb, const TileGeom &g) {
    return (int)std::min<int64_t>((int64_t)g.ntiles * (ncols + mb) * bce_chunks(g), 8192);
}

hipError_t qm_launch_bce(const float *A, const float *Ad, const uint8_t *X, float *gA, float *gAd, float *part,
                         const int32_t *cols, int ncols, const RowDesc *rows, int mb, const TileGeom &g, int F,
                         float weight, int accumulate, float *loss, hipStream_t s) {
    const int chunks = bce_chunks(g);
    const int blocks = qm_bce_blocks(ncols, mb, g);
    if ((int64_t)g.ntiles * chunks * (ncols + mb) >= (1LL << 31)) return hipErrorInvalidValue;
    const float inv = weight / ((float)F * (float)g.n);
    if (bce_frames_per_lane(g) == 4)
        hipLaunchKernelGGL(k_bce<4>, dim3((unsigned)blocks), dim3(256), 0, s, A, Ad, X, gA, gAd, part, cols, ncols,
                           rows, mb, g.Z, g.ft_log2, g.ntiles, chunks, (int64_t)g.n << g.ft_log2,
                           (int64_t)g.m << g.ft_log2, F, inv);
    else
        hipLaunchKernelGGL(k_bce<1>, dim3((unsigned)blocks), dim3(256), 0, s, A, Ad, X, gA, gAd, part, cols, ncols,
                           rows, mb, g.Z, g.ft_log2, g.ntiles, chunks, (int64_t)g.n << g.ft_log2,
                           (int64_t)g.m << g.ft_log2, F, inv);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, part, blocks, inv, accumulate, loss);
    return hipGetLastError();
}

hipError_t qm_launch_grad_reduce(const float *part, float *grad, int T, int mb, int per_row, int nsets,
                                 size_t set_stride, hipStream_t s) {
    if (nsets < 1) return hipErrorInvalidValue;
    if ((set_stride & 3) != 0 || (reinterpret_cast<uintptr_t>(part) & 15) != 0) return hipErrorInvalidValue;
    if (T * mb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)(T * mb)), dim3(256), 0, s, part, grad, T, mb, per_row, nsets,
                       (int64_t)set_stride);
    return hipGetLastError();
}

hipError_t qm_launch_adam(float *w, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                          int step, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, eps, c1,
                       c2);
    return hipGetLastError();
}
