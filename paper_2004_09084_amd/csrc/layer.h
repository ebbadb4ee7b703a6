// Layer kernels of the sum-product decoder (fixed sweeps, early
// termination, fused codes), templated on the message storage type.  Each
// layer_<type>.hip instantiates them for one type, so the three build in
// parallel.
#pragma once

#include "qcmet_internal.h"
#include "device_common.h"
#include "layer_launch.h"
#include "phi.h"

namespace {

using namespace qmdev;

// ---------------------------------------------------------------------------
// Layer update (Methods, steps 2-3; Results: one fused kernel per layer).
// A lane owns one check (base row i of the layer, lift k) for FPL adjacent
// frames of a frame tile.  For each degree>=2 edge j of the row:
//   q_j = APP[col_j][(k + a_j) mod Z] - r_j(old)                (step 3)
//   r_j = (-1)^{s ^ xor_{j'!=j}[q_j' < 0]} Phi(clip(sum_{j'!=j} Phi(clip|q_j'|)))
//                                                                (step 2 + flip)
//   APP = q_j + r_j(new)                                         (step 3)
// The degree-1 edge enters through K: its variable has this check only, so
// its q equals its channel LLR at every visit; |K| = Phi(clip|LLR_d|) and
// sign(K) = s ^ [LLR_d < 0] are constants.  Exclusive sums are a running
// prefix plus a precomputed suffix (no total-minus-self).  In the last sweep
// the degree-1 APP = LLR_d + r_d is formed from the same q's.
// Rows of one layer share no column and distinct k of a row touch distinct
// variables, so no two lanes of a launch touch the same APP or message.
// D is the row's exact number of degree>=2 edges (fully unrolled body).
// ---------------------------------------------------------------------------
// Per-lane state of an early-terminating sweep: which of the lane's frames
// still decode, and where the per-check degree-1 APPs go.
template <int FPL>
struct EtLane {
    bool live[FPL];
    bool all;                 // every frame of the lane is live
    bool tile_full;           // every frame of the tile is live (wave-uniform)
    bool leader;              // first lane of its check's lane group
    __amdgpu_buffer_rsrc_t rAd;  // this tile's channel LLRs of the degree-1 variables, per check
    uint8_t *Pd;              // this tile's packed degree-1 hard decisions per check
    const uint8_t *PS;        // this tile's packed syndrome bits per check
    int jl;                   // lane index in its check's lane group
    int lpl;                  // log2(lanes per check)
};

// Hard decisions [v < 0] of the FT frames of this lane's check (its lane
// group of LPC = FT/FPL lanes) as one packed word.  Bit order: frame
// j*FPL + f of the tile (lane j of the group, its frame f) is bit f*LPC + j,
// so the word is the group's slice of each frame's wave ballot, side by side
// (qm_pack_bit gives the same order to every producer and reader).
template <int FPL>
__device__ __forceinline__ uint64_t group_signs(const float (&v)[FPL], int lpl) {
    const int lane = (int)(threadIdx.x & 63u);
    const int first = (lane >> lpl) << lpl;
    const int lpc = 1 << lpl;
    const uint64_t mask = lpc >= 64 ? ~0ull : ((1ull << lpc) - 1ull);
    uint64_t w = 0;
#pragma unroll
    for (int f = 0; f < FPL; ++f) w |= ((__ballot(v[f] < 0.0f) >> first) & mask) << (f * lpc);
    return w;
}

// Store FPL adjacent values, or only the live ones when a frame of the lane
// has stopped (its state stays as it was when it stopped).
template <typename IO, int FPL, int AUX, bool ET>
__device__ __forceinline__ void store_live(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, const float (&v)[FPL],
                                           const EtLane<FPL> &e) {
    if (!ET || e.all) {
        IO::template store<FPL, AUX>(r, vo, so, v);
    } else {
#pragma unroll
        for (int f = 0; f < FPL; ++f)
            if (e.live[f]) {
                const float one[1] = {v[f]};
                IO::template store<1, AUX>(r, vo + (uint32_t)f * IO::bytes, so, one);
            }
    }
}

// Relative half-width of the band around |K| = clip(S) inside which the
// degree-1 hard decision of an early-terminating sweep takes the exact sum
// (d1_early), per message type.  Phi is decreasing and its own inverse,
// so |LLR_d| > |r_d| = Phi(clip S) exactly when Phi(clip|LLR_d|) < clip S.
// The float32 Phi is within eps = 1.5e-6 relative of Phi, the stored
// message within rho of the float32 one (0 for float32, 2^-11 for binary16
// normals), and ln Phi falls with ln x at a rate g(x) = x / (sinh(x) Phi(x))
// >= 1/29.9 on the clip interval (smallest at Phi(30)); a band of
// eps + 29.9 (eps + rho) therefore separates the two cases.  float32:
// 4.6e-5, taken as 2^-12; binary16: 0.015, taken as 2^-5, and only where
// the message stays a binary16 normal (clip S <= 9: Phi(9) = 2.5e-4 >
// 2^-14).  8-bit messages (rho = 1/16) always take the exact sum.
template <typename MsgT>
struct D1Band {
    static constexpr bool fast = false;
    static constexpr float lo = 0.0f, hi = 0.0f, smax = 0.0f;
};
template <>
struct D1Band<float> {
    static constexpr bool fast = true;
    static constexpr float lo = 1.0f - 0x1p-12f, hi = 1.0f + 0x1p-12f, smax = 1e30f;
};
template <>
struct D1Band<_Float16> {
    static constexpr bool fast = true;
    static constexpr float lo = 1.0f - 0x1p-5f, hi = 1.0f + 0x1p-5f, smax = 9.0f;
};

// Degree-1 variable of an early-terminating sweep: every sweep may be a
// frame's last, so every sweep needs the hard decision [APP_d < 0] of
// APP_d = LLR_d + r_d (|r_d| = Phi(clip S), S the check's Phi-sum over its
// degree>=2 edges; sign(r_d) = s ^ xor_j [q_j < 0]).  Outside the band of
// D1Band the comparison of |K| with clip(S) decides it (no Phi); inside,
// the exact sum is formed from LLR_d (kept per check in Ad).  The APP
// itself is formed only for the frames that stop, as they are written out
// (qm_launch_emit, with the same arithmetic): A's degree-1 slot keeps
// clip(S) with r_d's sign.
template <typename MsgT, int FPL, bool MASKED, typename PW>
__device__ __forceinline__ void d1_early(const LaneCtx &c, ConstRowDesc *rd, const EtLane<FPL> &et,
                                         const float (&kap)[FPL], const bool (&neg)[FPL], const float (&acc)[FPL],
                                         uint64_t sw, uint32_t row_so, uint32_t col_bytes) {
    typedef MsgIO<MsgT> IO;
    typedef D1Band<MsgT> B;
    float sd[FPL], bits[FPL];
    bool nd[FPL], exact[FPL];
    bool any = false;
#pragma unroll
    for (int f = 0; f < FPL; ++f) {
        const bool sb = ((sw >> ((f << et.lpl) + et.jl)) & 1ull) != 0ull;
        const bool lneg = ((int32_t)__float_as_uint(kap[f]) < 0) != sb;  // [LLR_d < 0]
        nd[f] = neg[f] != lneg;
        const float mc = qm_clip(acc[f]);
        const float a = fabsf(kap[f]);
        sd[f] = nd[f] ? -mc : mc;
        const bool ok = B::fast && mc <= B::smax;
        const bool lam_wins = ok && a < mc * B::lo;
        const bool msg_wins = ok && a > mc * B::hi;
        bits[f] = (lam_wins ? lneg : nd[f]) ? -1.0f : 1.0f;
        exact[f] = !(lam_wins || msg_wins);
        any = any || exact[f];
    }
    if (any) {
        float lam[FPL];
        bload_f32<FPL>(et.rAd, c.node * 4u, row_so, lam);
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            if (!exact[f]) continue;
            const float mag = qm_phi(qm_clip(acc[f]));
            const float out = lam[f] + IO::round(nd[f] ? -mag : mag);
            bits[f] = out < 0.0f ? -1.0f : 1.0f;
        }
    }
    const uint32_t off = shifted_off(c, rd->d1shift);
    store_live<MsgIO<float>, FPL, 0, MASKED>(c.rA, off, (uint32_t)rd->d1col * col_bytes, sd, et);
    const uint64_t w = group_signs<FPL>(bits, et.lpl);
    if (et.leader) reinterpret_cast<PW *>(et.Pd)[(int64_t)rd->row * c.Z + c.k] = (PW)w;
}

// Update modes of the check kernel.
constexpr int kLayered = 0;  // layered sweep (fixed iterations)
constexpr int kEarly = 1;    // layered sweep with early termination (EtLane)
constexpr int kFlood = 2;    // flooding: messages only, the APPs of the previous iteration stay

// MASK (early termination only): some frame of the tile has stopped, so
// stores go through the per-frame live mask; otherwise they are plain.
template <typename MsgT, int D, int FPL, int AUX, int MODE, bool MASK, typename PW>
__device__ __forceinline__ void check_update(const LaneCtx &c, ConstRowDesc *rd, int last, const EtLane<FPL> &et) {
    constexpr bool ET = MODE == kEarly;
    constexpr bool MASKED = ET && MASK;
    typedef MsgIO<MsgT> IO;
    const uint32_t col_bytes = c.colw * 4u;
    const uint32_t msg_col_bytes = c.colw * IO::bytes;
    const uint32_t vo4 = c.node * 4u;
    const uint32_t vom = c.node * IO::bytes;
    const uint32_t row_so = (uint32_t)rd->row * col_bytes;
    const int d1col = rd->d1col;
    const int d1shift = rd->d1shift;
    int sh[D > 0 ? D : 1];
    uint32_t col_so[D > 0 ? D : 1], ent_so[D > 0 ? D : 1];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        sh[j] = rd->shift[j];
        col_so[j] = (uint32_t)rd->col[j] * col_bytes;
        ent_so[j] = (uint32_t)rd->ent[j] * msg_col_bytes;
    }

    // kap = K (|K| = Phi(clip|LLR_d|), sign s ^ [LLR_d < 0]; |K| = 0 and sign
    // s without a degree-1 variable).  Early termination also reads the
    // check's packed syndrome bits: with the sign of K they give the sign of
    // LLR_d, which the degree-1 hard decision needs every sweep.
    float kap[FPL];
    float lam[FPL];
    bload_f32<FPL, AUX>(c.rK, vo4, row_so, kap);
    uint64_t sw = 0;
    if constexpr (ET) sw = (uint64_t)reinterpret_cast<const PW *>(et.PS)[(int64_t)rd->row * c.Z + c.k];
    // sign parities are per-lane booleans (lane masks in scalar registers)
    bool neg[FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) neg[f] = (int32_t)__float_as_uint(kap[f]) < 0;

    float q[D > 0 ? D : 1][FPL], ph[D > 0 ? D : 1][FPL], suf[D > 0 ? D : 1][FPL];
    uint32_t aoff[D > 0 ? D : 1];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        aoff[j] = shifted_off(c, sh[j]);
        float av[FPL], rv[FPL];
        bload_f32<FPL>(c.rA, aoff[j], col_so[j], av);
        IO::template load<FPL, AUX>(c.rR, vom, ent_so[j], rv);
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            q[j][f] = av[f] - rv[f];
            neg[f] = neg[f] != (q[j][f] < 0.0f);
            ph[j][f] = qm_phi(qm_clip(fabsf(q[j][f])));
        }
    }
    float acc[FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) acc[f] = 0.0f;
#pragma unroll
    for (int j = D - 1; j >= 0; --j) {
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            suf[j][f] = acc[f];
            acc[f] += ph[j][f];
        }
    }
    float pre[FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) pre[f] = fabsf(kap[f]);
#pragma unroll
    for (int j = 0; j < D; ++j) {
        float rm[FPL], an[FPL];
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            const float S = pre[f] + suf[j][f];
            pre[f] += ph[j][f];
            const bool nj = neg[f] != (q[j][f] < 0.0f);
            const float mag = qm_phi(qm_clip(S));
            rm[f] = IO::round(nj ? -mag : mag);
            an[f] = q[j][f] + rm[f];
        }
        store_live<IO, FPL, AUX, MASKED>(c.rR, vom, ent_so[j], rm, et);
        if constexpr (MODE != kFlood) store_live<MsgIO<float>, FPL, 0, MASKED>(c.rA, aoff[j], col_so[j], an, et);

    }
    if constexpr (ET) {
        if (d1col >= 0) d1_early<MsgT, FPL, MASKED, PW>(c, rd, et, kap, neg, acc, sw, row_so, col_bytes);
    } else if (last && d1col >= 0) {
        const uint32_t off = shifted_off(c, d1shift);
        const uint32_t so = (uint32_t)d1col * col_bytes;
        float out[FPL];
        bload_f32<FPL>(c.rA, off, so, lam);
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            // neg = s ^ [lam < 0] ^ xor_j [q_j < 0]; the degree-1 target
            // excludes only its own q (= lam): s ^ xor_j [q_j < 0]
            const bool nd = neg[f] != (lam[f] < 0.0f);
            const float mag = qm_phi(qm_clip(acc[f]));
            out[f] = lam[f] + IO::round(nd ? -mag : mag);
        }
        store_live<MsgIO<float>, FPL, 0, MASKED>(c.rA, off, so, out, et);
    }
}

template <typename MsgT, int D, int FPL, int AUX, int MODE, bool MASK = false, typename PW = uint8_t>
__device__ __forceinline__ void dispatch_degree(int d, const LaneCtx &c, ConstRowDesc *rd, int last,
                                                const EtLane<FPL> &et) {
    if constexpr (D >= 0) {
        if (d == D) {
            check_update<MsgT, D, FPL, AUX, MODE, MASK, PW>(c, rd, last, et);
            return;
        }
        dispatch_degree<MsgT, D - 1, FPL, AUX, MODE, MASK, PW>(d, c, rd, last, et);
    }
}

// Thread mapping: workgroup -> (frame tile, row of the layer, chunk of
// lanes); consecutive workgroups cycle through the frame tiles, so with 8
// tiles each tile's lanes stay on one XCD under round-robin dispatch.
// PW (early termination): the packed field's word type, max(FT, 8) bits.
template <typename MsgT, int MAXD, int FPL, int AUX, int MODE = kLayered, typename PW = uint8_t>
__device__ __forceinline__ void layer_body(const LayerArgs &a, int b) {
    constexpr bool ET = MODE == kEarly;
    constexpr int FPLL = LogOf<FPL>::v;
    int tile, rest;
    if constexpr (ET) {
        // only the leading ctl[1] tiles still hold decoding frames: the
        // blocks map over those alone (spread over every XCD), the rest exit
        const int nt = a.ctl[1];
        if (b >= nt * a.nrows * a.chunks) return;
        tile = b % nt;
        rest = b / nt;
    } else {
        tile = b % a.ntiles;
        rest = b / a.ntiles;
    }
    const int chunk = rest % a.chunks;
    const int rs = rest / a.chunks;
    LaneCtx c;
    c.Z = a.Z;
    c.ftl = a.ft_log2;
    const int lpl = c.ftl - FPLL;  // log2(lanes per check)
    const int idx = chunk * (int)blockDim.x + (int)threadIdx.x;
    if (idx >= (c.Z << lpl)) return;
    c.k = idx >> lpl;
    c.node = ((uint32_t)c.k << c.ftl) + ((uint32_t)(idx & ((1 << lpl) - 1)) << FPLL);
    c.colw = (uint32_t)c.Z << c.ftl;
    c.last = a.last;
    c.rA = make_rsrc(a.A + (int64_t)tile * a.strideA, (uint32_t)(a.strideA * 4));
    c.rR = make_rsrc(static_cast<char *>(a.R) + (int64_t)tile * a.strideR * MsgIO<MsgT>::bytes,
                     (uint32_t)(a.strideR * MsgIO<MsgT>::bytes));
    c.rK = make_rsrc(a.K + (int64_t)tile * a.strideK, (uint32_t)(a.strideK * 4));
    ConstRowDesc *rd = as_const(a.rows + rs);
    EtLane<FPL> et;
    if constexpr (ET) {
        // the tile's live mask is one scalar load, issued with the row
        // descriptor's (a per-lane load here would be waited for before the
        // lane's first data load)
        const uint64_t tm = a.tmask[tile];
        et.tile_full = tm == (c.ftl >= 6 ? ~0ull : (1ull << (1 << c.ftl)) - 1ull);
        const int fl0 = (int)(c.node & ((1u << c.ftl) - 1u));
        et.all = true;
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            et.live[f] = ((tm >> (fl0 + f)) & 1ull) != 0ull;
            et.all = et.all && et.live[f];
        }
        et.rAd = make_rsrc(a.Ad + (int64_t)tile * a.strideK, (uint32_t)(a.strideK * 4));
        et.lpl = lpl;
        et.leader = (idx & ((1 << lpl) - 1)) == 0;
        et.Pd = a.Pd + (int64_t)tile * (a.strideK >> c.ftl) * (int64_t)sizeof(PW);
        et.PS = a.PS + (int64_t)tile * (a.strideK >> c.ftl) * (int64_t)sizeof(PW);
        et.jl = idx & ((1 << lpl) - 1);
    }
    if constexpr (ET) {
        // a wave-uniform choice: tiles whose frames all decode (the common
        // case) take the body without per-frame masks
        if (et.tile_full) dispatch_degree<MsgT, MAXD, FPL, AUX, MODE, false, PW>(rd->d, c, rd, a.last, et);
        else dispatch_degree<MsgT, MAXD, FPL, AUX, MODE, true, PW>(rd->d, c, rd, a.last, et);
    } else {
        dispatch_degree<MsgT, MAXD, FPL, AUX, MODE>(rd->d, c, rd, a.last, et);
    }
}

template <typename MsgT, int MAXD, int FPL, int AUX>
__global__ void __launch_bounds__(256) k_layer_sp(const LayerArgs a) {
    layer_body<MsgT, MAXD, FPL, AUX>(a, (int)blockIdx.x);
}

// The same layer update for an early-terminating decode (see EtLane).
// Its register budget is set per maximum degree: left to itself the
// scheduler packs the degree-1 comparison's extra values into the widest
// body and falls to 5 waves per SIMD at degree 5, which costs more than
// the arithmetic the comparison saves.
template <int MAXD>
struct EtWaves {
    static constexpr int v = MAXD <= 5 ? 8 : MAXD <= 8 ? 6 : 1;
};
template <typename MsgT, int MAXD, int FPL, int AUX, typename PW>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(EtWaves<MAXD>::v)))
k_layer_sp_et(const LayerArgs a) {
    layer_body<MsgT, MAXD, FPL, AUX, kEarly, PW>(a, (int)blockIdx.x);
}

// The check half of a flooding iteration: every row of the code in one
// launch, each check reading the APPs of the previous iteration and storing
// only its new messages (and, in the last iteration, its degree-1 APP).
template <typename MsgT, int MAXD, int FPL, int AUX>
__global__ void __launch_bounds__(256) k_layer_flood(const LayerArgs a) {
    layer_body<MsgT, MAXD, FPL, AUX, kFlood>(a, (int)blockIdx.x);
}

// One launch for the current layer of every code of a mixed batch: the
// workgroups of code c are [block_off[c], block_off[c+1]).  Each code
// advances through its own layer sequence; codes never share memory.
template <typename MsgT, int MAXD, int FPL, int AUX>
__global__ void __launch_bounds__(256) k_layer_multi(const MultiLayerArgs m) {
    const int b = (int)blockIdx.x;
    int c = 0;
#pragma unroll
    for (int i = 1; i < QM_MAX_CODES; ++i)
        if (i < m.ncodes && b >= m.block_off[i]) c = i;
    layer_body<MsgT, MAXD, FPL, AUX>(m.code[c], b - m.block_off[c]);
}


// the two single-code layer kernels, for one dispatch over their variants
struct LayerSp {
    template <typename T, int D, int P, int H>
    static void go(dim3 g, dim3 b, hipStream_t s, const LayerArgs &a) {
        hipLaunchKernelGGL((k_layer_sp<T, D, P, H>), g, b, a.shmem, s, a);
    }
};
struct LayerSpEt {
    // one kernel per packed word width, so that every packed load and store
    // is one plain access of that width
    template <typename T, int D, int P, int H>
    static void go(dim3 g, dim3 b, hipStream_t s, const LayerArgs &a) {
        switch (qm_pack_bytes(a.ft_log2)) {
            case 1: hipLaunchKernelGGL((k_layer_sp_et<T, D, P, H, uint8_t>), g, b, a.shmem, s, a); break;
            case 2: hipLaunchKernelGGL((k_layer_sp_et<T, D, P, H, uint16_t>), g, b, a.shmem, s, a); break;
            case 4: hipLaunchKernelGGL((k_layer_sp_et<T, D, P, H, uint32_t>), g, b, a.shmem, s, a); break;
            default: hipLaunchKernelGGL((k_layer_sp_et<T, D, P, H, uint64_t>), g, b, a.shmem, s, a); break;
        }
    }
};
struct LayerFlood {
    template <typename T, int D, int P, int H>
    static void go(dim3 g, dim3 b, hipStream_t s, const LayerArgs &a) {
        hipLaunchKernelGGL((k_layer_flood<T, D, P, H>), g, b, a.shmem, s, a);
    }
};

template <class K, typename T, int D, int P>
void layer_go(dim3 g, dim3 b, hipStream_t s, const LayerArgs &a, int hint) {
    if (hint) K::template go<T, D, P, 2>(g, b, s, a);
    else K::template go<T, D, P, 0>(g, b, s, a);
}

template <class K, typename T>
void layer_maxd(dim3 g, dim3 b, hipStream_t s, const LayerArgs &a, int maxd, int fpl, int hint) {
#define QM_LP(D)                                              \
    if (fpl == 2) layer_go<K, T, D, 2>(g, b, s, a, hint);     \
    else layer_go<K, T, D, 1>(g, b, s, a, hint);              \
    break;
    switch (maxd) {
        case 2: { QM_LP(2) }
        case 3: { QM_LP(3) }
        case 4: { QM_LP(4) }
        case 5: { QM_LP(5) }
        case 6: { QM_LP(6) }
        case 8: { QM_LP(8) }
        default: { QM_LP(16) }
    }
#undef QM_LP
}

template <typename MsgT>
hipError_t layer_msg(const LayerArgs &a, int mode, int maxd, int fpl, int block, int hint, hipStream_t s) {
    const int64_t blocks = (int64_t)a.ntiles * a.nrows * a.chunks;
    if (blocks == 0) return hipSuccess;
    if (block < 64 || block > 256 || (fpl != 1 && fpl != 2) || (1 << a.ft_log2) < fpl)
        return hipErrorInvalidConfiguration;  // the kernels are built for <= 256 lanes
    dim3 grid((unsigned)blocks), tb((unsigned)block);
    if (mode == kEarly) layer_maxd<LayerSpEt, MsgT>(grid, tb, s, a, maxd, fpl, hint);
    else if (mode == kFlood) layer_maxd<LayerFlood, MsgT>(grid, tb, s, a, maxd, fpl, hint);
    else layer_maxd<LayerSp, MsgT>(grid, tb, s, a, maxd, fpl, hint);
    return hipGetLastError();
}

template <typename MsgT>
hipError_t layer_multi_msg(const MultiLayerArgs &m, int maxd, int fpl, int block, int hint, hipStream_t s) {
    const int64_t blocks = m.block_off[m.ncodes];
    if (blocks == 0) return hipSuccess;
    if (block < 64 || block > 256 || (fpl != 1 && fpl != 2) || m.ncodes < 1 || m.ncodes > QM_MAX_CODES)
        return hipErrorInvalidConfiguration;
    for (int c = 0; c < m.ncodes; ++c)
        if (m.block_off[c + 1] > m.block_off[c] && (1 << m.code[c].ft_log2) < fpl) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)blocks), tb((unsigned)block);
#define QM_L(D, P)                                                                    \
    do {                                                                              \
        if (hint) hipLaunchKernelGGL((k_layer_multi<MsgT, D, P, 2>), grid, tb, 0, s, m); \
        else hipLaunchKernelGGL((k_layer_multi<MsgT, D, P, 0>), grid, tb, 0, s, m);      \
    } while (0)
#define QM_LP(D)                \
    if (fpl == 2) QM_L(D, 2);   \
    else QM_L(D, 1);            \
    break;
    switch (maxd) {
        case 2: { QM_LP(2) }
        case 3: { QM_LP(3) }
        case 4: { QM_LP(4) }
        case 5: { QM_LP(5) }
        case 6: { QM_LP(6) }
        case 8: { QM_LP(8) }
        default: { QM_LP(16) }
    }
#undef QM_LP
#undef QM_L
    return hipGetLastError();
}

}  // namespace
