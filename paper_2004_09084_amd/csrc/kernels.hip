// HIP kernels of libqcmet for gfx950 (wave64).
//
// Data layout: every per-node array of one code is stored in "frame tiles"
// (TileGeom): [tile][node][FT], FT frames of a node adjacent.  A wavefront
// of the layer kernel covers 64/FT consecutive checks of one base row for
// FT frames, so every access of a circulant-shifted variable column is one
// contiguous run of 256 bytes (two at the single wrap-around point), and
// the row's shifts/columns are wave-uniform (scalar registers).
#include "qcmet_internal.h"
#include "device_common.h"
#include "phi.h"
#include "layer_launch.h"

#include <algorithm>
#include <cstring>

namespace {

using namespace qmdev;

// K for every check: degree-1 term of the row (or 0 if the row has none)
// with the syndrome bit folded into its sign.
template <int V>
__global__ void __launch_bounds__(256) k_kappa(const float *__restrict__ A, const uint8_t *__restrict__ Sil,
                                               float *__restrict__ K, const RowDesc *rows, int Z, int ftl,
                                               int ntiles, int chunks, int64_t strideA, int64_t strideM) {
    // a lane forms K for V adjacent frames of one check (V divides FT)
    typedef float vf __attribute__((ext_vector_type(V)));
    typedef uint8_t vb __attribute__((ext_vector_type(V)));
    const int b = blockIdx.x;
    const int tile = b % ntiles;
    const int rest = b / ntiles;
    const int chunk = rest % chunks;
    const int rs = rest / chunks;
    const int idx = (chunk * (int)blockDim.x + (int)threadIdx.x) * V;
    if (idx >= (Z << ftl)) return;
    const int k = idx >> ftl;
    const int fl = idx & ((1 << ftl) - 1);
    ConstRowDesc *rd = as_const(rows + rs);
    const int64_t moff = (int64_t)tile * strideM + (((rd->row * Z + k) << ftl) + fl);
    const vb sb = *reinterpret_cast<const vb *>(Sil + moff);
    vf out;
    if (rd->d1col >= 0) {
        int v = k + rd->d1shift;
        v = v >= Z ? v - Z : v;
        const vf lam = *reinterpret_cast<const vf *>(A + (int64_t)tile * strideA + (((rd->d1col * Z + v) << ftl) + fl));
#pragma unroll
        for (int i = 0; i < V; ++i)
            out[i] = with_sign(qm_phi(qm_clip(fabsf(lam[i]))), (uint32_t)(sb[i] & 1u) ^ (uint32_t)(lam[i] < 0.0f));
    } else {
#pragma unroll
        for (int i = 0; i < V; ++i) out[i] = with_sign(0.0f, (uint32_t)(sb[i] & 1u));
    }
    *reinterpret_cast<vf *>(K + moff) = out;
}

// Nodes per workgroup of the layout transposes: a frame's run of them is
// 128 bytes or more on the frame-major side.
constexpr int kRun = 128;

// Frame-major [F][N] -> frame tiles [ntiles][N][FT] (padding frames = 0),
// through a RUN-node x FT-frame LDS tile so both sides are coalesced.
// (LDS: FT x (RUN + 1) elements, dynamic.)  Byte arrays take longer runs, so
// that a workgroup moves as many bytes as a float one.
template <typename T, int RUN>
__global__ void __launch_bounds__(256) k_to_tiles(const T *__restrict__ in, T *__restrict__ out, int F,
                                                  int64_t N, int ftl) {
    static_assert((RUN & (RUN - 1)) == 0 && RUN >= 128, "run of nodes");
    extern __shared__ uint32_t dyn_lds[];
    T *lds = reinterpret_cast<T *>(dyn_lds);
    const int tile = blockIdx.y;
    const int64_t v0 = (int64_t)blockIdx.x * RUN;
    const int FT = 1 << ftl;
    const int tid = threadIdx.x;
#pragma unroll 4
    for (int e = tid; e < (RUN << ftl); e += 256) {
        const int fl = e / RUN;
        const int vv = e % RUN;
        const int f = tile * FT + fl;
        const int64_t v = v0 + vv;
        lds[fl * (RUN + 1) + vv] = (f < F && v < N) ? in[(int64_t)f * N + v] : (T)0;
    }
    __syncthreads();
    T *o = out + ((int64_t)tile * N + v0) * FT;
    for (int e = tid; e < (RUN << ftl); e += 256) {
        const int vv = e >> ftl;
        if (v0 + vv < N) o[e] = lds[(e & (FT - 1)) * (RUN + 1) + vv];
    }
}

// The same transpose for bytes, moved as 4-byte words (N a multiple of 4,
// both buffers 4-byte aligned, FT >= 4): a lane loads a word of 4 nodes of
// one frame, and builds each output word (4 frames of one node) from 4 LDS
// words.  LDS: FT rows of kRun + 1 words (4 kRun nodes).
__global__ void __launch_bounds__(256) k_to_tiles_u8w(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                      int F, int64_t N, int ftl) {
    extern __shared__ uint32_t dyn_lds[];
    const int tile = blockIdx.y;
    const int64_t v0 = (int64_t)blockIdx.x * (4 * kRun);
    const int FT = 1 << ftl;
    const int tid = threadIdx.x;
    const int64_t Nw = N >> 2;  // words per frame row
#pragma unroll 4
    for (int e = tid; e < (kRun << ftl); e += 256) {
        const int fl = e / kRun;
        const int w = e % kRun;
        const int f = tile * FT + fl;
        const int64_t v = v0 + 4 * w;  // v < N implies v + 3 < N
        dyn_lds[fl * (kRun + 1) + w] = (f < F && v < N) ? in[(int64_t)f * Nw + (v >> 2)] : 0u;
    }
    __syncthreads();
    const int qn = FT / 4;  // output words per node
    uint32_t *o = out + (((int64_t)tile * N + v0) << ftl) / 4;
    for (int e = tid; e < (kRun << ftl); e += 256) {
        const int vv = e / qn;
        const int q = e % qn;
        if (v0 + vv >= N) continue;
        const int sh = 8 * (vv & 3);
        const uint32_t *l = dyn_lds + (4 * q) * (kRun + 1) + (vv >> 2);
        o[e] = ((l[0] >> sh) & 0xffu) | (((l[kRun + 1] >> sh) & 0xffu) << 8) |
               (((l[2 * (kRun + 1)] >> sh) & 0xffu) << 16) | (((l[3 * (kRun + 1)] >> sh) & 0xffu) << 24);
    }
}

// Frame tiles -> frame-major APP and hard decisions (step 4: c = [APP < 0]);
// also the per-frame flags from the syndrome pass.  Slots whose frame is
// >= F are padding.
__global__ void __launch_bounds__(256) k_finalize(const float *__restrict__ A, const uint32_t *__restrict__ fail,
                                                  float *__restrict__ app, uint8_t *__restrict__ hard,
                                                  uint8_t *__restrict__ flags, int F, int64_t N, int ftl) {
    extern __shared__ uint32_t dyn_lds[];
    float *lds = reinterpret_cast<float *>(dyn_lds);  // FT x (kRun + 1)
    const int tile = blockIdx.y;
    const int64_t v0 = (int64_t)blockIdx.x * kRun;
    const int FT = 1 << ftl;
    const int tid = threadIdx.x;
    const float *a = A + ((int64_t)tile * N + v0) * FT;
    for (int e = tid; e < (kRun << ftl); e += 256) {
        const int vv = e >> ftl;
        lds[(e & (FT - 1)) * (kRun + 1) + vv] = (v0 + vv < N) ? a[e] : 0.0f;
    }
    __syncthreads();
    for (int fl = tid / kRun; fl < FT; fl += 256 / kRun) {
        const int f = tile * FT + fl;
        const int64_t v = v0 + (tid % kRun);
        if (f < F && v < N) {
            const float x = lds[fl * (kRun + 1) + tid % kRun];
            if (app) app[(int64_t)f * N + v] = x;
            hard[(int64_t)f * N + v] = x < 0.0f ? 1 : 0;
        }
    }
    if (blockIdx.x == 0 && blockIdx.y == 0) {
        const int Fpad = (int)gridDim.y * FT;
        for (int sl = tid; sl < Fpad; sl += 256) {
            if (sl < F) flags[sl] = fail[sl] == 0u ? 1 : 0;
        }
    }
}

// Syndrome test of the hard decisions (H c = s), per frame: a check fails
// iff s ^ xor of [APP < 0] over its variables is 1.  A lane tests V adjacent
// frames of one check (V divides FT); failures are OR-ed in LDS per frame,
// then one atomic per failing frame and workgroup.
// Ad (may be null): degree-1 APPs held per check instead of in A.
template <int V>
__global__ void __launch_bounds__(256) k_syndrome(const float *__restrict__ A, const float *__restrict__ Ad,
                                                  const uint8_t *__restrict__ Sil, const RowDesc *rows,
                                                  uint32_t *fail, int Z, int ftl, int ntiles, int chunks, int parts,
                                                  int64_t strideA, int64_t strideM, const int32_t *ctl) {
    typedef float vf __attribute__((ext_vector_type(V)));
    typedef uint8_t vb __attribute__((ext_vector_type(V)));
    __shared__ uint32_t lf[64];
    const int b = blockIdx.x;
    const int tile = b % ntiles;
    if (ctl && tile >= ctl[1]) return;  // early termination: tile has stopped
    const int rest = b / ntiles;
    const int part = rest % parts;
    const int rs = rest / parts;
    const int tid = threadIdx.x;
    const int FT = 1 << ftl;
    if (tid < 64) lf[tid] = 0u;
    __syncthreads();
    ConstRowDesc *rd = as_const(rows + rs);
    const float *At = A + (int64_t)tile * strideA;
    const uint8_t *St = Sil + (int64_t)tile * strideM;
    const int d = rd->d, row = rd->row, d1col = rd->d1col, d1shift = rd->d1shift;
    for (int c = part; c < chunks; c += parts) {
        const int idx = (c * (int)blockDim.x + tid) * V;
        if (idx < (Z << ftl)) {
            const int k = idx >> ftl;
            const int fl = idx & (FT - 1);
            const int moff = ((row * Z + k) << ftl) + fl;
            const vb sb = *reinterpret_cast<const vb *>(St + moff);
            uint32_t par[V];
#pragma unroll
            for (int i = 0; i < V; ++i) par[i] = sb[i] & 1u;
            for (int j = 0; j < d; ++j) {
                int v = k + rd->shift[j];
                v = v >= Z ? v - Z : v;
                const vf a = *reinterpret_cast<const vf *>(At + (((rd->col[j] * Z + v) << ftl) + fl));
#pragma unroll
                for (int i = 0; i < V; ++i) par[i] ^= (uint32_t)(a[i] < 0.0f);
            }
            if (d1col >= 0) {
                vf a;
                if (Ad) {
                    a = *reinterpret_cast<const vf *>(Ad + (int64_t)tile * strideM + moff);
                } else {
                    int v = k + d1shift;
                    v = v >= Z ? v - Z : v;
                    a = *reinterpret_cast<const vf *>(At + (((d1col * Z + v) << ftl) + fl));
                }
#pragma unroll
                for (int i = 0; i < V; ++i) par[i] ^= (uint32_t)(a[i] < 0.0f);
            }
#pragma unroll
            for (int i = 0; i < V; ++i)
                if (par[i]) lf[fl + i] = 1u;
        }
    }
    __syncthreads();
    // skip the atomic where the word already reads 1 (see k_syndrome_packed)
    if (tid < FT && lf[tid] && reinterpret_cast<volatile uint32_t *>(fail)[tile * FT + tid] == 0u)
        atomicOr(&fail[tile * FT + tid], 1u);
}

// Variable half of a flooding iteration: APP = LLR + the messages of the
// variable's checks, added in ascending row order (ColDesc), for the FPL
// frames of a lane.  Workgroup -> (tile, degree>=2 column, chunk of lanes).
template <typename MsgT, int FPL>
__global__ void __launch_bounds__(256) k_flood_vars(float *__restrict__ A, const float *__restrict__ Lam,
                                                    const void *__restrict__ R, const ColDesc *cols, int Z, int ftl,
                                                    int ntiles, int chunks, int64_t strideA, int64_t strideR,
                                                    int64_t strideL) {
    typedef MsgIO<MsgT> IO;
    constexpr int FPLL = LogOf<FPL>::v;
    const int b = blockIdx.x;
    const int tile = b % ntiles;
    const int rest = b / ntiles;
    const int chunk = rest % chunks;
    const int c = rest / chunks;
    const int lpl = ftl - FPLL;
    const int idx = chunk * (int)blockDim.x + (int)threadIdx.x;
    if (idx >= (Z << lpl)) return;
    const int z = idx >> lpl;
    const uint32_t node = (uint32_t)idx << FPLL;           // z * FT + first frame of the lane
    const uint32_t fl = node & ((1u << ftl) - 1u);
    const uint32_t colw = (uint32_t)Z << ftl;
    ConstColDesc *cd = as_const_col(cols + c);
    const __amdgpu_buffer_rsrc_t rL = make_rsrc(Lam + (int64_t)tile * strideL, (uint32_t)(strideL * 4));
    const __amdgpu_buffer_rsrc_t rR =
        make_rsrc(static_cast<const char *>(R) + (int64_t)tile * strideR * IO::bytes, (uint32_t)(strideR * IO::bytes));
    const __amdgpu_buffer_rsrc_t rA = make_rsrc(A + (int64_t)tile * strideA, (uint32_t)(strideA * 4));
    float sum[FPL];
    bload_f32<FPL>(rL, node * 4u, (uint32_t)c * colw * 4u, sum);
    const int deg = cd->deg;
    for (int e = 0; e < deg; ++e) {
        int k = z - cd->shift[e];
        k = k < 0 ? k + Z : k;
        float r[FPL];
        IO::template load<FPL>(rR, (((uint32_t)k << ftl) + fl) * IO::bytes, (uint32_t)cd->ent[e] * colw * IO::bytes, r);
#pragma unroll
        for (int f = 0; f < FPL; ++f) sum[f] += r[f];
    }
    bstore_f32<FPL>(rA, node * 4u, (uint32_t)cd->col * colw * 4u, sum);
}

// Lam[tile][c*Z*FT + e] = A[tile][cols1[c]*Z*FT + e]: the channel LLRs of the
// degree>=2 columns, kept for the flooding variable update.
__global__ void __launch_bounds__(256) k_copy_cols(const float *__restrict__ A, float *__restrict__ Lam,
                                                   const int32_t *cols1, int64_t colw, int64_t strideA,
                                                   int64_t strideL) {
    const int tile = blockIdx.z;
    const int c = blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= colw) return;
    Lam[(int64_t)tile * strideL + (int64_t)c * colw + e] = A[(int64_t)tile * strideA + (int64_t)cols1[c] * colw + e];
}

// Syndrome test of an early-terminating decode from packed hard decisions:
// each lane takes C checks of one row and tile (256 apart, so that every
// load of a wave is contiguous) and XORs the packed words of the row's
// variables (PA), of its degree-1 variable (Pd) and of its syndrome bits
// (PS); failing frames are OR-ed over the wave and in LDS, then one atomic
// per failing frame and workgroup.  W: the packed field's word type (one
// field per node, max(FT, 8) bits), so that every load is one plain load of
// that width.
constexpr int kSynChecks = 4;  // checks per lane of the packed syndrome test
template <typename W, int C>
__global__ void __launch_bounds__(256) k_syndrome_packed(const uint8_t *__restrict__ PA,
                                                         const uint8_t *__restrict__ Pd,
                                                         const uint8_t *__restrict__ PS, const RowDesc *rows,
                                                         uint32_t *fail, int Z, int ftl, int mb, int chunks,
                                                         int64_t n, int64_t m, const int32_t *ctl, int fpl) {
    __shared__ uint32_t lm[2];
    const int b = blockIdx.x;
    // blocks map over the tiles that still hold decoding frames (spread over
    // every XCD); the rest exit
    const int nt = ctl[1];
    if (b >= nt * mb * chunks) return;
    const int tile = b % nt;
    const int rest = b / nt;
    const int chunk = rest % chunks;
    const int rs = rest / chunks;
    const int tid = threadIdx.x;
    const int FT = 1 << ftl;
    if (tid < 2) lm[tid] = 0u;
    __syncthreads();
    const RowDesc *rd = rows + rs;
    const int d = rd->d;
    const int64_t rowb = (int64_t)rd->row * Z;
    const bool has_d1 = rd->d1col >= 0;
    const W *ps = reinterpret_cast<const W *>(PS) + (int64_t)tile * m + rowb;
    // a row without a degree-1 variable re-reads its syndrome word instead
    const W *p1 = has_d1 ? reinterpret_cast<const W *>(Pd) + (int64_t)tile * m + rowb : ps;
    const W *pa = reinterpret_cast<const W *>(PA) + (int64_t)tile * n;
    // every load of the lane's checks is issued before any word is used: a
    // check past Z re-reads check Z-1 and an entry past the row's degree
    // re-reads entry 0, and their words are dropped
    int kk[C];
    bool ok[C];
    W sv[C], dv[C], w[C][8];
#pragma unroll
    for (int i = 0; i < C; ++i) {
        const int k = chunk * (256 * C) + i * 256 + tid;
        ok[i] = k < Z;
        kk[i] = ok[i] ? k : Z - 1;
        sv[i] = ps[kk[i]];
        dv[i] = p1[kk[i]];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int jj = j < d ? j : 0;
        const W *pc = pa + (int64_t)rd->col[jj] * Z;
        const int sh = rd->shift[jj];
#pragma unroll
        for (int i = 0; i < C; ++i) {
            int v = kk[i] + sh;
            v = v >= Z ? v - Z : v;
            w[i][j] = pc[v];
        }
    }
    uint64_t par = 0;
#pragma unroll
    for (int i = 0; i < C; ++i) {
        W x = sv[i] ^ (has_d1 ? dv[i] : (W)0);
#pragma unroll
        for (int j = 0; j < 8; ++j) x ^= j < d ? w[i][j] : (W)0;
        // rows wider than 8 take the rest one entry at a time
        for (int j = 8; j < d; ++j) {
            int v = kk[i] + rd->shift[j];
            v = v >= Z ? v - Z : v;
            x ^= pa[(int64_t)rd->col[j] * Z + v];
        }
        par |= ok[i] ? (uint64_t)x : 0ull;
    }
    // OR over the wave first (most checks fail while frames decode, so a
    // per-lane LDS atomic would serialise), then one atomic per wave
    uint32_t lo = (uint32_t)par, hi = (uint32_t)(par >> 32);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo |= __shfl_xor(lo, o, 64);
        if constexpr (sizeof(W) == 8) hi |= __shfl_xor(hi, o, 64);
    }
    if ((tid & 63) == 0 && (lo | hi)) {
        atomicOr(&lm[0], lo);
        if constexpr (sizeof(W) == 8) atomicOr(&lm[1], hi);
    }
    __syncthreads();
    if (tid < FT) {
        // every workgroup of a tile reports to the same FT words, and while
        // frames decode nearly all of them fail: skip the atomic when the
        // word already reads 1 (it only ever goes from 0 to 1 in a test)
        const int bit = qm_pack_bit(tid, ftl, fpl);
        if (((bit < 32 ? lm[0] >> bit : lm[1] >> (bit - 32)) & 1u) &&
            reinterpret_cast<volatile uint32_t *>(fail)[tile * FT + tid] == 0u)
            atomicOr(&fail[tile * FT + tid], 1u);
    }
}

// Wave-cooperative packing of frame bits (order qm_pack_bit).  One pass of
// a wave covers 64 / FT consecutive nodes: lane L reads the frame that owns
// bit L mod FT of node L / FT, so the wave's reads span one contiguous
// segment of 64 elements; one ballot then holds the packed fields of all
// those nodes side by side, and the first lane of each field stores it.
// U passes per wave keep U loads in flight.
struct NegBit {
    __device__ bool operator()(float x) const { return x < 0.0f; }
};
struct LowBit {
    __device__ bool operator()(uint8_t x) const { return (x & 1u) != 0u; }
};
constexpr int kPackU = 4;      // passes per wave of the one-off packing passes
constexpr int kPackColsU = 8;  // passes per wave of the packing before every test

template <int U, typename T, typename Bit>
__device__ __forceinline__ void pack_wave(const T *__restrict__ X, uint8_t *__restrict__ P, int64_t node0,
                                          int64_t nend, int ftl, int fpl) {
    const int lane = (int)(threadIdx.x & 63u);
    const int FT = 1 << ftl;
    const int b = lane & (FT - 1);
    const int lpc = FT / fpl;
    const int fl = (b % lpc) * fpl + b / lpc;  // the frame whose decision is bit b
    const int esz = qm_pack_bytes(ftl);
    const uint64_t mask = FT >= 64 ? ~0ull : (1ull << FT) - 1ull;
    const int npw = 64 >> ftl;
    if (node0 >= nend) return;  // wave-uniform
    // all U loads first, so they are in flight together; a node past the end
    // reads the last node (node0 < nend here) and its bit is dropped
    T x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        int64_t node = node0 + (int64_t)u * npw + (lane >> ftl);
        node = node < nend ? node : nend - 1;
        x[u] = X[(node << ftl) + fl];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t node = node0 + (int64_t)u * npw + (lane >> ftl);
        const uint64_t w = __ballot(node < nend && Bit()(x[u]));
        if (b == 0 && node < nend) store_packed(P, node, esz, (w >> (lane - b)) & mask);
    }
}

// first node of this wave's U passes in block bx
template <int U = kPackU>
__device__ __forceinline__ int64_t pack_node0(int ftl, int64_t bx = -1) {
    const int64_t wave = (bx < 0 ? (int64_t)blockIdx.x : bx) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    return wave * U * (64 >> ftl);
}

// Packed hard decisions of every node of the tiles.
__global__ void __launch_bounds__(256) k_pack_signs(const float *__restrict__ X, uint8_t *__restrict__ P, int64_t N,
                                                    int ftl, int fpl) {
    const int64_t tile = blockIdx.y;
    pack_wave<kPackU, float, NegBit>(X + ((tile * N) << ftl), P + tile * N * qm_pack_bytes(ftl), pack_node0(ftl), N,
                                     ftl, fpl);
}

// Packed hard decisions of the degree>=2 columns (cols1) of the tiles that
// still decode (below ctl[1]), after a sweep.
__global__ void __launch_bounds__(256) k_pack_cols(const float *__restrict__ A, uint8_t *__restrict__ P,
                                                   const int32_t *cols1, int Z, int64_t n, int ftl, int fpl,
                                                   const int32_t *ctl) {
    const int64_t tile = blockIdx.z;
    if (tile >= ctl[1]) return;
    const int64_t base = (int64_t)cols1[blockIdx.y] * Z;
    pack_wave<kPackColsU, float, NegBit>(A + ((tile * n) << ftl), P + tile * n * qm_pack_bytes(ftl),
                                         base + pack_node0<kPackColsU>(ftl), base + Z, ftl, fpl);
}

// Packed syndrome bits (same order) of the tiles below ctl[1] (all tiles if
// ctl is null).
__global__ void __launch_bounds__(256) k_pack_syndrome(const uint8_t *__restrict__ Sil, uint8_t *__restrict__ PS,
                                                       int64_t m, int ftl, int fpl, const int32_t *ctl,
                                                       int after_compaction) {
    const int64_t tile = blockIdx.y;
    if (ctl && (tile >= ctl[1] || (after_compaction && ctl[2] == 0))) return;
    // grid-stride over the blocks of the tile: the call after every test
    // (which repacks only when a compaction moved frames) launches few
    const int64_t per_block = 4LL * kPackU * (64 >> ftl);
    const int64_t nb = (m + per_block - 1) / per_block;
    for (int64_t bx = blockIdx.x; bx < nb; bx += gridDim.x)
        pack_wave<kPackU, uint8_t, LowBit>(Sil + ((tile * m) << ftl), PS + tile * m * qm_pack_bytes(ftl),
                                           pack_node0(ftl, bx), m, ftl, fpl);
}

// Node-per-lane packing, for fields of at least 16 bytes (FT syndrome bytes
// with FT >= 16, FT APPs with FT >= 4) on 16-byte aligned tiles: a lane reads
// its node's FT values with 16-byte loads and assembles the packed field in
// registers (frame fl at bit qm_pack_bit), which takes fewer instructions
// per byte than a one-value-per-lane pass with ballots.
template <typename T>
struct FieldBit;
template <>
struct FieldBit<uint8_t> {  // a syndrome byte: its bit 0
    __device__ static bool get(uint32_t word, int byte) { return ((word >> (8 * byte)) & 1u) != 0u; }
};
template <>
struct FieldBit<float> {  // an APP: the hard decision x < 0
    __device__ static bool get(uint32_t word, int) { return __uint_as_float(word) < 0.0f; }
};

template <typename T, int FT, int FPL>
__device__ __forceinline__ uint64_t pack_node_field(const T *__restrict__ x) {
    constexpr int NL = FT * (int)sizeof(T) / 16;  // 16-byte loads per node
    static_assert(NL >= 1 && FT % FPL == 0, "field shape");
    uint4 r[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) r[i] = reinterpret_cast<const uint4 *>(x)[i];
    constexpr int lpc = FT / FPL;
    uint64_t w = 0;
#pragma unroll
    for (int fl = 0; fl < FT; ++fl) {
        const int byte = fl * (int)sizeof(T);
        const uint4 &q = r[byte / 16];
        const int k = (byte % 16) / 4;
        const uint32_t word = k == 0 ? q.x : k == 1 ? q.y : k == 2 ? q.z : q.w;
        w |= (uint64_t)FieldBit<T>::get(word, byte % 4) << ((fl % FPL) * lpc + fl / FPL);
    }
    return w;
}

// every node of the tiles (below ctl[1] and, after a compaction, only when
// one was planned, as k_pack_syndrome)
template <typename T, int FT, int FPL>
__global__ void __launch_bounds__(256) k_pack_nodes(const T *__restrict__ X, uint8_t *__restrict__ P, int64_t N,
                                                    const int32_t *ctl, int after_compaction) {
    const int64_t tile = blockIdx.y;
    if (ctl && (tile >= ctl[1] || (after_compaction && ctl[2] == 0))) return;
    constexpr int PB = FT <= 8 ? 1 : FT / 8;  // bytes of a packed field
    const T *x = X + tile * N * FT;
    uint8_t *p = P + tile * N * PB;
    for (int64_t node = (int64_t)blockIdx.x * 256 + threadIdx.x; node < N; node += (int64_t)gridDim.x * 256)
        store_packed(p, node, PB, pack_node_field<T, FT, FPL>(x + node * FT));
}

// the degree>=2 columns (cols1) of the tiles below ctl[1], as k_pack_cols
template <int FT, int FPL>
__global__ void __launch_bounds__(256) k_pack_cols_nodes(const float *__restrict__ A, uint8_t *__restrict__ P,
                                                         const int32_t *cols1, int Z, int64_t n, const int32_t *ctl) {
    const int64_t tile = blockIdx.z;
    if (tile >= ctl[1]) return;
    const int i = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (i >= Z) return;
    constexpr int PB = FT <= 8 ? 1 : FT / 8;
    const int64_t node = (int64_t)cols1[blockIdx.y] * Z + i;
    store_packed(P + tile * n * PB, node, PB, pack_node_field<float, FT, FPL>(A + (tile * n + node) * FT));
}

// ---------------------------------------------------------------------------
// Early termination (Results, Table tabearly): after every sweep each frame's
// hard decisions are tested against its syndrome (k_syndrome over the tiles
// still decoding); a frame that passes stops, keeping the state it has.
// Frame compaction: when stopped frames would free whole tiles, the frames
// still decoding are moved to the leading slots (stable order) and the
// stopped ones behind them, so the layer launches skip the trailing tiles.
// ---------------------------------------------------------------------------
__global__ void k_et_init(uint32_t *act, uint64_t *tmask, int32_t *map, int32_t *iters, int32_t *ctl, int Fpad,
                          int ntiles, int ftl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < Fpad) {
        act[i] = 1u;
        map[i] = i;
        iters[i] = 0;
    }
    if (i < ntiles) tmask[i] = ftl >= 6 ? ~0ull : (1ull << (1 << ftl)) - 1ull;
    if (i == 0) {
        ctl[0] = Fpad;
        ctl[1] = ntiles;
        for (int w = 2; w < QM_ET_CTL_WORDS; ++w) ctl[w] = 0;
        ctl[5] = Fpad;
    }
}

// Rank of pred among the block's 256 lanes in lane order, and the total.
__device__ __forceinline__ int block_rank(bool pred, int *total, int *wcnt) {
    const int tid = threadIdx.x;
    const uint64_t m = __ballot(pred);
    const int lane_rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if ((tid & 63) == 0) wcnt[tid >> 6] = __popcll(m);
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < 4; ++w) {
        off += (w < (tid >> 6)) ? wcnt[w] : 0;
        tot += wcnt[w];
    }
    __syncthreads();
    *total = tot;
    return off + lane_rank;
}

// One workgroup of 256 lanes.  t = sweeps done.  Frames whose syndrome
// passed stop: iterations t, flag 1.  final_pass (after the test of the last
// sweep): every frame still decoding stops too, with flag 0.  emit[slot] =
// the frame (< F) that stopped at that slot in this call, else -1, and
// ctl[4] = how many: their outputs are written from those slots before any
// data moves.  When the stopped frames free at least one tile, plan a
// compaction: the k-th stopped slot below alive (in slot order) receives the
// k-th decoding slot at or above alive (perm[dst] = src, and perm[s] = s for
// the other slots in [ctl[3], alive)).  Clears fail for the next test.
// act[slot] and tmask[tile] (bit fl = slot tile*FT + fl) take the new live
// state on every path.
__device__ __forceinline__ void plan_commit(const uint8_t *s_act, uint32_t *act, uint64_t *tmask, int Fpad, int ftl) {
    __syncthreads();
    const int tid = threadIdx.x;
    for (int sl = tid; sl < Fpad; sl += 256) act[sl] = s_act[sl];
    const int FT = 1 << ftl;
    for (int tl = tid; tl < (Fpad >> ftl); tl += 256) {
        uint64_t m = 0;
        for (int fl = 0; fl < FT; ++fl) m |= (uint64_t)s_act[(tl << ftl) + fl] << fl;
        tmask[tl] = m;
    }
}

__global__ void __launch_bounds__(256) k_et_plan(uint32_t *fail, uint32_t *act, uint64_t *tmask, int32_t *map,
                                                 int32_t *perm, int32_t *iters, int32_t *emit, uint8_t *flags, int F,
                                                 int32_t *ctl, int Fpad, int ftl, int t, int final_pass) {
    __shared__ uint8_t s_act[QM_ET_MAXF];
    __shared__ int16_t s_map[QM_ET_MAXF];
    __shared__ int16_t s_hole[QM_ET_MAXF];
    __shared__ int wcnt[4];
    __shared__ int s_emitted;
    const int tid = threadIdx.x;
    const int nold = ctl[0];
    if (tid == 0) s_emitted = 0;
    __syncthreads();
    int emitted = 0;
    for (int sl = tid; sl < Fpad; sl += 256) {
        bool a = act[sl] != 0u;
        const int fr = map[sl];
        int e = -1;
        if (a && sl < nold && (final_pass || fail[sl] == 0u)) {
            a = false;
            iters[fr] = t;
            if (fr < F) {
                flags[fr] = final_pass ? 0 : 1;
                e = fr;
                ++emitted;
            }
        }
        s_act[sl] = a ? 1 : 0;
        s_map[sl] = (int16_t)fr;
        emit[sl] = e;
        fail[sl] = 0u;
    }
    if (emitted) atomicAdd(&s_emitted, emitted);
    __syncthreads();
    if (tid == 0) ctl[4] = s_emitted;
    int alive = 0;
    for (int base = 0; base < nold; base += 256) {
        const int sl = base + tid;
        int tot;
        (void)block_rank(sl < nold && s_act[sl], &tot, wcnt);
        alive += tot;
    }
    const int FT = 1 << ftl;
    const int tiles_old = (nold + FT - 1) >> ftl, tiles_new = (alive + FT - 1) >> ftl;
    if (tid == 0) ctl[5] = alive;
    if (alive == 0 || (!final_pass && tiles_new == tiles_old)) {
        // no data moves (alive == 0: nothing left to decode)
        plan_commit(s_act, act, tmask, Fpad, ftl);
        if (tid == 0) {
            if (alive == 0) {
                ctl[0] = 0;
                ctl[1] = 0;
            }
            ctl[2] = 0;
        }
        return;
    }
    // stopped slots below alive, in slot order
    int nh = 0;
    for (int base = 0; base < alive; base += 256) {
        const int sl = base + tid;
        const bool h = sl < alive && !s_act[sl];
        int tot;
        const int r = block_rank(h, &tot, wcnt);
        if (h) s_hole[nh + r] = (int16_t)sl;
        nh += tot;
    }
    __syncthreads();
    if (nh == 0) {
        // the stopped frames already sit behind every decoding one
        plan_commit(s_act, act, tmask, Fpad, ftl);
        if (tid == 0) {
            ctl[0] = alive;
            ctl[1] = tiles_new;
            ctl[2] = 0;
        }
        return;
    }
    const int lo = ((int)s_hole[0] >> ftl) << ftl;
    for (int sl = lo + tid; sl < alive; sl += 256) perm[sl] = sl;
    __syncthreads();
    // decoding slots at or above alive fill the holes, in order
    int nm = 0;
    for (int base = alive; base < nold; base += 256) {
        const int sl = base + tid;
        const bool mv = sl < nold && s_act[sl];
        int tot;
        const int r = block_rank(mv, &tot, wcnt);
        if (mv) {
            const int h = s_hole[nm + r];
            perm[h] = sl;
            map[h] = s_map[sl];
        }
        nm += tot;
    }
    __syncthreads();  // every mover has read s_act
    for (int sl = tid; sl < Fpad; sl += 256) s_act[sl] = sl < alive ? 1 : 0;
    plan_commit(s_act, act, tmask, Fpad, ftl);
    if (tid == 0) {
        ctl[0] = alive;
        ctl[1] = tiles_new;
        ctl[2] = 1;
        ctl[3] = lo;
    }
}

// Outputs of the frames that stopped in the last planning call, read from
// their slots before any data moves: frame-major APPs and hard decisions
// (step 4: c = [APP < 0]), as k_finalize writes them.  Grid-stride over
// (run of kRun nodes, tile) items of the first ntiles tiles; a tile without
// an emitted slot is skipped.
// Degree-1 variables: while a frame decodes, A's slot of each degree-1
// variable holds clip(S) with the sign of r_d (S the check's Phi-sum over its
// degree>=2 edges in the frame's last sweep; k_layer_sp_et); the value
// written out is APP_d = LLR_d + r_d, |r_d| = Phi(clip S) rounded to the
// message type: the arithmetic the fixed-sweep layer kernel applies in its
// last sweep, so the outputs are the same bits.  Frames that stop before any
// sweep keep the channel LLR.  (LDS, dynamic: FT x (kRun + 1) floats, then
// nb column -> row entries.)
template <typename MsgT>
__global__ void __launch_bounds__(256) k_emit(const float *__restrict__ A, const float *__restrict__ Ad,
                                              const int32_t *__restrict__ emit, const int32_t *ctl,
                                              const int32_t *__restrict__ iters, const RowDesc *rows,
                                              const int32_t *__restrict__ d1row, int Z, float *__restrict__ app,
                                              uint8_t *__restrict__ hard, int64_t N,
                                              int ftl, int ntiles, int64_t strideM) {
    if (ctl[4] == 0) return;
    extern __shared__ uint32_t dyn_lds[];
    float *lds = reinterpret_cast<float *>(dyn_lds);
    __shared__ int32_t s_fr[64];
    __shared__ int32_t s_swept[64];  // the slot's frame is listed and ran at least one sweep
    const int FT = 1 << ftl;
    const int tid = threadIdx.x;
    // vector stores where every row of the outputs starts 16-byte (APP) and
    // 4-byte (hard) aligned
    const bool vec = (N & 3) == 0 && (reinterpret_cast<uintptr_t>(app) & 15u) == 0 &&
                     (reinterpret_cast<uintptr_t>(hard) & 3u) == 0;
    // item arithmetic in 32 bits (the launcher checks the item count)
    const uint32_t items = (uint32_t)((N + kRun - 1) / kRun) * (uint32_t)ntiles;
    for (uint32_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int tile = (int)(it % (uint32_t)ntiles);
        const int64_t v0 = (int64_t)(it / (uint32_t)ntiles) * kRun;
        __syncthreads();  // the previous item is done with s_fr and lds
        if (tid < FT) {
            const int f = emit[tile * FT + tid];
            s_fr[tid] = f;
            s_swept[tid] = f >= 0 && iters[f] > 0;
        }
        __syncthreads();
        bool any = false;
        for (int fl = 0; fl < FT; ++fl) any = any || s_fr[fl] >= 0;
        if (!any) continue;
        const float *a = A + ((int64_t)tile * N + v0) * FT;
        const float *ad = Ad + (int64_t)tile * strideM;
        if (FT >= 4) {
            // 16-byte loads: four frames of one node per lane
            const float4 *a4 = reinterpret_cast<const float4 *>(a);
            for (int e4 = tid; e4 < (kRun << ftl) / 4; e4 += 256) {
                const int e = e4 * 4;
                const int vv = e >> ftl;
                const int fl = e & (FT - 1);
                const int64_t v = v0 + vv;
                float x[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                if (v < N) {
                    const float4 xv = a4[e4];
                    x[0] = xv.x; x[1] = xv.y; x[2] = xv.z; x[3] = xv.w;
                    const uint32_t vu = (uint32_t)v;  // n < 2^31
                    const int c = (int)(vu / (uint32_t)Z);
                    const int r = d1row[c];
                    if (r >= 0) {
                        int k = (int)(vu - (uint32_t)c * (uint32_t)Z) - rows[r].d1shift;
                        k = k < 0 ? k + Z : k;
                        const float4 lv = *reinterpret_cast<const float4 *>(
                            ad + (((int64_t)rows[r].row * Z + k) << ftl) + fl);
                        const float lam[4] = {lv.x, lv.y, lv.z, lv.w};
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            if (!s_swept[fl + i]) continue;
                            const float mag = qm_phi(qm_clip(fabsf(x[i])));
                            x[i] = lam[i] + MsgIO<MsgT>::round(x[i] < 0.0f ? -mag : mag);
                        }
                    }
                }
                float *l = lds + fl * (kRun + 1) + vv;
                l[0] = x[0];
                l[kRun + 1] = x[1];
                l[2 * (kRun + 1)] = x[2];
                l[3 * (kRun + 1)] = x[3];
            }
        } else {
            for (int e = tid; e < (kRun << ftl); e += 256) {
                const int vv = e >> ftl;
                const int fl = e & (FT - 1);
                const int64_t v = v0 + vv;
                float x = 0.0f;
                if (v < N) {
                    x = a[e];
                    const uint32_t vu = (uint32_t)v;  // n < 2^31
                    const int c = (int)(vu / (uint32_t)Z);
                    const int r = d1row[c];
                    if (r >= 0 && s_swept[fl]) {
                        int k = (int)(vu - (uint32_t)c * (uint32_t)Z) - rows[r].d1shift;
                        k = k < 0 ? k + Z : k;
                        const float lam = ad[(((int64_t)rows[r].row * Z + k) << ftl) + fl];
                        const float mag = qm_phi(qm_clip(fabsf(x)));
                        x = lam + MsgIO<MsgT>::round(x < 0.0f ? -mag : mag);
                    }
                }
                lds[fl * (kRun + 1) + vv] = x;
            }
        }
        __syncthreads();
        if (vec) {
            // four adjacent nodes per lane: 16-byte APP and 4-byte hard stores
            constexpr int LPR = kRun / 4;  // lanes per frame
            for (int fl = tid / LPR; fl < FT; fl += 256 / LPR) {
                const int f = s_fr[fl];
                const int j = (tid % LPR) * 4;
                const int64_t v = v0 + j;  // N and v are multiples of 4, so v + 3 < N
                if (f >= 0 && v < N) {
                    const float *l = lds + fl * (kRun + 1) + j;
                    const float4 x = make_float4(l[0], l[1], l[2], l[3]);
                    if (app) *reinterpret_cast<float4 *>(app + (int64_t)f * N + v) = x;
                    *reinterpret_cast<uchar4 *>(hard + (int64_t)f * N + v) =
                        make_uchar4(x.x < 0.0f, x.y < 0.0f, x.z < 0.0f, x.w < 0.0f);
                }
            }
        } else {
            for (int fl = tid / kRun; fl < FT; fl += 256 / kRun) {
                const int f = s_fr[fl];
                const int64_t v = v0 + (tid % kRun);
                if (f >= 0 && v < N) {
                    const float x = lds[fl * (kRun + 1) + tid % kRun];
                    if (app) app[(int64_t)f * N + v] = x;
                    hard[(int64_t)f * N + v] = x < 0.0f ? 1 : 0;
                }
            }
        }
    }
}

// Gather the frames still decoding into the holes below alive = ctl[0]: for
// every slot s in [ctl[3], alive) with perm[s] != s, element s of every
// array takes element perm[s] (a slot >= alive, so no element is both read
// and written).  The stopped frames' elements are not kept: their outputs
// were written when they stopped.  Grid-stride over chunks of 256 elements
// of one tile's range; each lane walks the destination tiles.
struct CompactArgs {
    CompactArray arr[QM_COMPACT_ARRAYS];
    int64_t chunk_end[QM_COMPACT_ARRAYS];  // cumulative chunk counts
    int32_t narr, ftl;
    const int32_t *perm;
    const int32_t *ctl;
};

template <typename T>
__device__ __forceinline__ void gather_elem(T *p, int64_t N, int64_t e, int ftl, int lo, int alive,
                                            const int32_t *perm) {
    if (e >= (N << ftl)) return;
    const int FT = 1 << ftl;
    const int fl = (int)(e & (FT - 1));
    const int64_t node = e >> ftl;
    const int t1 = (alive + FT - 1) >> ftl;
    for (int tile = lo >> ftl; tile < t1; ++tile) {
        const int sl = (tile << ftl) + fl;
        if (sl < lo || sl >= alive) continue;
        const int src = perm[sl];
        if (src == sl) continue;
        p[((int64_t)tile * N << ftl) + e] = p[((((int64_t)(src >> ftl)) * N + node) << ftl) + (src & (FT - 1))];
    }
}

__global__ void __launch_bounds__(256) k_compact(const CompactArgs c) {
    if (c.ctl[2] == 0) return;
    const int alive = c.ctl[0], lo = c.ctl[3];
    const int64_t total = c.chunk_end[c.narr - 1];
    for (int64_t ch = blockIdx.x; ch < total; ch += gridDim.x) {
        int a = 0;
        while (ch >= c.chunk_end[a]) ++a;
        const int64_t first = a ? c.chunk_end[a - 1] : 0;
        const int64_t e = (ch - first) * 256 + threadIdx.x;
        const CompactArray &A = c.arr[a];
        if (A.esz == 4)
            gather_elem(static_cast<uint32_t *>(A.p), A.N, e, c.ftl, lo, alive, c.perm);
        else if (A.esz == 2)
            gather_elem(static_cast<uint16_t *>(A.p), A.N, e, c.ftl, lo, alive, c.perm);
        else
            gather_elem(static_cast<uint8_t *>(A.p), A.N, e, c.ftl, lo, alive, c.perm);
    }
}

// Before the frames still decoding move into a narrower tile: one wave
// ranks the live slots of tile 0 (FT_old <= 64 of them) and gives the k-th
// the new slot k (src[k] = its old slot, -1 for new slots without one);
// map, act, the tile mask and the control words follow.
__global__ void __launch_bounds__(64) k_et_narrow_plan(uint32_t *act, uint64_t *tmask, int32_t *map, int32_t *src,
                                                       int32_t *ctl, int ft_old, int ft_new) {
    const int l = (int)threadIdx.x;
    const bool live = l < ft_old && act[l] != 0u;
    const int fr = l < ft_old ? map[l] : 0;
    const uint64_t b = __ballot(live);
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
    const int n = __popcll(b);
    __syncthreads();  // every lane has read act and map
    if (l < ft_new) {
        src[l] = -1;
        act[l] = 0u;
    }
    __syncthreads();
    if (live && rank < ft_new) {
        src[rank] = l;
        map[rank] = fr;
        act[rank] = 1u;
    }
    if (l == 0) {
        tmask[0] = n >= 64 ? ~0ull : (1ull << n) - 1ull;
        ctl[0] = n;
        ctl[1] = n > 0 ? 1 : 0;
        ctl[2] = 0;
        ctl[5] = n;
    }
}

// The narrowed tile: out[node][k] = in[node][src[k]] (tile 0 of the old
// layout) for the new slots k < FT_out, 0 where src[k] < 0.
template <typename T>
__global__ void __launch_bounds__(256) k_narrow(const T *__restrict__ in, T *__restrict__ out, const int32_t *src,
                                                int64_t N, int ftl_in, int ftl_out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (N << ftl_out)) return;
    const int sl = src[e & ((1 << ftl_out) - 1)];
    out[e] = sl >= 0 ? in[((e >> ftl_out) << ftl_in) + sl] : (T)0;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_validate(const float *llr, size_t nl, const uint8_t *syn, size_t ns, uint32_t *err) {
    uint32_t bad = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nl; i += (size_t)gridDim.x * blockDim.x)
        if (!__builtin_isfinite(llr[i])) bad |= 1u;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += (size_t)gridDim.x * blockDim.x)
        if (syn[i] > 1) bad |= 2u;
    if (bad) atomicOr(err, bad);
}

inline int chunks_for(int Z, int ftl, int block) { return ((Z << ftl) + block - 1) / block; }

}  // namespace

hipError_t qm_launch_to_tiles_f32(const float *in, float *out, int F, int64_t N, int ft_log2, int ntiles,
                                  hipStream_t s) {
    dim3 grid((unsigned)((N + kRun - 1) / kRun), (unsigned)ntiles);
    const size_t lds = ((size_t)(kRun + 1) << ft_log2) * 4;
    hipLaunchKernelGGL((k_to_tiles<float, kRun>), grid, dim3(256), lds, s, in, out, F, N, ft_log2);
    return hipGetLastError();
}

hipError_t qm_launch_to_tiles_u8(const uint8_t *in, uint8_t *out, int F, int64_t N, int ft_log2, int ntiles,
                                 hipStream_t s) {
    if (N % 4 == 0 && ft_log2 >= 2 && (reinterpret_cast<uintptr_t>(in) & 3u) == 0 &&
        (reinterpret_cast<uintptr_t>(out) & 3u) == 0) {
        dim3 grid((unsigned)((N + 4 * kRun - 1) / (4 * kRun)), (unsigned)ntiles);
        const size_t lds = ((size_t)(kRun + 1) << ft_log2) * 4;
        hipLaunchKernelGGL(k_to_tiles_u8w, grid, dim3(256), lds, s, reinterpret_cast<const uint32_t *>(in),
                           reinterpret_cast<uint32_t *>(out), F, N, ft_log2);
        return hipGetLastError();
    }
    constexpr int run = 4 * kRun;
    dim3 grid((unsigned)((N + run - 1) / run), (unsigned)ntiles);
    const size_t lds = (((size_t)(run + 1) << ft_log2) + 3) / 4 * 4;
    hipLaunchKernelGGL((k_to_tiles<uint8_t, run>), grid, dim3(256), lds, s, in, out, F, N, ft_log2);
    return hipGetLastError();
}

hipError_t qm_launch_kappa(const float *A, const uint8_t *Sil, float *K, const RowDesc *rows, int mb,
                           const TileGeom &g, hipStream_t s) {
    const int V = g.ft_log2 >= 2 ? 4 : 1;  // 4 frames per lane (16-byte accesses) when a node holds >= 4
    const int chunks = chunks_for(g.Z, g.ft_log2, 256 * V);
    const int64_t blocks = (int64_t)g.ntiles * mb * chunks;
    if (blocks == 0) return hipSuccess;
    const int64_t sA = (int64_t)g.n << g.ft_log2, sM = (int64_t)g.m << g.ft_log2;
    if (V == 4)
        hipLaunchKernelGGL(k_kappa<4>, dim3((unsigned)blocks), dim3(256), 0, s, A, Sil, K, rows, g.Z, g.ft_log2,
                           g.ntiles, chunks, sA, sM);
    else
        hipLaunchKernelGGL(k_kappa<1>, dim3((unsigned)blocks), dim3(256), 0, s, A, Sil, K, rows, g.Z, g.ft_log2,
                           g.ntiles, chunks, sA, sM);
    return hipGetLastError();
}

hipError_t qm_launch_fill_u32(uint32_t *p, uint32_t v, size_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}

hipError_t qm_launch_layer(const LayerArgs &a, int msgk, int maxd, int fpl, int block, int hint, hipStream_t s) {
    switch (msgk) {
        case QM_MSGK_F32: return qm_layer_f32(a, 0, maxd, fpl, block, hint, s);
        case QM_MSGK_F16: return qm_layer_f16(a, 0, maxd, fpl, block, hint, s);
        case QM_MSGK_F8: return qm_layer_f8(a, 0, maxd, fpl, block, hint, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t qm_launch_layer_et(const LayerArgs &a, int msgk, int maxd, int fpl, int block, int hint, hipStream_t s) {
    if (!a.Ad || !a.tmask || !a.ctl) return hipErrorInvalidValue;
    switch (msgk) {
        case QM_MSGK_F32: return qm_layer_f32(a, 1, maxd, fpl, block, hint, s);
        case QM_MSGK_F16: return qm_layer_f16(a, 1, maxd, fpl, block, hint, s);
        case QM_MSGK_F8: return qm_layer_f8(a, 1, maxd, fpl, block, hint, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t qm_launch_layer_multi(const MultiLayerArgs &m, int msgk, int maxd, int fpl, int block, int hint,
                                 hipStream_t s) {
    switch (msgk) {
        case QM_MSGK_F32: return qm_layer_multi_f32(m, maxd, fpl, block, hint, s);
        case QM_MSGK_F16: return qm_layer_multi_f16(m, maxd, fpl, block, hint, s);
        case QM_MSGK_F8: return qm_layer_multi_f8(m, maxd, fpl, block, hint, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t qm_launch_syndrome_et(const float *A, const float *Ad, const uint8_t *Sil, const RowDesc *rows, int mb,
                                 uint32_t *fail, const int32_t *ctl, const TileGeom &g, hipStream_t s) {
    if ((1 << g.ft_log2) > 64) return hipErrorInvalidConfiguration;  // per-frame LDS flags
    const int V = g.ft_log2 >= 2 ? 4 : 1;  // 4 frames per lane (16-byte loads) when a node holds >= 4
    const int chunks = chunks_for(g.Z, g.ft_log2, 256 * V);
    const int parts = chunks < 16 ? chunks : 16;
    const int64_t blocks = (int64_t)g.ntiles * mb * parts;
    if (blocks == 0) return hipSuccess;
    const int64_t sA = (int64_t)g.n << g.ft_log2, sM = (int64_t)g.m << g.ft_log2;
    if (V == 4)
        hipLaunchKernelGGL(k_syndrome<4>, dim3((unsigned)blocks), dim3(256), 0, s, A, Ad, Sil, rows, fail, g.Z,
                           g.ft_log2, g.ntiles, chunks, parts, sA, sM, ctl);
    else
        hipLaunchKernelGGL(k_syndrome<1>, dim3((unsigned)blocks), dim3(256), 0, s, A, Ad, Sil, rows, fail, g.Z,
                           g.ft_log2, g.ntiles, chunks, parts, sA, sM, ctl);
    return hipGetLastError();
}

hipError_t qm_launch_syndrome(const float *A, const float *Ad, const uint8_t *Sil, const RowDesc *rows, int mb,
                              uint32_t *fail, const TileGeom &g, hipStream_t s) {
    return qm_launch_syndrome_et(A, Ad, Sil, rows, mb, fail, nullptr, g, s);
}

hipError_t qm_launch_finalize(const float *A, const uint32_t *fail, float *app, uint8_t *hard, uint8_t *flags,
                              int F, const TileGeom &g, hipStream_t s) {
    dim3 grid((unsigned)((g.n + kRun - 1) / kRun), (unsigned)g.ntiles);
    const size_t lds = ((size_t)(kRun + 1) << g.ft_log2) * 4;
    hipLaunchKernelGGL(k_finalize, grid, dim3(256), lds, s, A, fail, app, hard, flags, F, g.n, g.ft_log2);
    return hipGetLastError();
}

hipError_t qm_launch_layer_flood(const LayerArgs &a, int msgk, int maxd, int fpl, int block, int hint, hipStream_t s) {
    switch (msgk) {
        case QM_MSGK_F32: return qm_layer_f32(a, 2, maxd, fpl, block, hint, s);
        case QM_MSGK_F16: return qm_layer_f16(a, 2, maxd, fpl, block, hint, s);
        case QM_MSGK_F8: return qm_layer_f8(a, 2, maxd, fpl, block, hint, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t qm_launch_flood_vars(float *A, const float *Lam, const void *R, const ColDesc *cols, int ncols1, int msgk,
                                int fpl, int block, const TileGeom &g, hipStream_t s) {
    if (ncols1 == 0 || g.ntiles == 0) return hipSuccess;
    if (block < 64 || block > 256 || (fpl != 1 && fpl != 2) || (1 << g.ft_log2) < fpl)
        return hipErrorInvalidConfiguration;
    const int lanes = (g.Z << g.ft_log2) / fpl;
    const int chunks = (lanes + block - 1) / block;
    const int64_t blocks = (int64_t)g.ntiles * ncols1 * chunks;
    const int64_t sA = g.n << g.ft_log2, sR = (g.nent1 * g.Z) << g.ft_log2, sL = ((int64_t)ncols1 * g.Z) << g.ft_log2;
    dim3 grid((unsigned)blocks), tb((unsigned)block);
#define QM_FV(T)                                                                                                   \
    do {                                                                                                           \
        if (fpl == 2)                                                                                              \
            hipLaunchKernelGGL((k_flood_vars<T, 2>), grid, tb, 0, s, A, Lam, R, cols, g.Z, g.ft_log2, g.ntiles,     \
                               chunks, sA, sR, sL);                                                                \
        else                                                                                                       \
            hipLaunchKernelGGL((k_flood_vars<T, 1>), grid, tb, 0, s, A, Lam, R, cols, g.Z, g.ft_log2, g.ntiles,     \
                               chunks, sA, sR, sL);                                                                \
    } while (0)
    switch (msgk) {
        case QM_MSGK_F32: QM_FV(float); break;
        case QM_MSGK_F16: QM_FV(_Float16); break;
        case QM_MSGK_F8: QM_FV(Fp8Msg); break;
        default: return hipErrorInvalidValue;
    }
#undef QM_FV
    return hipGetLastError();
}

hipError_t qm_launch_copy_cols(const float *A, float *Lam, const int32_t *cols1, int ncols1, const TileGeom &g,
                               hipStream_t s) {
    if (ncols1 == 0 || g.ntiles == 0) return hipSuccess;
    const int64_t colw = (int64_t)g.Z << g.ft_log2;
    dim3 grid((unsigned)((colw + 255) / 256), (unsigned)ncols1, (unsigned)g.ntiles);
    hipLaunchKernelGGL(k_copy_cols, grid, dim3(256), 0, s, A, Lam, cols1, colw, g.n << g.ft_log2,
                       ((int64_t)ncols1 * g.Z) << g.ft_log2);
    return hipGetLastError();
}

hipError_t qm_launch_syndrome_packed(const uint8_t *PA, const uint8_t *Pd, const uint8_t *PS, const RowDesc *rows,
                                     int mb, uint32_t *fail, const int32_t *ctl, int fpl, const TileGeom &g,
                                     hipStream_t s) {
    if ((1 << g.ft_log2) > 64 || !ctl || fpl < 1) return hipErrorInvalidValue;
    const int chunks = (g.Z + 256 * kSynChecks - 1) / (256 * kSynChecks);
    const int64_t blocks = (int64_t)g.ntiles * mb * chunks;
    if (blocks == 0) return hipSuccess;
    switch (qm_pack_bytes(g.ft_log2)) {
#define QM_SP(W)                                                                                                  \
    hipLaunchKernelGGL((k_syndrome_packed<W, kSynChecks>), dim3((unsigned)blocks), dim3(256), 0, s, PA, Pd, PS,  \
                       rows, fail, g.Z, g.ft_log2, mb, chunks, g.n, g.m, ctl, fpl)
        case 1: QM_SP(uint8_t); break;
        case 2: QM_SP(uint16_t); break;
        case 4: QM_SP(uint32_t); break;
        default: QM_SP(uint64_t); break;
#undef QM_SP
    }
    return hipGetLastError();
}

// The node-per-lane packing applies when a node's field of FT values is at
// least 16 bytes, every tile starts 16-byte aligned, and a lane holds one or
// two frames.
static bool node_fields(const void *X, int64_t N, int ftl, int fpl, size_t esz) {
    const size_t field = esz << ftl;
    return field >= 16 && field % 16 == 0 && (reinterpret_cast<uintptr_t>(X) & 15u) == 0 &&
           ((size_t)N * field) % 16 == 0 && (fpl == 1 || fpl == 2) && ftl <= 6;
}
static unsigned node_blocks(int64_t N) { return (unsigned)std::min<int64_t>((N + 255) / 256, 65535); }
// float fields: FT = 4 .. 64, one or two frames per lane
#define QM_NODE_DISPATCH(ftl, fpl, M)        \
    switch ((ftl) * 2 + (fpl) - 1) {         \
        case 4: M(4, 1); break;              \
        case 5: M(4, 2); break;              \
        case 6: M(8, 1); break;              \
        case 7: M(8, 2); break;              \
        case 8: M(16, 1); break;             \
        case 9: M(16, 2); break;             \
        case 10: M(32, 1); break;            \
        case 11: M(32, 2); break;            \
        case 12: M(64, 1); break;            \
        default: M(64, 2); break;            \
    }

// blocks of 256 lanes for a packing pass over N nodes
static unsigned pack_blocks(int64_t N, int ftl, int U = kPackU) {
    const int64_t per_block = 4LL * U * (64 >> ftl);
    return (unsigned)((N + per_block - 1) / per_block);
}

hipError_t qm_launch_pack_signs(const float *X, uint8_t *P, int64_t N, int fpl, const TileGeom &g, hipStream_t s) {
    if ((1 << g.ft_log2) > 64 || fpl < 1 || fpl > (1 << g.ft_log2)) return hipErrorInvalidValue;
    if (N == 0 || g.ntiles == 0) return hipSuccess;
    if (node_fields(X, N, g.ft_log2, fpl, sizeof(float))) {
        dim3 grid(node_blocks(N), (unsigned)g.ntiles);
#define QM_PN(FT, FPL) hipLaunchKernelGGL((k_pack_nodes<float, FT, FPL>), grid, dim3(256), 0, s, X, P, N, nullptr, 0)
        QM_NODE_DISPATCH(g.ft_log2, fpl, QM_PN);
#undef QM_PN
        return hipGetLastError();
    }
    dim3 grid(pack_blocks(N, g.ft_log2), (unsigned)g.ntiles);
    hipLaunchKernelGGL(k_pack_signs, grid, dim3(256), 0, s, X, P, N, g.ft_log2, fpl);
    return hipGetLastError();
}

hipError_t qm_launch_pack_cols(const float *A, uint8_t *P, const int32_t *cols1, int ncols1, const int32_t *ctl, int fpl,
                               const TileGeom &g, hipStream_t s) {
    if ((1 << g.ft_log2) > 64 || fpl < 1 || fpl > (1 << g.ft_log2) || !ctl) return hipErrorInvalidValue;
    if (ncols1 == 0 || g.ntiles == 0) return hipSuccess;
    if (node_fields(A, g.n, g.ft_log2, fpl, sizeof(float))) {
        dim3 grid((unsigned)((g.Z + 255) / 256), (unsigned)ncols1, (unsigned)g.ntiles);
#define QM_PC(FT, FPL) \
    hipLaunchKernelGGL((k_pack_cols_nodes<FT, FPL>), grid, dim3(256), 0, s, A, P, cols1, g.Z, g.n, ctl)
        QM_NODE_DISPATCH(g.ft_log2, fpl, QM_PC);
#undef QM_PC
        return hipGetLastError();
    }
    dim3 grid(pack_blocks(g.Z, g.ft_log2, kPackColsU), (unsigned)ncols1, (unsigned)g.ntiles);
    hipLaunchKernelGGL(k_pack_cols, grid, dim3(256), 0, s, A, P, cols1, g.Z, g.n, g.ft_log2, fpl, ctl);
    return hipGetLastError();
}

hipError_t qm_launch_pack_syndrome(const uint8_t *Sil, uint8_t *PS, const int32_t *ctl, int after_compaction, int fpl,
                                   const TileGeom &g, hipStream_t s) {
    if ((1 << g.ft_log2) > 64 || fpl < 1 || fpl > (1 << g.ft_log2)) return hipErrorInvalidValue;
    if (g.m == 0 || g.ntiles == 0) return hipSuccess;
    if (g.ft_log2 >= 4 && node_fields(Sil, g.m, g.ft_log2, fpl, 1)) {
        const unsigned nb = node_blocks(g.m);
        dim3 grid(after_compaction ? std::min(nb, 512u) : nb, (unsigned)g.ntiles);
#define QM_PS(FT, FPL)                                                                                              \
    hipLaunchKernelGGL((k_pack_nodes<uint8_t, FT, FPL>), grid, dim3(256), 0, s, Sil, PS, g.m, ctl, after_compaction)
        switch (g.ft_log2 * 2 + fpl - 1) {
            case 8: QM_PS(16, 1); break;
            case 9: QM_PS(16, 2); break;
            case 10: QM_PS(32, 1); break;
            case 11: QM_PS(32, 2); break;
            case 12: QM_PS(64, 1); break;
            default: QM_PS(64, 2); break;
        }
#undef QM_PS
        return hipGetLastError();
    }
    const unsigned bx = after_compaction ? std::min(pack_blocks(g.m, g.ft_log2), 512u) : pack_blocks(g.m, g.ft_log2);
    dim3 grid(bx, (unsigned)g.ntiles);
    hipLaunchKernelGGL(k_pack_syndrome, grid, dim3(256), 0, s, Sil, PS, g.m, g.ft_log2, fpl, ctl, after_compaction);
    return hipGetLastError();
}

hipError_t qm_launch_et_init(uint32_t *act, uint64_t *tmask, int32_t *map, int32_t *iters, int32_t *ctl, int Fpad,
                             int ntiles, int ft_log2, hipStream_t s) {
    if (ft_log2 < 0 || ft_log2 > 6 || (ntiles << ft_log2) != Fpad) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_et_init, dim3((unsigned)((Fpad + 255) / 256)), dim3(256), 0, s, act, tmask, map, iters, ctl,
                       Fpad, ntiles, ft_log2);
    return hipGetLastError();
}

hipError_t qm_launch_et_plan(uint32_t *fail, uint32_t *act, uint64_t *tmask, int32_t *map, int32_t *perm,
                             int32_t *iters, int32_t *emit, uint8_t *flags, int F, int32_t *ctl, int Fpad, int ft_log2,
                             int t, int final_pass, hipStream_t s) {
    // F (the code's frame count) may exceed Fpad once the frames still
    // decoding sit in a narrowed tile: frame ids come from map
    if (Fpad < 1 || Fpad > QM_ET_MAXF || F < 0 || ft_log2 < 0 || ft_log2 > 6 || (Fpad & ((1 << ft_log2) - 1)))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_et_plan, dim3(1), dim3(256), 0, s, fail, act, tmask, map, perm, iters, emit, flags, F, ctl,
                       Fpad, ft_log2, t, final_pass);
    return hipGetLastError();
}

hipError_t qm_launch_emit(const float *A, const float *Ad, const int32_t *emit, const int32_t *ctl,
                          const int32_t *iters, const RowDesc *rows, const int32_t *d1row, int msgk, float *app,
                          uint8_t *hard, const TileGeom &g, hipStream_t s) {
    if ((1 << g.ft_log2) > 64 || g.Z < 1 || g.n % g.Z != 0 || g.n >= (1LL << 31)) return hipErrorInvalidValue;
    const int64_t items = ((g.n + kRun - 1) / kRun) * g.ntiles;
    if (items == 0) return hipSuccess;
    if (items >= (1LL << 31)) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)std::min<int64_t>(items, 4096);
    const size_t lds = ((size_t)(kRun + 1) << g.ft_log2) * 4;
    const int64_t sM = (int64_t)g.m << g.ft_log2;
#define QM_EM(T)                                                                                              \
    hipLaunchKernelGGL(k_emit<T>, dim3(blocks), dim3(256), lds, s, A, Ad, emit, ctl, iters, rows, d1row, g.Z, \
                       app, hard, g.n, g.ft_log2, g.ntiles, sM)
    switch (msgk) {
        case QM_MSGK_F32: QM_EM(float); break;
        case QM_MSGK_F16: QM_EM(_Float16); break;
        case QM_MSGK_F8: QM_EM(Fp8Msg); break;
        default: return hipErrorInvalidValue;
    }
#undef QM_EM
    return hipGetLastError();
}

hipError_t qm_launch_compact(const CompactArray *arr, int narr, const int32_t *perm, const int32_t *ctl,
                             int ft_log2, hipStream_t s) {
    if (narr < 1 || narr > QM_COMPACT_ARRAYS) return hipErrorInvalidValue;
    CompactArgs c;
    std::memset(&c, 0, sizeof(c));
    c.narr = narr;
    c.ftl = ft_log2;
    c.perm = perm;
    c.ctl = ctl;
    int64_t acc = 0;
    for (int i = 0; i < narr; ++i) {
        c.arr[i] = arr[i];
        acc += ((arr[i].N << ft_log2) + 255) / 256;
        c.chunk_end[i] = acc;
    }
    if (acc == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<int64_t>(acc, 8192);
    hipLaunchKernelGGL(k_compact, dim3(blocks), dim3(256), 0, s, c);
    return hipGetLastError();
}

hipError_t qm_launch_et_narrow_plan(uint32_t *act, uint64_t *tmask, int32_t *map, int32_t *src, int32_t *ctl,
                                    int ft_log2_old, int ft_log2_new, hipStream_t s) {
    if (ft_log2_new < 0 || ft_log2_new >= ft_log2_old || ft_log2_old > 6) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_et_narrow_plan, dim3(1), dim3(64), 0, s, act, tmask, map, src, ctl, 1 << ft_log2_old,
                       1 << ft_log2_new);
    return hipGetLastError();
}

hipError_t qm_launch_narrow(const void *in, void *out, const int32_t *src, int64_t N, int esz, int ft_log2_in,
                            int ft_log2_out, hipStream_t s) {
    if (ft_log2_out < 0 || ft_log2_out > ft_log2_in || ft_log2_in > 6) return hipErrorInvalidValue;
    const int64_t total = N << ft_log2_out;
    if (total == 0) return hipSuccess;
    const dim3 grid((unsigned)((total + 255) / 256));
    switch (esz) {
        case 4:
            hipLaunchKernelGGL(k_narrow<uint32_t>, grid, dim3(256), 0, s, static_cast<const uint32_t *>(in),
                               static_cast<uint32_t *>(out), src, N, ft_log2_in, ft_log2_out);
            break;
        case 2:
            hipLaunchKernelGGL(k_narrow<uint16_t>, grid, dim3(256), 0, s, static_cast<const uint16_t *>(in),
                               static_cast<uint16_t *>(out), src, N, ft_log2_in, ft_log2_out);
            break;
        case 1:
            hipLaunchKernelGGL(k_narrow<uint8_t>, grid, dim3(256), 0, s, static_cast<const uint8_t *>(in),
                               static_cast<uint8_t *>(out), src, N, ft_log2_in, ft_log2_out);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t qm_launch_validate(const float *llr, size_t nl, const uint8_t *syn, size_t ns, uint32_t *err,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_validate, dim3(1024), dim3(256), 0, s, llr, nl, syn, ns, err);
    return hipGetLastError();
}
