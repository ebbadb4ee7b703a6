// HIP kernels of libqcmet for gfx950 (wave64).
//
// Data layout: every per-node array of one code is stored in "frame tiles"
// (TileGeom): [tile][node][FT], FT frames of a node adjacent.  A wavefront
// of the layer kernel covers 64/FT consecutive checks of one base row for
// FT frames, so every access of a circulant-shifted variable column is one
// contiguous run of 256 bytes (two at the single wrap-around point), and
// the row's shifts/columns are wave-uniform (scalar registers).
#include "qcmet_internal.h"

namespace {

// ---------------------------------------------------------------------------
// Check-node transform Phi(x) = -ln(tanh(x/2)) (Methods, step 2), float32,
// for x already clipped to [Phi(30), 30].  Two branch-free regions:
//   x >= 1: Phi = 2 atanh(u), u = e^-x <= 1/e, evaluated as 2u * P(u^2);
//   x <  1: Phi = ln(2/x) - ln(tanh(h)/h), h = x/2, with the second term
//           y * Q(y), y = h^2 <= 1/4.
// P (degree 4) and Q (degree 3) are least-squares fits on Chebyshev nodes of
// the analytic functions atanh(u)/u and ln(tanh(h)/h)/h^2 (fit_phi_coeffs.py
// next to this file); their own error is below 1.2e-8, so the float32 result
// is within ~2e-6 relative of Phi over the whole interval, most of it from
// the rounding of x itself at large x.  v_exp_f32 / v_log_f32 are the
// hardware base-2 exponential and logarithm.
// ---------------------------------------------------------------------------
constexpr float kLog2eHi = 1.44269502162933349609375f;
constexpr float kLog2eLo = 1.925963033500011079e-08f;
constexpr float kLn2 = 0.693147180559945309f;
constexpr float kXLo = 1.87152459e-13f;  // Phi(30)
constexpr float kP0 = 1.0000000112364562f, kP1 = 0.33332923606239323f, kP2 = 0.2002375193642375f,
                kP3 = 0.13809908933873744f, kP4 = 0.14878416970977898f;
constexpr float kQ0 = -0.33333283877243064f, kQ1 = 0.07775853015298553f,
                kQ2 = -0.02163326744699287f, kQ3 = 0.00554818214693421f;

__device__ __forceinline__ float qm_clip(float x) { return fminf(fmaxf(x, kXLo), QM_X_HI); }

__device__ __forceinline__ float qm_phi(float x) {
    const float t = fmaf(-x, kLog2eHi, -x * kLog2eLo);
    const float u = __builtin_amdgcn_exp2f(t);
    const float w = u * u;
    float p = fmaf(w, kP4, kP3);
    p = fmaf(w, p, kP2);
    p = fmaf(w, p, kP1);
    p = fmaf(w, p, kP0);
    const float big = (2.0f * u) * p;
    const float y = 0.25f * x * x;
    float qy = fmaf(y, kQ3, kQ2);
    qy = fmaf(y, qy, kQ1);
    qy = fmaf(y, qy, kQ0);
    const float lg = __builtin_amdgcn_logf(x);  // log2(x)
    const float small = fmaf(1.0f - lg, kLn2, -y * qy);
    return x < 1.0f ? small : big;
}

// magnitude (>= 0) with the sign bit set iff neg
__device__ __forceinline__ float with_sign(float mag, uint32_t neg) {
    return __uint_as_float(__float_as_uint(mag) | (neg << 31));
}

template <typename MsgT>
__device__ __forceinline__ MsgT to_msg(float v);
template <>
__device__ __forceinline__ float to_msg<float>(float v) { return v; }
template <>
__device__ __forceinline__ _Float16 to_msg<_Float16>(float v) { return (_Float16)v; }  // RNE

// ---------------------------------------------------------------------------
// Layer update (Methods, steps 2-3; Results: one fused kernel per layer).
// Thread = (frame tile, row of the layer, check k, frame fl).  For the
// check of base row i at lift k:
//   q_j   = APP[col_j][(k + a_j) mod Z] - r_j(old)          (step 3)
//   r_j   = (-1)^{s ^ xor_{j'!=j}[q_j' < 0]} Phi(clip(sum_{j'!=j} Phi(clip|q_j'|)))
//                                                            (step 2 + flip)
//   APP   = q_j + r_j(new)                                   (step 3)
// over the row's degree>=2 edges j.  The degree-1 edge enters through K:
// its variable has this check only, so its q equals its channel LLR at every
// visit and |K| = Phi(clip|LLR_d|), sign(K) = s ^ [LLR_d < 0] are constants.
// Exclusive sums are prefix + suffix sums (no total-minus-self).  In the last
// sweep the degree-1 APP = LLR_d + r_d is formed from the same q's.
// Rows of one layer share no column and distinct k of a row touch distinct
// variables, so no two threads of a launch touch the same APP or message.
// ---------------------------------------------------------------------------
template <typename MsgT, int MAXD>
__global__ void __launch_bounds__(512) k_layer_sp(const LayerArgs a) {
    const int b = blockIdx.x;
    const int tile = b % a.ntiles;
    const int rest = b / a.ntiles;
    const int chunk = rest % a.chunks;
    const int rs = rest / a.chunks;
    const int Z = a.Z;
    const int ftl = a.ft_log2;
    const int idx = chunk * (int)blockDim.x + (int)threadIdx.x;
    if (idx >= (Z << ftl)) return;
    const int k = idx >> ftl;
    const int fl = idx & ((1 << ftl) - 1);
    const RowDesc *rd = a.rows + rs;
    const int d = rd->d;
    float *__restrict__ A = a.A + (int64_t)tile * a.strideA;
    MsgT *__restrict__ R = static_cast<MsgT *>(a.R) + (int64_t)tile * a.strideR;
    const float *__restrict__ K = a.K + (int64_t)tile * a.strideK;

    const float kap = K[((rd->row * Z + k) << ftl) + fl];
    uint32_t neg = __float_as_uint(kap) >> 31;
    const float phi0 = fabsf(kap);

    float q[MAXD], ph[MAXD], pre[MAXD];
    int aoff[MAXD], roff[MAXD];
#pragma unroll
    for (int j = 0; j < MAXD; ++j) {
        if (j < d) {
            int v = k + rd->shift[j];
            v = v >= Z ? v - Z : v;
            aoff[j] = ((rd->col[j] * Z + v) << ftl) + fl;
            roff[j] = ((rd->ent[j] * Z + k) << ftl) + fl;
            q[j] = A[aoff[j]] - (float)R[roff[j]];
            neg ^= (uint32_t)(q[j] < 0.0f);
            ph[j] = qm_phi(qm_clip(fabsf(q[j])));
        }
    }
    float acc = phi0;
#pragma unroll
    for (int j = 0; j < MAXD; ++j) {
        if (j < d) {
            pre[j] = acc;
            acc += ph[j];
        }
    }
    float suf = 0.0f;
#pragma unroll
    for (int j = MAXD - 1; j >= 0; --j) {
        if (j < d) {
            const float S = pre[j] + suf;
            suf += ph[j];
            const uint32_t nj = neg ^ (uint32_t)(q[j] < 0.0f);
            const MsgT rm = to_msg<MsgT>(with_sign(qm_phi(qm_clip(S)), nj));
            R[roff[j]] = rm;
            A[aoff[j]] = q[j] + (float)rm;
        }
    }
    if (a.last && rd->d1col >= 0) {
        int v = k + rd->d1shift;
        v = v >= Z ? v - Z : v;
        const int off = ((rd->d1col * Z + v) << ftl) + fl;
        const float lam = A[off];
        float sd = 0.0f;
#pragma unroll
        for (int j = 0; j < MAXD; ++j)
            if (j < d) sd += ph[j];
        // neg = s ^ [lam < 0] ^ xor_j [q_j < 0]; the degree-1 target excludes
        // only its own q (= lam): s ^ xor_j [q_j < 0] = neg ^ [lam < 0]
        const uint32_t nd = neg ^ (uint32_t)(lam < 0.0f);
        const MsgT rm = to_msg<MsgT>(with_sign(qm_phi(qm_clip(sd)), nd));
        A[off] = lam + (float)rm;
    }
}

// K for every check: degree-1 term of the row (or 0 if the row has none)
// with the syndrome bit folded into its sign.
__global__ void __launch_bounds__(256) k_kappa(const float *__restrict__ A, const uint8_t *__restrict__ Sil,
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
    const RowDesc *rd = rows + rs;
    const int moff = ((rd->row * Z + k) << ftl) + fl;
    uint32_t neg = Sil[(int64_t)tile * strideM + moff] & 1u;
    float mag = 0.0f;
    if (rd->d1col >= 0) {
        int v = k + rd->d1shift;
        v = v >= Z ? v - Z : v;
        const float lam = A[(int64_t)tile * strideA + (((rd->d1col * Z + v) << ftl) + fl)];
        mag = qm_phi(qm_clip(fabsf(lam)));
        neg ^= (uint32_t)(lam < 0.0f);
    }
    K[(int64_t)tile * strideM + moff] = with_sign(mag, neg);
}

// Frame-major [F][N] -> frame tiles [ntiles][N][FT] (padding frames = 0),
// through a 64-node x FT-frame LDS tile so both sides are coalesced.
template <typename T>
__global__ void __launch_bounds__(256) k_to_tiles(const T *__restrict__ in, T *__restrict__ out, int F,
                                                  int64_t N, int ftl) {
    __shared__ T lds[64][65];
    const int tile = blockIdx.y;
    const int64_t v0 = (int64_t)blockIdx.x * 64;
    const int FT = 1 << ftl;
    const int tid = threadIdx.x;
    for (int fl = tid >> 6; fl < FT; fl += 4) {
        const int f = tile * FT + fl;
        const int64_t v = v0 + (tid & 63);
        lds[fl][tid & 63] = (f < F && v < N) ? in[(int64_t)f * N + v] : (T)0;
    }
    __syncthreads();
    T *o = out + ((int64_t)tile * N + v0) * FT;
    for (int e = tid; e < (64 << ftl); e += 256) {
        const int vv = e >> ftl;
        if (v0 + vv < N) o[e] = lds[e & (FT - 1)][vv];
    }
}

// Frame tiles -> frame-major APP and hard decisions (step 4: c = [APP < 0]);
// also the per-frame flags from the syndrome pass.
__global__ void __launch_bounds__(256) k_finalize(const float *__restrict__ A, const uint32_t *__restrict__ fail,
                                                  float *__restrict__ app, uint8_t *__restrict__ hard,
                                                  uint8_t *__restrict__ flags, int F, int64_t N, int ftl) {
    __shared__ float lds[64][65];
    const int tile = blockIdx.y;
    const int64_t v0 = (int64_t)blockIdx.x * 64;
    const int FT = 1 << ftl;
    const int tid = threadIdx.x;
    const float *a = A + ((int64_t)tile * N + v0) * FT;
    for (int e = tid; e < (64 << ftl); e += 256) {
        const int vv = e >> ftl;
        lds[e & (FT - 1)][vv] = (v0 + vv < N) ? a[e] : 0.0f;
    }
    __syncthreads();
    for (int fl = tid >> 6; fl < FT; fl += 4) {
        const int f = tile * FT + fl;
        const int64_t v = v0 + (tid & 63);
        if (f < F && v < N) {
            const float x = lds[fl][tid & 63];
            if (app) app[(int64_t)f * N + v] = x;
            hard[(int64_t)f * N + v] = x < 0.0f ? 1 : 0;
        }
    }
    if (blockIdx.x == 0 && blockIdx.y == 0)
        for (int f = tid; f < F; f += 256) flags[f] = fail[f] == 0u ? 1 : 0;
}

// Syndrome test of the hard decisions (H c = s), per frame: a check fails
// iff s ^ xor of [APP < 0] over its variables is 1.  Failures are OR-ed in
// LDS per frame, then one atomic per frame and workgroup.
__global__ void __launch_bounds__(256) k_syndrome(const float *__restrict__ A, const uint8_t *__restrict__ Sil,
                                                  const RowDesc *rows, uint32_t *fail, int Z, int ftl,
                                                  int ntiles, int chunks, int parts, int64_t strideA,
                                                  int64_t strideM) {
    __shared__ uint32_t lf[64];
    const int b = blockIdx.x;
    const int tile = b % ntiles;
    const int rest = b / ntiles;
    const int part = rest % parts;
    const int rs = rest / parts;
    const int tid = threadIdx.x;
    const int FT = 1 << ftl;
    if (tid < 64) lf[tid] = 0u;
    __syncthreads();
    const RowDesc *rd = rows + rs;
    const float *At = A + (int64_t)tile * strideA;
    const uint8_t *St = Sil + (int64_t)tile * strideM;
    for (int c = part; c < chunks; c += parts) {
        const int idx = c * (int)blockDim.x + tid;
        if (idx < (Z << ftl)) {
            const int k = idx >> ftl;
            const int fl = idx & (FT - 1);
            uint32_t par = St[((rd->row * Z + k) << ftl) + fl] & 1u;
            for (int j = 0; j < rd->d; ++j) {
                int v = k + rd->shift[j];
                v = v >= Z ? v - Z : v;
                par ^= (uint32_t)(At[((rd->col[j] * Z + v) << ftl) + fl] < 0.0f);
            }
            if (rd->d1col >= 0) {
                int v = k + rd->d1shift;
                v = v >= Z ? v - Z : v;
                par ^= (uint32_t)(At[((rd->d1col * Z + v) << ftl) + fl] < 0.0f);
            }
            if (par) lf[fl] = 1u;
        }
    }
    __syncthreads();
    if (tid < FT && lf[tid]) atomicOr(&fail[tile * FT + tid], 1u);
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
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)ntiles);
    hipLaunchKernelGGL(k_to_tiles<float>, grid, dim3(256), 0, s, in, out, F, N, ft_log2);
    return hipGetLastError();
}

hipError_t qm_launch_to_tiles_u8(const uint8_t *in, uint8_t *out, int F, int64_t N, int ft_log2, int ntiles,
                                 hipStream_t s) {
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)ntiles);
    hipLaunchKernelGGL(k_to_tiles<uint8_t>, grid, dim3(256), 0, s, in, out, F, N, ft_log2);
    return hipGetLastError();
}

hipError_t qm_launch_kappa(const float *A, const uint8_t *Sil, float *K, const RowDesc *rows, int mb,
                           const TileGeom &g, hipStream_t s) {
    const int chunks = chunks_for(g.Z, g.ft_log2, 256);
    const int64_t blocks = (int64_t)g.ntiles * mb * chunks;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_kappa, dim3((unsigned)blocks), dim3(256), 0, s, A, Sil, K, rows, g.Z, g.ft_log2,
                       g.ntiles, chunks, (int64_t)g.n << g.ft_log2, (int64_t)g.m << g.ft_log2);
    return hipGetLastError();
}

hipError_t qm_launch_fill_u32(uint32_t *p, uint32_t v, size_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}

hipError_t qm_launch_layer(const LayerArgs &a, int msg16, int maxd, int block, hipStream_t s) {
    const int64_t blocks = (int64_t)a.ntiles * a.nrows * a.chunks;
    if (blocks == 0) return hipSuccess;
    dim3 grid((unsigned)blocks), tb((unsigned)block);
#define QM_LAYER_CASE(T, D)                                        \
    hipLaunchKernelGGL((k_layer_sp<T, D>), grid, tb, 0, s, a);     \
    break;
    if (!msg16) {
        switch (maxd) {
            case 4: QM_LAYER_CASE(float, 4)
            case 8: QM_LAYER_CASE(float, 8)
            default: QM_LAYER_CASE(float, 16)
        }
    } else {
        switch (maxd) {
            case 4: QM_LAYER_CASE(_Float16, 4)
            case 8: QM_LAYER_CASE(_Float16, 8)
            default: QM_LAYER_CASE(_Float16, 16)
        }
    }
#undef QM_LAYER_CASE
    return hipGetLastError();
}

hipError_t qm_launch_syndrome(const float *A, const uint8_t *Sil, const RowDesc *rows, int mb, uint32_t *fail,
                              const TileGeom &g, hipStream_t s) {
    const int chunks = chunks_for(g.Z, g.ft_log2, 256);
    const int parts = chunks < 16 ? chunks : 16;
    const int64_t blocks = (int64_t)g.ntiles * mb * parts;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_syndrome, dim3((unsigned)blocks), dim3(256), 0, s, A, Sil, rows, fail, g.Z, g.ft_log2,
                       g.ntiles, chunks, parts, (int64_t)g.n << g.ft_log2, (int64_t)g.m << g.ft_log2);
    return hipGetLastError();
}

hipError_t qm_launch_finalize(const float *A, const uint32_t *fail, float *app, uint8_t *hard, uint8_t *flags,
                              int F, const TileGeom &g, hipStream_t s) {
    dim3 grid((unsigned)((g.n + 63) / 64), (unsigned)g.ntiles);
    hipLaunchKernelGGL(k_finalize, grid, dim3(256), 0, s, A, fail, app, hard, flags, F, g.n, g.ft_log2);
    return hipGetLastError();
}

hipError_t qm_launch_validate(const float *llr, size_t nl, const uint8_t *syn, size_t ns, uint32_t *err,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_validate, dim3(1024), dim3(256), 0, s, llr, nl, syn, ns, err);
    return hipGetLastError();
}
