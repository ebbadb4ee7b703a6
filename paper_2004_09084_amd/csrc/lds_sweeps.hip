// LDS-resident layered sum-product (Methods, steps 2-4) for codes whose
// degree>=2 APPs of one frame fit in a compute unit's LDS (for example the
// rate-0.02 code: 2 x 10000 variables, 80 KB).  One workgroup decodes one
// frame through every sweep: the APPs live in LDS from the first layer to
// the last, layers are separated by workgroup barriers (frames never share
// state, so no barrier crosses workgroups), and only the messages and the
// per-check degree-1 terms stream through HBM.
//
// Per check the arithmetic is the tiled layer kernel's, operation for
// operation (same Phi, clip, exclusive prefix/suffix sums and rounding), so
// the two paths decode to identical bits.  A lane takes U checks of a row
// at a time (k, k + blockDim, ...) to keep several independent loads in
// flight (more checks per lane spill registers).
#include "qcmet_internal.h"
#include "device_common.h"
#include "phi.h"

#include <algorithm>

namespace {

using namespace qmdev;

// message element i of a frame's message array
template <typename MsgT> struct Msg;
template <> struct Msg<float> {
    static constexpr int bytes = 4;
    __device__ static float ld(const void *p, int64_t i) { return static_cast<const float *>(p)[i]; }
    __device__ static void st(void *p, int64_t i, float v) { static_cast<float *>(p)[i] = v; }
};
template <> struct Msg<_Float16> {
    static constexpr int bytes = 2;
    __device__ static float ld(const void *p, int64_t i) { return (float)static_cast<const _Float16 *>(p)[i]; }
    __device__ static void st(void *p, int64_t i, float v) { static_cast<_Float16 *>(p)[i] = (_Float16)v; }
};
template <> struct Msg<Fp8Msg> {
    static constexpr int bytes = 1;
    __device__ static float ld(const void *p, int64_t i) {
        return __builtin_amdgcn_cvt_f32_fp8((int)static_cast<const uint8_t *>(p)[i], 0);
    }
    __device__ static void st(void *p, int64_t i, float v) {
        static_cast<uint8_t *>(p)[i] = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false) & 0xff);
    }
};

// checks per lane and pass: enough independent loads in flight per lane
// without exceeding the register budget of 1024-lane workgroups
template <int D> struct ChecksPerLane { static constexpr int v = D <= 3 ? 8 : D <= 6 ? 4 : 2; };

template <typename MsgT, int D>
__device__ __forceinline__ void lds_checks(float *s_app, float *A, void *R, const float *K, ConstRowDesc *rd, int Z,
                                           int k0, int last) {
    constexpr int U = ChecksPerLane<D>::v;
    typedef MsgIO<MsgT> IO;
    typedef Msg<MsgT> M;
    const int stride = (int)blockDim.x;
    const int row = rd->row;
    int kk[U];  // this lane's checks; lanes past Z take check 0 and store nothing
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        kk[u] = k0 + u * stride;
        ok[u] = kk[u] < Z;
        kk[u] = ok[u] ? kk[u] : 0;
    }
    float kap[U];
    bool neg[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        kap[u] = K[(int64_t)row * Z + kk[u]];
        neg[u] = (int32_t)__float_as_uint(kap[u]) < 0;
    }
    float q[D > 0 ? D : 1][U], ph[D > 0 ? D : 1][U], suf[D > 0 ? D : 1][U];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const int sh = rd->shift[j];
        const int lc = rd->lcol[j];
        const int64_t eo = (int64_t)rd->ent[j] * Z;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int v = kk[u] + sh;
            v = v >= Z ? v - Z : v;
            const float av = s_app[lc * Z + v];
            const float rv = M::ld(R, eo + kk[u]);
            q[j][u] = av - rv;
            neg[u] = neg[u] != (q[j][u] < 0.0f);
            ph[j][u] = qm_phi(qm_clip(fabsf(q[j][u])));
        }
    }
    float acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = 0.0f;
#pragma unroll
    for (int j = D - 1; j >= 0; --j) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            suf[j][u] = acc[u];
            acc[u] += ph[j][u];
        }
    }
    float pre[U];
#pragma unroll
    for (int u = 0; u < U; ++u) pre[u] = fabsf(kap[u]);
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const int64_t eo = (int64_t)rd->ent[j] * Z;
        const int sh = rd->shift[j];
        const int lc = rd->lcol[j];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int v = kk[u] + sh;
            v = v >= Z ? v - Z : v;
            const float S = pre[u] + suf[j][u];
            pre[u] += ph[j][u];
            const bool nj = neg[u] != (q[j][u] < 0.0f);
            const float mag = qm_phi(qm_clip(S));
            const float rm = IO::round(nj ? -mag : mag);
            if (ok[u]) {
                s_app[lc * Z + v] = q[j][u] + rm;
                M::st(R, eo + kk[u], rm);
            }
        }
    }
    const int d1col = rd->d1col;
    if (last && d1col >= 0) {
        const int d1shift = rd->d1shift;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!ok[u]) continue;
            int v = kk[u] + d1shift;
            v = v >= Z ? v - Z : v;
            const int64_t ai = (int64_t)d1col * Z + v;
            const float lam = A[ai];
            const bool nd = neg[u] != (lam < 0.0f);
            const float mag = qm_phi(qm_clip(acc[u]));
            A[ai] = lam + IO::round(nd ? -mag : mag);
        }
    }
}

template <typename MsgT, int D>
__device__ __forceinline__ void lds_dispatch(int d, float *s_app, float *A, void *R, const float *K, ConstRowDesc *rd,
                                             int Z, int last) {
    if constexpr (D >= 0) {
        if (d == D) {
            constexpr int U = ChecksPerLane<D>::v;
            for (int k0 = (int)threadIdx.x; k0 < Z; k0 += U * (int)blockDim.x)
                lds_checks<MsgT, D>(s_app, A, R, K, rd, Z, k0, last);
            return;
        }
        lds_dispatch<MsgT, D - 1>(d, s_app, A, R, K, rd, Z, last);
    }
}

template <typename MsgT, int MAXD>
__global__ void __launch_bounds__(1024) k_sweeps_lds(const LdsArgs a) {
    extern __shared__ float s_app[];
    const int frame = (int)blockIdx.x;
    float *A = a.A + (int64_t)frame * a.n;
    void *R = static_cast<char *>(a.R) + (int64_t)frame * a.nr * Msg<MsgT>::bytes;
    const float *K = a.K + (int64_t)frame * a.m;
    const int Z = a.Z;
    const int n1 = a.ncols1 * Z;
    for (int i = (int)threadIdx.x; i < n1; i += (int)blockDim.x) {
        const int c = i / Z;
        s_app[i] = A[(int64_t)a.cols1[c] * Z + (i - c * Z)];
    }
    __syncthreads();
    for (int t = 0; t < a.T; ++t) {
        const int last = t == a.T - 1;
        for (int g = 0; g < a.G; ++g) {
            const int p1 = a.gptr[g + 1];
            for (int p = a.gptr[g]; p < p1; ++p) {
                ConstRowDesc *rd = as_const(a.rows + p);
                lds_dispatch<MsgT, MAXD>(rd->d, s_app, A, R, K, rd, Z, last);
            }
            __syncthreads();  // the next layer reads these APPs
        }
    }
    for (int i = (int)threadIdx.x; i < n1; i += (int)blockDim.x) {
        const int c = i / Z;
        A[(int64_t)a.cols1[c] * Z + (i - c * Z)] = s_app[i];
    }
}

template <typename MsgT, int MAXD>
hipError_t launch_lds_d(const LdsArgs &a, int F, size_t lds, hipStream_t s) {
    const void *fn = reinterpret_cast<const void *>(&k_sweeps_lds<MsgT, MAXD>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sweeps_lds<MsgT, MAXD>), dim3((unsigned)F), dim3(1024), lds, s, a);
    return hipGetLastError();
}

template <typename MsgT>
hipError_t launch_lds(const LdsArgs &a, int F, int maxd, size_t lds, hipStream_t s) {
    switch (maxd) {
        case 2: return launch_lds_d<MsgT, 2>(a, F, lds, s);
        case 3: return launch_lds_d<MsgT, 3>(a, F, lds, s);
        case 4: return launch_lds_d<MsgT, 4>(a, F, lds, s);
        case 5: return launch_lds_d<MsgT, 5>(a, F, lds, s);
        case 6: return launch_lds_d<MsgT, 6>(a, F, lds, s);
        case 8: return launch_lds_d<MsgT, 8>(a, F, lds, s);
        default: return hipErrorInvalidValue;  // rows of more than 8 degree>=2 entries use the tiled kernels
    }
}

}  // namespace

size_t qm_lds_bytes(int ncols1, int Z) { return (size_t)ncols1 * (size_t)Z * sizeof(float); }

hipError_t qm_launch_sweeps_lds(const LdsArgs &a, int F, int msgk, int maxd, hipStream_t s) {
    if (F == 0 || a.T == 0) return hipSuccess;
    const size_t lds = qm_lds_bytes(a.ncols1, a.Z);
    switch (msgk) {
        case QM_MSGK_F32: return launch_lds<float>(a, F, maxd, lds, s);
        case QM_MSGK_F16: return launch_lds<_Float16>(a, F, maxd, lds, s);
        case QM_MSGK_F8: return launch_lds<Fp8Msg>(a, F, maxd, lds, s);
        default: return hipErrorInvalidValue;
    }
}
