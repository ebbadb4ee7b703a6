// Synthetic training frames on the GPU: x uniform bits, BIAWGN channel
// LLRs and the syndrome s = H x (Methods, step 1: LLR = 2 y / sigma^2 with
// y = 1 - 2x + noise, sigma^2 = 1/SNR).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC 2011), a counter-based generator:
// each (frame, bit pair) is its own counter, so any frame can be drawn
// independently and reproducibly.  Counter (p, frame lo, frame hi, 0) with
// key (seed lo, seed hi) gives words r0..r3:
//   bit 2p = r2 >> 31, bit 2p+1 = r3 >> 31,
//   u1 = (r0 + 1/2) 2^-32, u2 = (r1 + 1/2) 2^-32,
//   Box-Muller: n0 = sqrt(-2 ln u1) cos(2 pi u2), n1 = sqrt(-2 ln u1) sin(2 pi u2).
#include "device_common.h"
#include "qcmet_internal.h"

namespace {

using namespace qmdev;

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint32_t hi0 = __umulhi(kPhiloxM0, c.x), lo0 = kPhiloxM0 * c.x;
        const uint32_t hi1 = __umulhi(kPhiloxM1, c.z), lo1 = kPhiloxM1 * c.z;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    }
    return c;
}

__global__ void __launch_bounds__(256) k_philox_frames(uint8_t *__restrict__ x, float *__restrict__ llr, int64_t n,
                                                       int F, uint64_t seed, uint64_t first, float snr) {
    const int f = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // bit pair
    if (f >= F || 2 * p >= n) return;
    const uint64_t frame = first + (uint64_t)f;
    const U4 r = philox4x32_10(U4{(uint32_t)p, (uint32_t)frame, (uint32_t)(frame >> 32), 0u}, (uint32_t)seed,
                               (uint32_t)(seed >> 32));
    const float u1 = ((float)r.x + 0.5f) * 2.3283064365386963e-10f;  // 2^-32
    const float u2 = ((float)r.y + 0.5f) * 2.3283064365386963e-10f;
    const float rad = sqrtf(-2.0f * logf(u1));
    float sn, cs;
    sincospif(2.0f * u2, &sn, &cs);
    const float sigma = sqrtf(1.0f / snr);
    const uint32_t b0 = r.z >> 31, b1 = r.w >> 31;
    const int64_t o = (int64_t)f * n + 2 * p;
    x[o] = (uint8_t)b0;
    llr[o] = 2.0f * snr * ((1.0f - 2.0f * (float)b0) + sigma * rad * cs);
    if (2 * p + 1 < n) {
        x[o + 1] = (uint8_t)b1;
        llr[o + 1] = 2.0f * snr * ((1.0f - 2.0f * (float)b1) + sigma * rad * sn);
    }
}

// s[f][i Z + k] = xor over the row's entries of x[f][col Z + (k + a) mod Z]
__global__ void __launch_bounds__(256) k_encode(const uint8_t *__restrict__ x, uint8_t *__restrict__ s,
                                                const RowDesc *rows, int mb, int Z, int64_t n, int64_t m) {
    const int f = blockIdx.z;
    const int rs = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Z) return;
    ConstRowDesc *rd = as_const(rows + rs);
    const uint8_t *xf = x + (int64_t)f * n;
    uint32_t par = 0;
    for (int j = 0; j < rd->d; ++j) {
        int v = k + rd->shift[j];
        v = v >= Z ? v - Z : v;
        par ^= xf[(int64_t)rd->col[j] * Z + v];
    }
    if (rd->d1col >= 0) {
        int v = k + rd->d1shift;
        v = v >= Z ? v - Z : v;
        par ^= xf[(int64_t)rd->d1col * Z + v];
    }
    s[(int64_t)f * m + (int64_t)rd->row * Z + k] = (uint8_t)(par & 1u);
}

}  // namespace

hipError_t qm_launch_framegen(uint8_t *x, float *llr, uint8_t *syn, const RowDesc *rows, int mb, int Z, int64_t n,
                              int64_t m, int F, uint64_t seed, uint64_t first, float snr, hipStream_t s) {
    if (F <= 0) return hipSuccess;
    const int64_t pairs = (n + 1) / 2;
    hipLaunchKernelGGL(k_philox_frames, dim3((unsigned)((pairs + 255) / 256), (unsigned)F), dim3(256), 0, s, x, llr,
                       n, F, seed, first, snr);
    hipLaunchKernelGGL(k_encode, dim3((unsigned)((Z + 255) / 256), (unsigned)mb, (unsigned)F), dim3(256), 0, s, x,
                       syn, rows, mb, Z, n, m);
    return hipGetLastError();
}
