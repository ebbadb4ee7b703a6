// Device-side helpers shared by the kernels of libqcmet (gfx950, wave64).
#pragma once

#include "qcmet_internal.h"

namespace qmdev {

constexpr float kXLo = 1.87152459e-13f;  // Phi(30), lower clip bound of the check-node transform

// clip to [Phi(30), 30] in one v_med3_f32
__device__ __forceinline__ float qm_clip(float x) { return __builtin_amdgcn_fmed3f(x, kXLo, QM_X_HI); }


// magnitude (>= 0) with the sign bit set iff neg
__device__ __forceinline__ float with_sign(float mag, uint32_t neg) {
    return __uint_as_float(__float_as_uint(mag) | (neg << 31));
}

// ---- buffer access: every array of a frame tile is addressed through a
// buffer resource (base = tile start, range = tile bytes), a wave-uniform
// SGPR offset (block column / message slot / check row) and a 32-bit VGPR
// offset inside that column.  No 64-bit address arithmetic per lane, and an
// access outside the tile range is dropped by the hardware range check.
constexpr int kRsrcWord3 = 0x00020000;  // gfx9 raw buffer: 32-bit data format

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kRsrcWord3);
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// N adjacent float32 values.  AUX is the cache-policy operand of the buffer
// instruction: 0 = default, 2 = non-temporal (streamed data that is not
// reused soon, so it should not displace reused lines).
template <int N, int AUX = 0>
__device__ __forceinline__ void bload_f32(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float (&v)[N]) {
    if constexpr (N == 1) {
        v[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
    } else if constexpr (N == 2) {
        const u32x2 t = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX);
        v[0] = __uint_as_float(t.x);
        v[1] = __uint_as_float(t.y);
    } else {
        const u32x4 t = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX);
        v[0] = __uint_as_float(t.x);
        v[1] = __uint_as_float(t.y);
        v[2] = __uint_as_float(t.z);
        v[3] = __uint_as_float(t.w);
    }
}
template <int N, int AUX = 0>
__device__ __forceinline__ void bstore_f32(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, const float (&v)[N]) {
    if constexpr (N == 1) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[0]), r, voff, soff, AUX);
    } else if constexpr (N == 2) {
        u32x2 t;
        t.x = __float_as_uint(v[0]);
        t.y = __float_as_uint(v[1]);
        __builtin_amdgcn_raw_buffer_store_b64(t, r, voff, soff, AUX);
    } else {
        u32x4 t;
        t.x = __float_as_uint(v[0]);
        t.y = __float_as_uint(v[1]);
        t.z = __float_as_uint(v[2]);
        t.w = __float_as_uint(v[3]);
        __builtin_amdgcn_raw_buffer_store_b128(t, r, voff, soff, AUX);
    }
}

// messages: float32, or binary16 widened to float32 (conversion to binary16
// rounds to nearest even)
template <typename MsgT> struct MsgIO;
template <> struct MsgIO<float> {
    static constexpr uint32_t bytes = 4;
    template <int N, int AUX = 0>
    __device__ static __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float (&v)[N]) {
        bload_f32<N, AUX>(r, vo, so, v);
    }
    __device__ static __forceinline__ float round(float x) { return x; }
    template <int N, int AUX = 0>
    __device__ static __forceinline__ void store(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, const float (&v)[N]) {
        bstore_f32<N, AUX>(r, vo, so, v);
    }
};
template <> struct MsgIO<_Float16> {
    static constexpr uint32_t bytes = 2;
    __device__ static __forceinline__ uint32_t pack2(float a, float b) {
        const _Float16 ha = (_Float16)a, hb = (_Float16)b;
        return (uint32_t)__builtin_bit_cast(uint16_t, ha) | ((uint32_t)__builtin_bit_cast(uint16_t, hb) << 16);
    }
    __device__ static __forceinline__ float lo(uint32_t w) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu)); }
    __device__ static __forceinline__ float hi(uint32_t w) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16)); }
    template <int N, int AUX = 0>
    __device__ static __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float (&v)[N]) {
        if constexpr (N == 1) {
            const uint16_t t = __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, AUX);
            v[0] = (float)__builtin_bit_cast(_Float16, t);
        } else if constexpr (N == 2) {
            const uint32_t t = __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, AUX);
            v[0] = lo(t);
            v[1] = hi(t);
        } else {
            const u32x2 t = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, AUX);
            v[0] = lo(t.x);
            v[1] = hi(t.x);
            v[2] = lo(t.y);
            v[3] = hi(t.y);
        }
    }
    __device__ static __forceinline__ float round(float x) { return (float)(_Float16)x; }
    template <int N, int AUX = 0>
    __device__ static __forceinline__ void store(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, const float (&v)[N]) {
        if constexpr (N == 1) {
            __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, (_Float16)v[0]), r, vo, so, AUX);
        } else if constexpr (N == 2) {
            __builtin_amdgcn_raw_buffer_store_b32(pack2(v[0], v[1]), r, vo, so, AUX);
        } else {
            u32x2 t;
            t.x = pack2(v[0], v[1]);
            t.y = pack2(v[2], v[3]);
            __builtin_amdgcn_raw_buffer_store_b64(t, r, vo, so, AUX);
        }
    }
};

// 8-bit float messages (4 exponent bits, 3 mantissa bits), converted by the
// hardware (round to nearest even); the tag type only selects the storage.
struct Fp8Msg {};
template <> struct MsgIO<Fp8Msg> {
    static constexpr uint32_t bytes = 1;
    __device__ static __forceinline__ float at(uint32_t w, int i) {
        switch (i) {
            case 0: return __builtin_amdgcn_cvt_f32_fp8((int)w, 0);
            case 1: return __builtin_amdgcn_cvt_f32_fp8((int)w, 1);
            case 2: return __builtin_amdgcn_cvt_f32_fp8((int)w, 2);
            default: return __builtin_amdgcn_cvt_f32_fp8((int)w, 3);
        }
    }
    // two values into the low 16 bits of a word
    __device__ static __forceinline__ uint32_t pack2(float a, float b) {
        return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xffffu;
    }
    template <int N, int AUX = 0>
    __device__ static __forceinline__ void load(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float (&v)[N]) {
        if constexpr (N == 1) {
            v[0] = at((uint32_t)__builtin_amdgcn_raw_buffer_load_b8(r, vo, so, AUX), 0);
        } else if constexpr (N == 2) {
            const uint32_t t = (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, vo, so, AUX);
            v[0] = at(t, 0);
            v[1] = at(t, 1);
        } else {
            const uint32_t t = __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, AUX);
            v[0] = at(t, 0);
            v[1] = at(t, 1);
            v[2] = at(t, 2);
            v[3] = at(t, 3);
        }
    }
    __device__ static __forceinline__ float round(float x) { return at(pack2(x, 0.0f), 0); }
    template <int N, int AUX = 0>
    __device__ static __forceinline__ void store(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, const float (&v)[N]) {
        if constexpr (N == 1) {
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)pack2(v[0], 0.0f), r, vo, so, AUX);
        } else if constexpr (N == 2) {
            __builtin_amdgcn_raw_buffer_store_b16((uint16_t)pack2(v[0], v[1]), r, vo, so, AUX);
        } else {
            const uint32_t t = pack2(v[0], v[1]) | (pack2(v[2], v[3]) << 16);
            __builtin_amdgcn_raw_buffer_store_b32(t, r, vo, so, AUX);
        }
    }
};

template <int FPL> struct LogOf;
template <> struct LogOf<1> { static constexpr int v = 0; };
template <> struct LogOf<2> { static constexpr int v = 1; };

// Row descriptors are read through the constant address space: they are
// never written while a kernel runs, so every field becomes a scalar load.
typedef const __attribute__((address_space(4))) RowDesc ConstRowDesc;
__device__ __forceinline__ ConstRowDesc *as_const(const RowDesc *p) { return (ConstRowDesc *)p; }
typedef const __attribute__((address_space(4))) ColDesc ConstColDesc;
__device__ __forceinline__ ConstColDesc *as_const_col(const ColDesc *p) { return (ConstColDesc *)p; }

// packed frame bits: a field of esz bytes (1, 2, 4 or 8) at index i
__device__ __forceinline__ void store_packed(uint8_t *p, int64_t i, int esz, uint64_t w) {
    switch (esz) {
        case 1: p[i] = (uint8_t)w; break;
        case 2: reinterpret_cast<uint16_t *>(p)[i] = (uint16_t)w; break;
        case 4: reinterpret_cast<uint32_t *>(p)[i] = (uint32_t)w; break;
        default: reinterpret_cast<uint64_t *>(p)[i] = w; break;
    }
}
__device__ __forceinline__ uint64_t load_packed(const uint8_t *p, int64_t i, int esz) {
    switch (esz) {
        case 1: return p[i];
        case 2: return reinterpret_cast<const uint16_t *>(p)[i];
        case 4: return reinterpret_cast<const uint32_t *>(p)[i];
        default: return reinterpret_cast<const uint64_t *>(p)[i];
    }
}

// Per-lane context of one layer update.
struct LaneCtx {
    __amdgpu_buffer_rsrc_t rA, rR, rK;
    uint32_t node;   // in-column element index of (k, first frame of the lane)
    uint32_t colw;   // elements per block column of a tile (Z * FT)
    int k, Z, ftl;
    int last;        // last sweep of the decode
};

// byte offset of variable (k + a) mod Z inside its block column
__device__ __forceinline__ uint32_t shifted_off(const LaneCtx &c, int sh) {
    uint32_t off = c.node + ((uint32_t)sh << c.ftl);
    off = (c.k >= c.Z - sh) ? off - c.colw : off;
    return off * 4u;
}


}  // namespace qmdev
