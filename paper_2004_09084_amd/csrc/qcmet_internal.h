// Internal types of libqcmet shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Largest number of degree>=2 ("type-1") entries one base row may hold.
#define QM_MAXD 16

// Clip interval of the check-node transform: messages are kept in
// [Phi(30), 30] so that Phi stays finite (Results, kernel optimisations:
// values are clipped to avoid infinities; the bounds are this library's).
#define QM_X_HI 30.0f

// One base row of a layer, as the kernels read it (uniform per workgroup,
// so it lands in scalar registers).  This is the per-row form of the
// paper's packed index file: for every non-(-1) entry its shift and its
// block column, plus where its messages live.
struct RowDesc {
    int32_t row;              // base row i
    int32_t d;                // entries in degree>=2 columns
    int32_t d1col;            // the row's degree-1 column, or -1
    int32_t d1shift;          // its shift
    int32_t col[QM_MAXD];     // degree>=2 columns, ascending
    int32_t shift[QM_MAXD];   // their shifts
    int32_t ent[QM_MAXD];     // index of the entry among all degree>=2 entries (message slot)
};

// Device-side layout of one code's frames ("frame tiles"): frames are
// padded to Fpad and split into Fpad/FT tiles of FT frames; inside a tile
// every per-node array is [node][FT], so the FT frames of a node are
// adjacent and one wavefront reads 64/FT consecutive nodes of FT frames.
struct TileGeom {
    int32_t Z;
    int32_t ft_log2;
    int32_t ntiles;
    int64_t n, m;             // variables, checks
    int64_t nent1;            // degree>=2 entries (message rows of Z)
};

struct LayerArgs {
    float *A;                 // [ntiles][n][FT]  APP (degree>=2 cols), LLR/APP (degree-1 cols)
    void *R;                  // [ntiles][nent1*Z][FT]  check-to-variable messages
    const float *K;           // [ntiles][m][FT]  per-check degree-1 term (sign: s ^ [lam<0])
    const RowDesc *rows;      // rows of this layer
    int32_t nrows;
    int32_t Z;
    int32_t ft_log2;
    int32_t ntiles;
    int32_t chunks;           // workgroups per (tile, row)
    int32_t fpl;              // frames per lane (1, 2, 4)
    int32_t last;             // 1 in the last sweep: also form the degree-1 APPs
    int64_t strideA, strideR, strideK;  // per-tile strides (elements)
};

// Kernel launchers (kernels.hip).  All return hipError_t of the launch.
hipError_t qm_launch_to_tiles_f32(const float *in, float *out, int F, int64_t N, int ft_log2,
                                  int ntiles, hipStream_t s);
hipError_t qm_launch_to_tiles_u8(const uint8_t *in, uint8_t *out, int F, int64_t N, int ft_log2,
                                 int ntiles, hipStream_t s);
hipError_t qm_launch_kappa(const float *A, const uint8_t *Sil, float *K, const RowDesc *rows,
                           int mb, const TileGeom &g, hipStream_t s);
hipError_t qm_launch_fill_u32(uint32_t *p, uint32_t v, size_t count, hipStream_t s);
hipError_t qm_launch_layer(const LayerArgs &a, int msg16, int maxd, int fpl, int block, hipStream_t s);
hipError_t qm_launch_syndrome(const float *A, const uint8_t *Sil, const RowDesc *rows, int mb,
                              uint32_t *fail, const TileGeom &g, hipStream_t s);
hipError_t qm_launch_finalize(const float *A, const uint32_t *fail, float *app, uint8_t *hard,
                              uint8_t *flags, int F, const TileGeom &g, hipStream_t s);
hipError_t qm_launch_validate(const float *llr, size_t nl, const uint8_t *syn, size_t ns,
                              uint32_t *err, hipStream_t s);
