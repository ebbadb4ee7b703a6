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
    int32_t d1pos;            // its position among the row's columns (ascending column order)
    int32_t col[QM_MAXD];     // degree>=2 columns, ascending
    int32_t shift[QM_MAXD];   // their shifts
    int32_t ent[QM_MAXD];     // index of the entry among all degree>=2 entries (message slot)
    int32_t lcol[QM_MAXD];    // rank of the column among the degree>=2 columns (LDS-resident decode)
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
    // early termination (null otherwise): every sweep forms the degree-1
    // hard decisions and keeps in A's degree-1 slots clip(S) with r_d's sign
    // (the APP is formed when the frame stops), reading the channel LLRs of
    // the degree-1 variables from Ad where the exact sum decides; frames
    // whose tmask bit is 0 are left untouched; tiles at or past ctl[1] are
    // skipped, and the grid may cover fewer than ntiles tiles (any count
    // >= ctl[1])
    const float *Ad;          // [ntiles][m][FT] LLR of each check's degree-1 variable
    const uint64_t *tmask;    // [ntiles] frames of each tile still decoding (bit fl)
    const int32_t *ctl;       // EtCtl
    uint8_t *Pd;              // [ntiles][m] hard decisions of the FT frames of each check's degree-1
                              // variable (bit = frame), max(FT, 8) bits each
    const uint8_t *PS;        // [ntiles][m] syndrome bits, packed the same way
    uint32_t shmem;           // dynamic LDS bytes requested per workgroup; the kernels do not use
                              // it, it only caps how many workgroups a compute unit holds
};

// bytes of one packed field of FT = 2^ft_log2 frame bits
__host__ __device__ inline int qm_pack_bytes(int ft_log2) { return ft_log2 <= 3 ? 1 : (1 << (ft_log2 - 3)); }
// bit of frame fl of a tile in a packed field, with fpl frames per lane:
// frame j*fpl + f (lane j of the check's lane group, its frame f) sits at
// bit f*(FT/fpl) + j
__host__ __device__ inline int qm_pack_bit(int fl, int ft_log2, int fpl) {
    const int lpc = (1 << ft_log2) / fpl;
    return (fl % fpl) * lpc + fl / fpl;
}

// Device-side control words of an early-terminating decode of one code.
//   [0] nact: slots >= nact hold stopped frames
//   [1] tiles that still hold a decoding frame (ceil(nact / FT))
//   [2] 1: the planning kernel planned a compaction (perm, from slot ctl[3])
//   [3] first slot the compaction writes
//   [4] frames that stopped in the last planning call (outputs to write)
//   [5] frames still decoding
#define QM_ET_CTL_WORDS 8
// Largest padded frame count of one code in an early-terminating decode
// (the planning kernel keeps per-slot state in LDS).
#define QM_ET_MAXF 8192

// One code decoded with its degree>=2 APPs resident in LDS: one workgroup
// per frame runs every sweep, layers separated by workgroup barriers.
// Frame-major layout (frame tiles of one frame).
struct LdsArgs {
    float *A;                 // [F][n]  APP (degree>=2 cols), LLR/APP (degree-1 cols)
    void *R;                  // [F][nent1*Z] messages
    const float *K;           // [F][m]  degree-1 terms
    const RowDesc *rows;      // all rows, schedule order
    const int32_t *gptr;      // [G+1] layer boundaries
    const int32_t *cols1;     // [ncols1] degree>=2 block columns, in LDS order
    int32_t G, Z, T, ncols1;
    int64_t n, m, nr;         // per-frame elements of A, K, R
};

// Flooding schedule: one degree>=2 column and its entries in ascending row
// order (the order its messages are added in).
#define QM_MAXCD 128
struct ColDesc {
    int32_t col;              // block column
    int32_t deg;              // entries (rows) in the column
    int32_t ent[QM_MAXCD];    // message slot of each entry
    int32_t shift[QM_MAXCD];  // its shift: row check k meets variable (k + shift) mod Z
};

// Codes one decoder can mix in a single fused launch.
#define QM_MAX_CODES 4

struct MultiLayerArgs {
    LayerArgs code[QM_MAX_CODES];          // this step's layer of each code
    int32_t block_off[QM_MAX_CODES + 1];   // workgroup ranges per code
    int32_t ncodes;
};

// Min-sum (learned decoder) layer arguments.
struct NmsLayerArgs {
    LayerArgs L;              // A, R (float32), K = |LLR_d| with sign s ^ [LLR_d < 0]; L.last = 1:
                              // also form the degree-1 APPs into Ad
    float *Ad;                // [ntiles][m][FT] degree-1 APP per check
    float *Q;                 // [ntiles][nent1*Z][FT] q recorded for the backward pass, or null
    const float *W;           // this sweep's weights [mb][2 target types][alpha, beta]
    const uint32_t *act;      // [Fpad] per-frame active flags (early termination), or null
    const uint64_t *tmask;    // [ntiles] the same per tile (bit fl), with act
};

struct NmsBwdArgs {
    LayerArgs L;              // A (LLR in degree-1 columns), K, rows, geometry; L.last = last sweep
    const float *Q;           // q of this sweep (recomputed)
    float *gA;                // [ntiles][n][FT] dLoss/dAPP (in/out)
    float *gR;                // [ntiles][nent1*Z][FT] dLoss/dr from later sweeps (in/out; not read
                              // in the loss term's own sweep, L.last, which starts it)
    const float *gAd;         // [ntiles][m][FT] dLoss/dAPP of degree-1 variables (last sweep)
    const float *W;           // this sweep's weights
    float *part;              // per-workgroup sums [T][mb][ntiles][chunks][4], accumulated
    int32_t *clamps;          // adjoint components that reached the bound (device counter)
    int32_t t, mb;
};

// Kernel launchers (kernels.hip).  All return hipError_t of the launch.
hipError_t qm_launch_to_tiles_f32(const float *in, float *out, int F, int64_t N, int ft_log2,
                                  int ntiles, hipStream_t s);
hipError_t qm_launch_to_tiles_u8(const uint8_t *in, uint8_t *out, int F, int64_t N, int ft_log2,
                                 int ntiles, hipStream_t s);
hipError_t qm_launch_kappa(const float *A, const uint8_t *Sil, float *K, const RowDesc *rows,
                           int mb, const TileGeom &g, hipStream_t s);
hipError_t qm_launch_fill_u32(uint32_t *p, uint32_t v, size_t count, hipStream_t s);
// message storage kinds (msgk)
#define QM_MSGK_F32 0
#define QM_MSGK_F16 1
#define QM_MSGK_F8 2
hipError_t qm_launch_layer(const LayerArgs &a, int msgk, int maxd, int fpl, int block, int hint, hipStream_t s);
hipError_t qm_launch_layer_multi(const MultiLayerArgs &m, int msgk, int maxd, int fpl, int block, int hint,
                                 hipStream_t s);
hipError_t qm_launch_syndrome(const float *A, const float *Ad, const uint8_t *Sil, const RowDesc *rows, int mb,
                              uint32_t *fail, const TileGeom &g, hipStream_t s);
hipError_t qm_launch_finalize(const float *A, const uint32_t *fail, float *app, uint8_t *hard,
                              uint8_t *flags, int F, const TileGeom &g, hipStream_t s);
// LDS-resident decode (lds_sweeps.hip): all T sweeps of F frames in one
// launch; bytes of LDS it needs per workgroup, and the launch.
size_t qm_lds_bytes(int ncols1, int Z);
hipError_t qm_launch_sweeps_lds(const LdsArgs &a, int F, int msgk, int maxd, hipStream_t s);
// flooding schedule (kernels.hip): the check half of an iteration, then the
// variable half APP = LLR + sum of the column's messages (ascending rows);
// Lam holds the channel LLRs of the ncols1 degree>=2 columns, [tile][c*Z][FT].
hipError_t qm_launch_layer_flood(const LayerArgs &a, int msgk, int maxd, int fpl, int block, int hint, hipStream_t s);
hipError_t qm_launch_flood_vars(float *A, const float *Lam, const void *R, const ColDesc *cols, int ncols1, int msgk,
                                int fpl, int block, const TileGeom &g, hipStream_t s);
hipError_t qm_launch_copy_cols(const float *A, float *Lam, const int32_t *cols1, int ncols1, const TileGeom &g,
                               hipStream_t s);
// early termination (kernels.hip)
hipError_t qm_launch_layer_et(const LayerArgs &a, int msgk, int maxd, int fpl, int block, int hint, hipStream_t s);
hipError_t qm_launch_syndrome_et(const float *A, const float *Ad, const uint8_t *Sil, const RowDesc *rows, int mb,
                                 uint32_t *fail, const int32_t *ctl, const TileGeom &g, hipStream_t s);
// Syndrome test from packed hard decisions (early termination): per check,
// the row's variables' words of PA (packed hard decisions per variable), the
// check's word of Pd and the syndrome
// bytes; tiles at or past ctl[1] are skipped.
hipError_t qm_launch_syndrome_packed(const uint8_t *PA, const uint8_t *Pd, const uint8_t *PS, const RowDesc *rows,
                                     int mb, uint32_t *fail, const int32_t *ctl, int fpl, const TileGeom &g,
                                     hipStream_t s);
// Packed hard decisions of every frame tile: bit qm_pack_bit(fl) of
// P[tile][node] = [X[tile][node][fl] < 0].
hipError_t qm_launch_pack_signs(const float *X, uint8_t *P, int64_t N, int fpl, const TileGeom &g, hipStream_t s);
// Packed hard decisions of the degree>=2 columns of the tiles below ctl[1].
hipError_t qm_launch_pack_cols(const float *A, uint8_t *P, const int32_t *cols1, int ncols1, const int32_t *ctl, int fpl,
                               const TileGeom &g, hipStream_t s);
// Packed syndrome bits (same order) of the tiles below ctl[1]; with
// after_compaction, only when the planning kernel moved frames (ctl[2] != 0).
hipError_t qm_launch_pack_syndrome(const uint8_t *Sil, uint8_t *PS, const int32_t *ctl, int after_compaction, int fpl,
                                   const TileGeom &g, hipStream_t s);
hipError_t qm_launch_et_init(uint32_t *act, uint64_t *tmask, int32_t *map, int32_t *iters, int32_t *ctl, int Fpad,
                             int ntiles, int ft_log2, hipStream_t s);
hipError_t qm_launch_et_plan(uint32_t *fail, uint32_t *act, uint64_t *tmask, int32_t *map, int32_t *perm,
                             int32_t *iters, int32_t *emit, uint8_t *flags, int F, int32_t *ctl, int Fpad, int ft_log2,
                             int t, int final_pass, hipStream_t s);
// frame-major APPs and hard decisions of the frames the planning kernel
// stopped (emit[slot] = frame or -1), from the first g.ntiles tiles; the
// degree-1 APPs are formed from A's signed sums and Ad's channel LLRs for
// frames that ran at least one sweep (iters); d1row[c] is the schedule
// index of the row whose degree-1 column is block column c, or -1
hipError_t qm_launch_emit(const float *A, const float *Ad, const int32_t *emit, const int32_t *ctl,
                          const int32_t *iters, const RowDesc *rows, const int32_t *d1row, int msgk, float *app,
                          uint8_t *hard, const TileGeom &g, hipStream_t s);
// move the planned frames (slot perm[s] into slot s) in every per-node array
struct CompactArray {
    void *p;                  // [ntiles][N][FT] elements of esz bytes
    int64_t N;
    int32_t esz;              // 1, 2 or 4
};
#define QM_COMPACT_ARRAYS 5
hipError_t qm_launch_compact(const CompactArray *arr, int narr, const int32_t *perm, const int32_t *ctl,
                             int ft_log2, hipStream_t s);
// moving the frames still decoding (all in tile 0) into a tile of
// 2^ft_log2_new slots: src[k] = the old slot that new slot k takes (-1:
// none), with map, act, the tile mask and the control words updated
hipError_t qm_launch_et_narrow_plan(uint32_t *act, uint64_t *tmask, int32_t *map, int32_t *src, int32_t *ctl,
                                    int ft_log2_old, int ft_log2_new, hipStream_t s);
// out[node][k] = in[node][src[k]] for k < 2^ft_log2_out (tile 0 of a layout
// of 2^ft_log2_in frames per tile; N nodes, esz-byte elements; in and out
// must not overlap)
hipError_t qm_launch_narrow(const void *in, void *out, const int32_t *src, int64_t N, int esz, int ft_log2_in,
                            int ft_log2_out, hipStream_t s);
// nms.hip
hipError_t qm_launch_nms_kappa(const float *A, const uint8_t *Sil, float *K, const RowDesc *rows, int mb,
                               const TileGeom &g, hipStream_t s);
hipError_t qm_launch_nms_layer(const NmsLayerArgs &na, int maxd, int fpl, int block, hipStream_t s);
hipError_t qm_launch_nms_bwd(const NmsBwdArgs &ba, int maxd, int fpl, int block, hipStream_t s);
// to_A = 1: A[d1col][(k + a) mod Z] = Ad[row][k]; to_A = 0: the reverse.
hipError_t qm_launch_commit_d1(float *A, float *Ad, int to_A, const RowDesc *rows, int mb, const TileGeom &g,
                               hipStream_t s);
hipError_t qm_launch_et_update(uint32_t *fail, uint32_t *act, uint64_t *tmask, int32_t *iters, int Fpad, int ft_log2,
                               int done, hipStream_t s);
// tmask[tile] = bits fl of the slots tile*FT + fl with act != 0
hipError_t qm_launch_tile_masks(const uint32_t *act, uint64_t *tmask, int Fpad, int ft_log2, hipStream_t s);
hipError_t qm_launch_et_final(const uint32_t *act, int32_t *iters, int Fpad, int T, hipStream_t s);
int qm_bce_blocks(int ncols, int mb, const TileGeom &g);
hipError_t qm_launch_bce(const float *A, const float *Ad, const uint8_t *X, float *gA, float *gAd, float *part,
                         const int32_t *cols, int ncols, const RowDesc *rows, int mb, const TileGeom &g, int F,
                         float weight, int accumulate, float *loss, hipStream_t s);
// grad[t][i][c] = the sum of the per-workgroup partials of (t, i, c) over
// nsets partial sets, set_stride floats apart (double accumulation, fixed order)
hipError_t qm_launch_grad_reduce(const float *part, float *grad, int T, int mb, int per_row, int nsets,
                                 size_t set_stride, hipStream_t s);
hipError_t qm_launch_adam(float *w, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                          int step, hipStream_t s);

// framegen.hip
hipError_t qm_launch_framegen(uint8_t *x, float *llr, uint8_t *syn, const RowDesc *rows, int mb, int Z, int64_t n,
                              int64_t m, int F, uint64_t seed, uint64_t first, float snr, hipStream_t s);

hipError_t qm_launch_validate(const float *llr, size_t nl, const uint8_t *syn, size_t ns,
                              uint32_t *err, hipStream_t s);

// Host runtime entry points shared with the allocation-free decode
// (noalloc.hip).
struct qm_decoder;
int qm_set_error(int code, const char *msg);
int qm_decode_on_workspace(qm_decoder *d, char *ws, size_t ws_bytes, const float *llr, const uint8_t *syn,
                           int32_t iters, uint8_t *hard, float *app, uint8_t *flags, hipStream_t st);
