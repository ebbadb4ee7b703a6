/*
 * qcmet.h -- C ABI of libqcmet: layered belief-propagation decoding of
 * quasi-cyclic (multi-edge-type) LDPC codes in syndrome form on gfx950.
 *
 * Method: Li et al., arXiv 2004.09084 (Methods, steps 1-4: layered
 * sum-product with the syndrome flip; Results: merged layers of rows with
 * disjoint columns, many codewords decoded in parallel, one fused check/
 * variable update per layer).
 *
 * Conventions for every entry point
 *  - Every call returns QM_OK (0) or a negative QM_ERR_* code; no call
 *    throws.  qm_last_error() gives a message for the calling thread, valid
 *    until that thread's next call.
 *  - "host" pointers are read during the call only; the library copies what
 *    it keeps.  "device" pointers are HIP device allocations owned by the
 *    caller; they must stay valid until the work queued on the given stream
 *    has completed.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Decoding calls are asynchronous on that stream; HIP errors raised by
 *    queued work surface at the caller's next synchronisation.
 *  - Bits are uint8 holding 0 or 1.  LLRs follow the paper's sign: LLR > 0
 *    favours bit 0 (BPSK 0 -> +1), and a hard decision is 1 iff APP < 0.
 *  - Calls on one decoder must not overlap (they share its workspace).
 */
#ifndef QCMET_H
#define QCMET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QM_ABI_VERSION 1

enum qm_status {
    QM_OK = 0,
    QM_ERR_INVALID_ARG = -1,       /* NULL pointer, value out of range */
    QM_ERR_SHAPE = -2,             /* sizes inconsistent with the code/decoder */
    QM_ERR_SCHEDULE_CONFLICT = -3, /* rows of one layer share a block column */
    QM_ERR_NO_WORKSPACE = -4,      /* decode before a large-enough workspace is bound */
    QM_ERR_OOM = -5,               /* host allocation failed */
    QM_ERR_HIP = -6,               /* a HIP runtime call failed */
    QM_ERR_INPUT = -7,             /* QM_VALIDATE: non-finite LLR or syndrome bit > 1 */
    QM_ERR_UNSUPPORTED = -8,       /* code structure outside what the kernels handle */
    QM_ERR_STATE = -9              /* call order violated (e.g. backward without forward) */
};

/* Decoder flags (qm_decoder_create). */
#define QM_MSG_FP32   0x0  /* check-to-variable messages stored as float32 */
#define QM_MSG_FP16   0x1  /* messages stored as IEEE binary16 (round to nearest even);
                              all arithmetic and the APP LLRs stay float32 */
#define QM_MSG_FP8    0x2  /* messages stored as 8-bit floats (1 sign, 4 exponent, 3 mantissa
                              bits; round to nearest even by the hardware conversion); all
                              arithmetic and the APP LLRs stay float32.  Excludes QM_MSG_FP16 */
#define QM_VALIDATE   0x4  /* qm_decode checks inputs first (synchronises the stream) */
#define QM_GRAPH      0x8  /* replay the whole decode (every code, every sweep) as one captured
                              hipGraph, re-captured when buffers or iters change */
#define QM_FLOODING   0x20 /* qm_decode runs the flooding schedule instead of layers: per
                              iteration every check updates from the previous iteration's
                              APPs (one launch over all rows), then every variable takes
                              APP = LLR + its messages added in ascending row order.  Not with
                              QM_EARLY_STOP or the min-sum decoder; columns of at most 128
                              entries.  Workspace per frame: 4 B per degree>=2 variable. */
#define QM_EARLY_STOP 0x10 /* reserve the workspace of qm_decode_early (per code and frame:
                              6 B per check, 1 B per variable and 20 B; at most 8192
                              frames per code) */

typedef struct qm_code qm_code;
typedef struct qm_decoder qm_decoder;

typedef struct {
    int32_t mb, nb, Z;        /* base matrix rows, columns, lifting factor */
    int64_t n, m;             /* code length nb*Z, number of checks mb*Z */
    int32_t n_type1_cols;     /* block columns of degree >= 2 */
    int32_t n_deg1_cols;      /* block columns of degree 1 (deferred, see qm_decode) */
    int32_t n_type1_entries;  /* non-(-1) entries in degree >= 2 columns */
    int32_t max_row_type1;    /* largest number of such entries in one row */
    int64_t edges;            /* Tanner-graph edges (all entries times Z) */
    int32_t G;                /* layers in the current schedule */
} qm_code_info;

/* Tuning knobs that never change results (see qm_autotune). */
typedef struct {
    int32_t frames_per_tile;  /* FT: frames interleaved fastest in HBM; power of two
                                 dividing the padded frame count; 0 = default */
    int32_t block;            /* threads per workgroup of the layer kernel (64..256, mult. of 64) */
    int32_t merge;            /* 1: run each merged layer as one launch; 0: one launch per row
                                 (same row order, bit-identical results) */
    int32_t graph;            /* 1: replay a captured hipGraph (as QM_GRAPH) */
    int32_t frames_per_lane;  /* 1 or 2 adjacent frames per GPU lane (<= frames_per_tile);
                                 0 = default (2).  4 is rejected (QM_ERR_UNSUPPORTED). */
    int32_t fuse_codes;       /* with several codes (at most 4) and merge = 1: 1, one launch runs
                                 the current layer of every code (each code walks its own layer
                                 sequence); 2, each code runs its own layer sequence on its own
                                 stream, forked from and joined to the decode stream (launches
                                 of different codes overlap; the default); 0, the codes are swept
                                 one after another.  Results are bit-identical in every mode. */
    int32_t stream_hint;      /* 1: messages and per-check terms are read and written with the
                                 non-temporal cache policy (they are used once per sweep), so the
                                 APP columns that the next layers reuse stay cached */
    int32_t lds_resident;     /* 1: a code whose degree>=2 APPs of one frame fit in one workgroup's
                                 LDS (at most 8 such entries per row) is decoded by one workgroup
                                 per frame that keeps those APPs in LDS through every sweep, with
                                 workgroup barriers between layers (one launch per decode; such a
                                 code uses one frame per tile).  2 (default): the same, only for a
                                 code with at least as many frames as the device has compute
                                 units (with fewer, compute units stay idle and the layer kernels
                                 are faster).  0: never.  Decoders created with QM_FLOODING or
                                 QM_EARLY_STOP, or with a min-sum workspace bound, always use the
                                 layer kernels.  Bit-identical to the layer kernels. */
    int32_t tile_groups;      /* 1, 2, 4 or 8 (0 = 1): a layered decode of one code splits its frame
                                 tiles into this many groups (fewer if it does not divide the
                                 tile count), each running its own layer sequence on its own
                                 stream, forked from and joined to the decode stream; one
                                 group's launch fills the ramp-down of another's.  Frames never
                                 depend on other frames, so results are bit-identical.  Not used
                                 by fused mixed batches, flooding or early termination. */
    int32_t spread_codes;     /* fused mixed batches: 1 (default) spreads each code's layers evenly
                                 over the launches (the code with the most layers runs in every
                                 launch, a code with a third as many in every third), so every
                                 launch carries a similar share of the traffic; 0 runs every code
                                 from the first launch until its layers are done.  Each code
                                 keeps its own layer order, so results are bit-identical. */
    int32_t frames_per_batch; /* layered decode of one code: frames whose sweeps run together.  With
                                 more frames, whole frame tiles are decoded in batches, one batch's
                                 sweeps after another's (each launch then touches one batch's state:
                                 past about 12 GiB of per-frame state, address translation slows
                                 every launch).  0 (default): all frames while their state stays
                                 within 12 GiB, else batches of the largest power-of-two tile count
                                 within it; otherwise rounded down to whole tiles (at least one).
                                 Frames never
                                 depend on other frames, so results are bit-identical. */
    int32_t resident_cap;     /* codes on their own streams (fuse_codes 2): workgroups per compute
                                 unit that the layer launches of every code but the one with the
                                 most layers per sweep may hold at once, so the launches of that
                                 longest chain (which bounds the decode) find free slots.  Applied
                                 as a request of (LDS per compute unit) / resident_cap bytes of
                                 dynamic LDS that the kernels leave unused.  0: no cap; otherwise
                                 3..64 (default 10, measured with 128-lane workgroups).  Results
                                 are bit-identical. */
} qm_tuning;

int qm_abi_version(void);
const char *qm_last_error(void);

/* Loads a QC base matrix (paper, Results: a non-negative entry a is the
 * Z x Z identity cyclically shifted right by a, i.e. check row k of block row
 * i meets variable (k + a) mod Z of block column j; -1 is an all-zero block).
 *   shifts: host int32 [mb*nb], row-major, each -1 or in [0, Z).
 * Columns with exactly one non-(-1) entry are degree-1 columns; a row may
 * hold at most one of them (QM_ERR_UNSUPPORTED otherwise), and at most 16
 * entries in degree >= 2 columns.  The default schedule is the greedy merge
 * of rows with disjoint columns (Results, Eq. (m)-(m2)): open a layer with
 * the first unassigned row, add every later unassigned row disjoint from it,
 * repeat; layers ordered by their first row.
 *   out: receives the new code (free with qm_code_destroy). */
int qm_code_create(int32_t mb, int32_t nb, int32_t Z, const int32_t *shifts, qm_code **out);
int qm_code_destroy(qm_code *code);
int qm_code_get_info(const qm_code *code, qm_code_info *info);

/* Replaces the schedule.  The rows of layer g are rows[group_ptr[g] ..
 * group_ptr[g+1]-1]; together the layers list every row exactly once.  The
 * row order is part of what the layered decoder computes; grouping is not
 * (rows in one layer share no column, so they commute).  Host arrays:
 * group_ptr int32 [G+1], rows int32 [mb].  QM_ERR_SCHEDULE_CONFLICT if two
 * rows of a layer share a column, QM_ERR_INVALID_ARG if not a partition.
 * Decoders created earlier keep the schedule they were created with. */
int qm_code_set_schedule(qm_code *code, int32_t G, const int32_t *group_ptr, const int32_t *rows);
/* Copies the schedule out: *G, group_ptr [G+1] and rows [mb] (host, caller-sized). */
int qm_code_get_schedule(const qm_code *code, int32_t *G, int32_t *group_ptr, int32_t *rows);

/* Creates a decoder for frames_per_code[c] frames of codes[c], c < ncodes.
 * All per-frame buffers of the decode calls are the concatenation over
 * codes (in this order) of frame-major blocks [F_c][n_c] (or [F_c][m_c]).
 * The codes must outlive the decoder. */
int qm_decoder_create(const qm_code *const *codes, int32_t ncodes, const int32_t *frames_per_code,
                      int32_t flags, qm_decoder **out);
int qm_decoder_destroy(qm_decoder *dec);

/* Device workspace: size it, allocate it (any allocator, 256-byte aligned),
 * bind it.  The decoder borrows it; the caller frees it after the last
 * queued decode has completed.  Binding copies the schedule descriptors to
 * the device (synchronously).  The size does not depend on the tuning. */
size_t qm_decoder_workspace_bytes(const qm_decoder *dec);
int qm_decoder_bind_workspace(qm_decoder *dec, void *device_ptr, size_t bytes);
int qm_decoder_set_tuning(qm_decoder *dec, const qm_tuning *tuning);
int qm_decoder_get_tuning(const qm_decoder *dec, qm_tuning *tuning);

/* Layered sum-product decode (Methods, steps 1-4) of every frame for exactly
 * `iters` full sweeps over the layers (no early termination).
 *   llr      device float [sum_c F_c * n_c]  channel LLRs 2R/sigma^2
 *   syndrome device uint8 [sum_c F_c * m_c]  s (H x = s)
 *   iters    >= 0; 0 returns the channel decisions
 *   hard     device uint8 [sum_c F_c * n_c]  out: c_n = [APP_n < 0]
 *   app      device float [sum_c F_c * n_c]  out: APP LLRs, or NULL
 *   flags    device uint8 [sum_c F_c]        out: 1 iff H c = s for the frame
 * Degree-1 variables are deferred (their single check makes q = LLR exact at
 * every layer); their APP is formed from the messages of the last sweep.
 * Codes created with 0 frames take no part.  A decoder without any frame
 * returns QM_OK at once (as does qm_decode_early); its buffers may be NULL. */
int qm_decode(qm_decoder *dec, const float *llr, const uint8_t *syndrome, int32_t iters,
              uint8_t *hard, float *app, uint8_t *flags, void *stream);

/* Allocation-free variant of qm_decode, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It decodes exactly as qm_decode (same
 * kernels, bit-identical outputs) but takes as the decoder's workspace a
 * static array of QM_NOALLOC_SCRATCH_BYTES that the library holds on every
 * device it runs on until the process ends; no workspace need be bound, and
 * a bound one is neither used nor changed.  The call allocates nothing: it
 * copies the decoder's descriptors (a few KB) into the array on `stream` and
 * launches on `stream` alone (no graph, tile groups, side streams or
 * profiling for this call; each gives bit-identical outputs).
 *   Limits: qm_decoder_workspace_bytes(dec) <= QM_NOALLOC_SCRATCH_BYTES, else
 *   QM_ERR_NO_WORKSPACE (for example 3 frames of a 10^6-bit rate-0.1 code,
 *   or thousands of frames of a 3200-bit code); decoders created with
 *   QM_EARLY_STOP or QM_FLOODING give QM_ERR_UNSUPPORTED.
 *   Every call on one device shares that device's array and overwrites it
 *   (each call initialises what it reads), so calls that overlap on one
 *   device, on any streams, race: the caller must order them.
 * Arguments as qm_decode. */
#define QM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int qm_decode_noalloc(qm_decoder *dec, const float *llr, const uint8_t *syndrome, int32_t iters,
                      uint8_t *hard, float *app, uint8_t *flags, void *stream);

/* Layered sum-product decode with early termination (Results, Table
 * tabearly): before the first sweep and after every sweep each frame's hard
 * decisions are tested against its syndrome, and a frame that passes stops
 * there.  A frame that stops after t sweeps gets exactly the outputs of a
 * qm_decode with iters = t.  Frames that stop free their tile slots: once
 * enough have stopped to empty a tile of frames, the frames still decoding
 * are moved to the leading tiles and later sweeps skip the empty ones.
 * The per-sweep test reads packed hard decisions (one bit per frame) that
 * the layer kernel writes as it updates each variable and check. 
 * Needs a decoder created with QM_EARLY_STOP (else QM_ERR_UNSUPPORTED).
 *   max_iters  >= 0: sweeps for frames that never pass
 *   iters_used device int32 [sum_c F_c] out: sweeps each frame ran (or NULL)
 *   other arguments as qm_decode.
 * The host polls the device every 2 sweeps (pinned memory, one poll late) and
 * stops enqueueing sweeps once no frame is left, so the call returns before
 * the decode has finished but may block on earlier sweeps; it is not
 * captured into a graph (QM_GRAPH does not apply).  With profiling on, the
 * layer launches of the first sweep are timed (every tile still decodes);
 * their layer_bytes add, per check with a degree-1 column, the LLR_d read and
 * the degree-1 APP written every sweep (2 x 4 bytes). */
int qm_decode_early(qm_decoder *dec, const float *llr, const uint8_t *syndrome, int32_t max_iters,
                    uint8_t *hard, float *app, uint8_t *flags, int32_t *iters_used, void *stream);

/* Times result-preserving tunings on the given inputs and keeps the fastest:
 * frames per tile {16, 32, 64} x frames per lane {1, 2} x block {128, 256}
 * on the layer kernels (lds_resident 0; each trial decoding min(iters, 8)
 * sweeps), then, on the best, per-row
 * launches, the other mixed-batch mode (streams per code or fused launches),
 * graph replay, the other stream_hint, (if a code fits) lds_resident 1,
 * (one code) 2 and 4 tile groups, (fused launches) the
 * other spread_codes and (streams per code) resident_cap 0, 8 and 12, each
 * decoding min(iters, 256) sweeps: a graph or extra
 * streams over a few sweeps do not predict the whole decode.  The schedule
 * (row order) is never changed, so every trial decodes to the same bits.
 * Trials decode into the caller's output buffers (same shapes as
 * qm_decode); the call synchronises the stream.  cache_path (may be NULL)
 * gets one JSON line appended per trial. */
int qm_autotune(qm_decoder *dec, const float *llr, const uint8_t *syndrome, int32_t iters,
                uint8_t *hard, float *app, uint8_t *flags, const char *cache_path, void *stream);

/* Live timing of the layer kernel (the decode's hot loop).
 * qm_decoder_set_profiling(dec, 1): every later qm_decode records one pair of
 * HIP events on its stream around each of up to 4 sweeps from the middle of
 * the decode (never the last sweep; with fused codes, around one sweep's
 * worth of fused launches).  No event sits between two layer launches, so
 * layer_ms / launches is the average launch duration including the launch
 * gaps.  Graph replay is bypassed while profiling.  qm_decoder_get_profile
 * waits for the recorded events, sums them into *out and, if reset, forgets
 * them.
 * layer_bytes counts the algorithmic HBM bytes of the timed launches: per
 * check and frame 4 (its degree-1 term) plus, per degree>=2 edge, the message
 * read and written (2 x 4 bytes; 2 x 2 with QM_MSG_FP16, 2 x 1 with QM_MSG_FP8) and the APP read
 * and written (2 x 4 bytes). */
typedef struct {
    int32_t launches;     /* layer launches inside the timed windows */
    int32_t sweeps;       /* timed windows */
    double layer_ms;      /* summed duration of the timed windows */
    double sweep_ms;      /* unused (0) */
    double layer_bytes;   /* algorithmic bytes of the timed layer launches */
    double checks;        /* check-frame updates in the timed launches */
    int32_t lds_launches; /* LDS-resident decodes timed (one launch each, every sweep) */
    double lds_ms;        /* their summed duration */
    double lds_bytes;     /* their algorithmic HBM bytes: per check and frame and sweep 4 (its
                             degree-1 term) plus, per degree>=2 edge, the message read and
                             written; plus each frame's degree>=2 APPs read and written once */
    int32_t et_narrowings; /* early-terminating decodes: times the frames still decoding were
                              moved into a narrower frame tile (counted whether or not profiling
                              is enabled) */
} qm_profile;

int qm_decoder_set_profiling(qm_decoder *dec, int32_t enable);
int qm_decoder_get_profile(qm_decoder *dec, qm_profile *out, int32_t reset);

/* ---- Learned decoder: normalized/offset min-sum (not in the paper) -------
 * The same layered sweep over the decoder's schedule, with the check update
 *   r_e = (-1)^{s ^ xor_{e'!=e}[q_e' < 0]} * alpha * max(min_{e'!=e}|q_e'| - beta, 0)
 * (ties of the minimum: the lowest block column wins; a check with a single
 * edge sees 30).  Weights are per (sweep t, base row i, target edge type):
 *   weights: device float [T][mb][2][2]; [t][i][0] = (alpha, beta) for a
 *   target edge in a column of degree >= 2, [t][i][1] for the degree-1 edge.
 * Degree-1 variables keep q = LLR (their single check); their message only
 * reaches APP_d = LLR_d + r_d.  The decoder must hold exactly one code with
 * float32 messages (QM_ERR_UNSUPPORTED otherwise).
 * Workspace: a second device buffer, sized for at most T sweeps; train = 1
 * adds the per-sweep records of q (T x messages) and two sets of adjoints
 * and gradient partial sums (qm_nms_train_grad runs two loss terms'
 * reverse sweeps at once). */
size_t qm_nms_workspace_bytes(const qm_decoder *dec, int32_t T, int32_t train);
int qm_nms_bind_workspace(qm_decoder *dec, void *device_ptr, size_t bytes, int32_t T, int32_t train);

/* Min-sum decode of every frame for up to T sweeps (T <= the bound T).
 * early_stop = 1: after every sweep the hard decisions are tested (H c = s)
 * and a frame that passes is frozen; iters_used[f] (device int32 [F], or
 * NULL) receives the sweeps it ran (0 if its channel decisions already
 * pass).  Outputs as for qm_decode. */
int qm_nms_decode(qm_decoder *dec, const float *weights, const float *llr, const uint8_t *syndrome, int32_t T,
                  int32_t early_stop, uint8_t *hard, float *app, uint8_t *flags, int32_t *iters_used, void *stream);

/* Training step core: T fixed min-sum sweeps from the channel LLRs, a loss
 * on the APPs against the true bits x, and its gradient with respect to the
 * weights by reverse sweeps over the q's each forward sweep recorded.
 * Loss term of sweep t: the mean over frames and all n bits of
 *   softplus(-(1 - 2x) APP_t)   (binary cross-entropy, P(bit = 1) = sigmoid(-APP)),
 * APP_t being the APPs after sweep t (degree-1 variables included).
 *   every_sweep = 0: loss = the term of the last sweep;
 *   every_sweep = 1: loss = the mean of the T terms.
 *   window in [1, T] (0 = T): the gradient of each term runs back through at
 *   most `window` sweeps, the term's own and the ones before it, holding the
 *   state before the earliest of them fixed; the weights of sweep u then
 *   receive the exact derivatives of the terms t = u .. u + window - 1.
 *   every_sweep = 0 with window = T is the exact gradient of the final-sweep
 *   loss (qm_nms_loss_grad).
 * Over many sweeps the reverse-sweep adjoints grow geometrically (about 20x
 * per sweep on the workload codes); each is bounded at 1e30, so nothing
 * becomes inf or NaN, and `clamped` (device int32, or NULL) receives how
 * many adjoint components reached the bound: 0 means the gradient is exact.
 * With every_sweep = 1 consecutive terms' reverse sweeps run on two streams
 * of the decoder, forked from and joined back to `stream` inside the call
 * (the terms alternate between two sets of adjoints and partial sums), beside
 * the forward sweeps.  Gradient sums over workgroups and sets are reduced in
 * a fixed order (run-to-run identical).
 *   x: device uint8 [F][n]; loss: device float scalar; grad: device float,
 *   same layout as weights (first T sweeps).  Needs a train workspace bound
 *   for at least T sweeps. */
int qm_nms_train_grad(qm_decoder *dec, const float *weights, const float *llr, const uint8_t *syndrome,
                      const uint8_t *x, int32_t T, int32_t every_sweep, int32_t window, float *loss, float *grad,
                      int32_t *clamped, void *stream);

/* qm_nms_train_grad with every_sweep = 0, window = T, clamped = NULL: the
 * mean binary cross-entropy of the final APPs and its exact gradient
 * (wherever no adjoint reaches the bound). */
int qm_nms_loss_grad(qm_decoder *dec, const float *weights, const float *llr, const uint8_t *syndrome,
                     const uint8_t *x, int32_t T, float *loss, float *grad, void *stream);

/* Synthetic frames of code `code_index` of the decoder (its workspace must
 * be bound): for frame f (global index first_frame + f) x is uniform random
 * bits, y = 1 - 2x + N(0, 1/snr), llr = 2 snr y (Methods, step 1) and
 * s = H x.  Random numbers are Philox4x32-10 (Salmon et al., SC 2011) with
 * key = seed and counter (bit pair p, frame lo, frame hi, 0): bits 2p, 2p+1
 * are the top bits of words 2 and 3; words 0 and 1 give two normals by
 * Box-Muller (u = (word + 1/2) 2^-32).  Outputs device [F][n] x and llr,
 * [F][m] syndrome. */
int qm_generate_frames(qm_decoder *dec, int32_t code_index, uint64_t seed, uint64_t first_frame, float snr,
                       int32_t F, uint8_t *x, float *llr, uint8_t *syndrome, void *stream);

/* Adam (Kingma & Ba) on device arrays of `count` floats, step >= 1:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * w -= lr * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps),
 * with a non-finite g taken as 0 and |g| capped at 1e15 (so g^2 is finite). */
int qm_adam_step(float *w, const float *g, float *m, float *v, int32_t count, float lr, float b1, float b2,
                 float eps, int32_t step, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* QCMET_H */
