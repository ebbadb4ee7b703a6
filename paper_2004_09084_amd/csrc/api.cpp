// Host runtime and C ABI of libqcmet (declared in include/qcmet.h).
//
// Code ingestion (column classes, message slots, default greedy layer merge),
// decoder workspace layout, schedule descriptors, the launch sequence of a
// decode and its hipGraph replay.  No device work happens outside qm_decode,
// qm_decoder_bind_workspace and qm_autotune.
#include "../../include/qcmet.h"
#include "qcmet_internal.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define QM_HIP(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) return fail(QM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

inline bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }
inline int log2i(int x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

}  // namespace

struct qm_code {
    int32_t mb = 0, nb = 0, Z = 0;
    std::vector<int32_t> sh;       // [mb*nb]
    std::vector<int32_t> col_deg;  // [nb]
    std::vector<int32_t> ent;      // [mb*nb]: message slot of a degree>=2 entry, else -1
    int32_t nent1 = 0, max_d = 0, ntype1 = 0, ndeg1 = 0;
    int64_t edges = 0;
    std::vector<int32_t> gptr, rows;  // schedule
};

namespace {

// Greedy merge of rows with disjoint block columns (Results, Eq. (m)-(m2)):
// open a layer with the first unassigned row, add each later unassigned row
// that shares no column with the layer so far, repeat.
void greedy_schedule(const qm_code &c, std::vector<int32_t> &gptr, std::vector<int32_t> &rows) {
    std::vector<char> used(c.mb, 0);
    gptr.clear();
    rows.clear();
    for (int first = 0; first < c.mb; ++first) {
        if (used[first]) continue;
        gptr.push_back((int32_t)rows.size());
        std::vector<char> taken(c.nb, 0);
        for (int cand = first; cand < c.mb; ++cand) {
            if (used[cand]) continue;
            bool clash = false;
            for (int j = 0; j < c.nb && !clash; ++j) clash = c.sh[cand * c.nb + j] >= 0 && taken[j];
            if (clash) continue;
            for (int j = 0; j < c.nb; ++j)
                if (c.sh[cand * c.nb + j] >= 0) taken[j] = 1;
            used[cand] = 1;
            rows.push_back(cand);
        }
    }
    gptr.push_back((int32_t)rows.size());
}

int check_schedule(const qm_code &c, int32_t G, const int32_t *gptr, const int32_t *rows) {
    if (G < 1 || gptr[0] != 0 || gptr[G] != c.mb)
        return fail(QM_ERR_INVALID_ARG, "schedule: group_ptr must start at 0 and end at mb");
    std::vector<char> seen(c.mb, 0);
    for (int g = 0; g < G; ++g) {
        if (gptr[g + 1] <= gptr[g]) return fail(QM_ERR_INVALID_ARG, "schedule: empty or decreasing layer");
        std::vector<char> taken(c.nb, 0);
        for (int p = gptr[g]; p < gptr[g + 1]; ++p) {
            const int r = rows[p];
            if (r < 0 || r >= c.mb || seen[r]) return fail(QM_ERR_INVALID_ARG, "schedule: rows are not a permutation");
            seen[r] = 1;
            for (int j = 0; j < c.nb; ++j) {
                if (c.sh[r * c.nb + j] < 0) continue;
                if (taken[j])
                    return fail(QM_ERR_SCHEDULE_CONFLICT, "schedule: rows of layer " + std::to_string(g) +
                                                               " share block column " + std::to_string(j));
                taken[j] = 1;
            }
        }
    }
    return QM_OK;
}

RowDesc make_desc(const qm_code &c, int i) {
    RowDesc d;
    std::memset(&d, 0, sizeof(d));
    d.row = i;
    d.d1col = -1;
    for (int j = 0; j < c.nb; ++j) {
        const int a = c.sh[i * c.nb + j];
        if (a < 0) continue;
        if (c.col_deg[j] == 1) {
            d.d1col = j;
            d.d1shift = a;
            d.d1pos = d.d;  // degree>=2 entries before it
        } else {
            d.col[d.d] = j;
            d.shift[d.d] = a;
            d.ent[d.d] = c.ent[i * c.nb + j];
            int rank = 0;
            for (int jj = 0; jj < j; ++jj) rank += c.col_deg[jj] >= 2 ? 1 : 0;
            d.lcol[d.d] = rank;
            d.d++;
        }
    }
    return d;
}

struct Slot {
    const qm_code *code = nullptr;
    int32_t F = 0, Fpad = 0;
    int64_t n = 0, m = 0;
    size_t oA = 0, oR = 0, oK = 0, oS = 0, oFail = 0, oRows = 0;
    // early termination (decoders created with QM_EARLY_STOP)
    size_t oAd = 0, oAct = 0, oTmask = 0, oMap = 0, oPerm = 0, oIt = 0, oCtl = 0, oEmit = 0, oPA = 0, oPd = 0, oPS = 0;
    std::vector<RowDesc> hrows;  // schedule order
    std::vector<int32_t> d1row;  // block column -> schedule index of the row whose degree-1 column it is, or -1
    size_t oD1Row = 0;           // its device copy (early termination)
    std::vector<int32_t> gptr;
    std::vector<int32_t> cols1;  // degree>=2 block columns (LDS order)
    size_t oGptr = 0, oCols1 = 0;
    std::vector<ColDesc> hcols;  // flooding: column descriptors of cols1
    size_t oColD = 0, oLam = 0;
    int maxd_t = 4;
};

}  // namespace

struct qm_decoder {
    std::vector<Slot> slots;
    int32_t flags = 0;
    qm_tuning tun{};
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool bound = false;
    size_t oErr = 0, total = 0;
    // one cached graph of the whole decode
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    const void *gkey[7] = {};
    int32_t giters = -1;
    hipStream_t cap = nullptr;  // private stream the graph is captured on
    // live profiling of the layer kernel
    int32_t profiling = 0;
    std::vector<hipEvent_t> ev_pool;     // created lazily, reused after a reset
    size_t ev_used = 0;
    struct Pending { size_t a, b; double bytes, checks; int launches; };  // one timed window of layer launches
    std::vector<Pending> pending;
    // learned-decoder (min-sum) workspace
    char *nws = nullptr;
    size_t nws_bytes = 0;
    int32_t nT = 0, ntrain = 0;
    size_t oAd = 0, oAct = 0, oTmask = 0, oIt = 0, oCols = 0, oLossP = 0, oLoss = 0, oX = 0, ogA = 0, ogAd = 0,
           ogR = 0, oQ = 0, oPart = 0, oClamp = 0, nTotal = 0;
    size_t adjSet = 0, partSet = 0;  // bytes of one adjoint set (gA, gAd, gR) and of one partial-sum set
    // training: events of the loss terms' reverse sweeps (one per term,
    // cycled) and of each term's forward part, for the reverse streams
    std::vector<hipEvent_t> term_done;
    hipEvent_t term_fwd = nullptr;
    std::vector<int32_t> acols;  // columns whose APP lives in A (degree != 1)
    int64_t lds_limit = 0;      // LDS bytes one workgroup may use (queried at bind)
    int64_t lds_per_cu = 0;     // LDS bytes of one compute unit (queried at bind)
    int32_t ncu = 0;            // compute units of the device (queried at bind)
    // LDS-resident codes of a mixed decode run on a side stream, forked from
    // and joined back to the decode stream with events
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // tile groups of a layered decode: one stream per group after the first
    std::vector<hipStream_t> gstreams;
    std::vector<hipEvent_t> gjoin;
    hipEvent_t gfork = nullptr;
    struct LdsPending { size_t a, b; double bytes; };
    std::vector<LdsPending> lds_pending;
    // early termination: host polls of the frames still decoding
    int32_t *h_poll = nullptr;   // pinned, 2 copies of the control words
    int32_t et_narrowings = 0;   // early termination: narrowing steps since the last profile reset
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
};

namespace {

// message storage kind and bytes per message
int msg_kind(const qm_decoder &d) {
    return (d.flags & QM_MSG_FP16) ? QM_MSGK_F16 : (d.flags & QM_MSG_FP8) ? QM_MSGK_F8 : QM_MSGK_F32;
}
size_t msg_bytes(const qm_decoder &d) {
    const int k = msg_kind(d);
    return k == QM_MSGK_F16 ? 2 : k == QM_MSGK_F8 ? 1 : 4;
}

// decoded by the LDS-resident kernel (one frame per tile)?  Tuning
// lds_resident 1: whenever the code fits; 2: when it fits and has at least
// one frame per compute unit (with fewer, its one workgroup per frame leaves
// compute units idle and the layer kernels are faster).  Flooding and
// early-terminating decoders, and decoders with a min-sum workspace bound
// (whose kernels take the same frame tiles), always use the layer kernels.
bool lds_slot(const qm_decoder &d, const Slot &s) {
    const bool want = d.tun.lds_resident == 1 || (d.tun.lds_resident == 2 && d.ncu > 0 && s.F >= d.ncu);
    return want && !(d.flags & (QM_FLOODING | QM_EARLY_STOP)) && !d.nws && s.F > 0 && s.code->max_d <= 8 && d.lds_limit > 0 &&
           (int64_t)qm_lds_bytes((int)s.cols1.size(), s.code->Z) <= d.lds_limit;
}

int slot_ft(const qm_decoder &d, const Slot &s) {
    if (lds_slot(d, s)) return 1;
    int ft = d.tun.frames_per_tile;
    if (ft > s.Fpad) ft = s.Fpad;
    return ft < 1 ? 1 : ft;
}

TileGeom geom(const qm_decoder &d, const Slot &s) {
    TileGeom g;
    const int ft = slot_ft(d, s);
    g.Z = s.code->Z;
    g.ft_log2 = log2i(ft);
    g.ntiles = s.Fpad / ft;
    g.n = s.n;
    g.m = s.m;
    g.nent1 = s.code->nent1;
    return g;
}

void layout(qm_decoder &d) {
    size_t off = 0;
    const size_t msg = msg_bytes(d);
    for (Slot &s : d.slots) {
        const size_t fp = (size_t)s.Fpad;
        s.oA = off; off = align_up(off + fp * (size_t)s.n * 4);
        s.oR = off; off = align_up(off + fp * (size_t)s.code->nent1 * (size_t)s.code->Z * msg);
        s.oK = off; off = align_up(off + fp * (size_t)s.m * 4);
        s.oS = off; off = align_up(off + fp * (size_t)s.m);
        s.oFail = off; off = align_up(off + fp * 4);
        s.oRows = off; off = align_up(off + s.hrows.size() * sizeof(RowDesc));
        s.oGptr = off; off = align_up(off + s.gptr.size() * 4);
        s.oCols1 = off; off = align_up(off + std::max<size_t>(1, s.cols1.size()) * 4);
        if (d.flags & QM_FLOODING) {
            s.oColD = off; off = align_up(off + std::max<size_t>(1, s.hcols.size()) * sizeof(ColDesc));
            s.oLam = off; off = align_up(off + fp * s.cols1.size() * (size_t)s.code->Z * 4);
        }
        if (d.flags & QM_EARLY_STOP) {
            s.oAd = off; off = align_up(off + fp * (size_t)s.m * 4);
            s.oAct = off; off = align_up(off + fp * 4);
            s.oTmask = off; off = align_up(off + fp * 8);  // one word per tile (at most Fpad tiles)
            s.oMap = off; off = align_up(off + fp * 4);
            s.oPerm = off; off = align_up(off + fp * 4);
            s.oIt = off; off = align_up(off + fp * 4);
            s.oCtl = off; off = align_up(off + QM_ET_CTL_WORDS * 4);
            s.oEmit = off; off = align_up(off + fp * 4);
            // packed hard decisions: max(FT, 8) bits per tile and node, at
            // most one byte per frame and node (FT = 1), whatever the tuning
            s.oPA = off; off = align_up(off + fp * (size_t)s.n);
            s.oPd = off; off = align_up(off + fp * (size_t)s.m);
            s.oPS = off; off = align_up(off + fp * (size_t)s.m);
            s.oD1Row = off; off = align_up(off + s.d1row.size() * 4);
        }
    }
    d.oErr = off;
    off = align_up(off + 4);
    d.total = off;
}

int take_event(qm_decoder &d, hipEvent_t *ev, size_t *index) {
    if (d.ev_used == d.ev_pool.size()) {
        hipEvent_t e;
        QM_HIP(hipEventCreate(&e));
        d.ev_pool.push_back(e);
    }
    *index = d.ev_used;
    *ev = d.ev_pool[d.ev_used++];
    return QM_OK;
}

// algorithmic bytes / check updates of one layer launch over `rows`
// (early: the early-terminating form, which also reads LLR_d and writes the
// degree-1 APP of every check that has a degree-1 column, every sweep)
void layer_work(const Slot &s, const RowDesc *hrows, int nrows, size_t msg, double *bytes, double *checks,
                bool early = false) {
    // per check and frame: APP read + write and message read + write per
    // degree>=2 edge, plus K read (4); early termination reads the degree-1
    // LLR instead of K (4) and writes the degree-1 APP (4), plus its packed
    // syndrome bits (one bit per frame)
    const double per_edge = 8.0 + 2.0 * (double)msg;
    double b = 0.0;
    for (int r = 0; r < nrows; ++r) b += per_edge * hrows[r].d + (early ? 8.125 : 4.0);
    const double fz = (double)s.F * s.code->Z;
    *bytes = b * fz;
    *checks = (double)nrows * fz;
}

void drop_graph(qm_decoder &d) {
    if (d.gexec) (void)hipGraphExecDestroy(d.gexec);
    if (d.graph) (void)hipGraphDestroy(d.graph);
    d.gexec = nullptr;
    d.graph = nullptr;
    d.giters = -1;
}

struct SlotBufs {
    float *A;
    void *R;
    float *K;
    uint8_t *S;
    uint32_t *fail;
    const RowDesc *rows;
};

SlotBufs slot_bufs(const qm_decoder &d, const Slot &s) {
    SlotBufs b;
    b.A = reinterpret_cast<float *>(d.ws + s.oA);
    b.R = d.ws + s.oR;
    b.K = reinterpret_cast<float *>(d.ws + s.oK);
    b.S = reinterpret_cast<uint8_t *>(d.ws + s.oS);
    b.fail = reinterpret_cast<uint32_t *>(d.ws + s.oFail);
    b.rows = reinterpret_cast<const RowDesc *>(d.ws + s.oRows);
    return b;
}

LayerArgs layer_args(const qm_decoder &d, const Slot &s) {
    const TileGeom g = geom(d, s);
    const SlotBufs b = slot_bufs(d, s);
    LayerArgs la;
    std::memset(&la, 0, sizeof(la));
    la.A = b.A;
    la.R = b.R;
    la.K = b.K;
    la.Z = s.code->Z;
    la.ft_log2 = g.ft_log2;
    la.ntiles = g.ntiles;
    la.fpl = std::min(d.tun.frames_per_lane, 1 << g.ft_log2);
    const int lanes = (s.code->Z << g.ft_log2) / la.fpl;
    la.chunks = (lanes + d.tun.block - 1) / d.tun.block;
    la.strideA = (int64_t)s.n << g.ft_log2;
    la.strideR = ((int64_t)s.code->nent1 * s.code->Z) << g.ft_log2;
    la.strideK = (int64_t)s.m << g.ft_log2;
    return la;
}

// record a pair of events around a launch (profiling)
struct ProfScope {
    qm_decoder &d;
    hipStream_t st;
    bool on;
    size_t i0 = 0;
    ProfScope(qm_decoder &d_, hipStream_t st_, bool on_) : d(d_), st(st_), on(on_) {}
    int begin() {
        if (!on) return QM_OK;
        hipEvent_t e;
        int rc = take_event(d, &e, &i0);
        if (rc != QM_OK) return rc;
        QM_HIP(hipEventRecord(e, st));
        return QM_OK;
    }
    int end(double bytes, double checks, int launches) {
        if (!on) return QM_OK;
        hipEvent_t e;
        size_t i1;
        int rc = take_event(d, &e, &i1);
        if (rc != QM_OK) return rc;
        QM_HIP(hipEventRecord(e, st));
        d.pending.push_back(qm_decoder::Pending{i0, i1, bytes, checks, launches});
        return QM_OK;
    }
};

// early: an early-terminating decode, whose layer kernel forms K itself
int enqueue_init(qm_decoder &d, const float *llr, const uint8_t *syn, hipStream_t st) {
    size_t on = 0, om = 0;
    const size_t msg = msg_bytes(d);
    for (Slot &s : d.slots) {
        if (s.F == 0) continue;
        const qm_code &c = *s.code;
        const TileGeom g = geom(d, s);
        const SlotBufs b = slot_bufs(d, s);
        QM_HIP(qm_launch_to_tiles_f32(llr + on, b.A, s.F, s.n, g.ft_log2, g.ntiles, st));
        QM_HIP(qm_launch_to_tiles_u8(syn + om, b.S, s.F, s.m, g.ft_log2, g.ntiles, st));
        QM_HIP(qm_launch_kappa(b.A, b.S, b.K, b.rows, c.mb, g, st));
        const size_t rbytes = align_up((size_t)s.Fpad * c.nent1 * c.Z * msg);
        QM_HIP(qm_launch_fill_u32(reinterpret_cast<uint32_t *>(b.R), 0u, rbytes / 4, st));
        QM_HIP(qm_launch_fill_u32(b.fail, 0u, (size_t)s.Fpad, st));
        on += (size_t)s.F * s.n;
        om += (size_t)s.F * s.m;
    }
    return QM_OK;
}

int enqueue_finalize(qm_decoder &d, uint8_t *hard, float *app, uint8_t *flags, hipStream_t st) {
    size_t on = 0, of = 0;
    for (Slot &s : d.slots) {
        if (s.F == 0) continue;
        const TileGeom g = geom(d, s);
        const SlotBufs b = slot_bufs(d, s);
        QM_HIP(qm_launch_syndrome(b.A, nullptr, b.S, b.rows, s.code->mb, b.fail, g, st));
        QM_HIP(qm_launch_finalize(b.A, b.fail, app ? app + on : nullptr, hard + on, flags + of, s.F, g, st));
        on += (size_t)s.F * s.n;
        of += (size_t)s.F;
    }
    return QM_OK;
}

// Tile groups (tuning tile_groups) usable over nt frame tiles: the largest
// count not above the tuning value that divides nt.
int64_t total_frames(const qm_decoder &d) {
    int64_t F = 0;
    for (const Slot &s : d.slots) F += s.F;
    return F;
}

int tile_groups(const qm_decoder &d, int nt) {
    int g = std::max(1, std::min<int>(d.tun.tile_groups, nt));
    while (g > 1 && nt % g) --g;
    return g;
}

// Frame tiles decoded together by a layered decode of one code (tuning
// frames_per_batch): all of them unless their per-frame state (APPs,
// messages, K, syndrome bits) exceeds kBatchBytes, then batches of the
// largest power-of-two tile count within it (a multiple of the 8 XCDs keeps
// each tile's workgroups on one XCD); an explicit frames_per_batch is
// rounded down to whole tiles.
constexpr size_t kBatchBytes = (size_t)12 << 30;

int batch_tiles(const qm_decoder &d, const Slot &s) {
    const TileGeom g = geom(d, s);
    const int ft = 1 << g.ft_log2;
    if (d.tun.frames_per_batch > 0)
        return (int)std::max<int64_t>(1, std::min<int64_t>(g.ntiles, d.tun.frames_per_batch / ft));
    const size_t per_frame = (size_t)s.n * 4 + (size_t)s.code->nent1 * s.code->Z * msg_bytes(d) + (size_t)s.m * 5;
    if ((size_t)g.ntiles * ft * per_frame <= kBatchBytes) return g.ntiles;
    int64_t bt = 1;
    while ((size_t)(bt * 2) * ft * per_frame <= kBatchBytes) bt *= 2;
    return (int)std::min<int64_t>(g.ntiles, bt);
}

int ensure_group_streams(qm_decoder &d, int groups) {
    while ((int)d.gstreams.size() < groups - 1) {
        hipStream_t st = nullptr;
        QM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        d.gstreams.push_back(st);
        hipEvent_t e = nullptr;
        QM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        d.gjoin.push_back(e);
    }
    if (!d.gfork) QM_HIP(hipEventCreateWithFlags(&d.gfork, hipEventDisableTiming));
    return QM_OK;
}

int enqueue_sweeps_tiles(qm_decoder &d, Slot &s, int32_t iters, hipStream_t st, int t0, int nt, bool profile);

// Sweeps of one code, one launch per layer (or per row with merge = 0), over
// its frame tiles in batches (batch_tiles): each batch runs every sweep before
// the next starts.
int enqueue_sweeps_slot(qm_decoder &d, Slot &s, int32_t iters, hipStream_t st) {
    const int ntiles = geom(d, s).ntiles;
    const int bt = batch_tiles(d, s);
    for (int t0 = 0; t0 < ntiles; t0 += bt) {
        const int rc = enqueue_sweeps_tiles(d, s, iters, st, t0, std::min(bt, ntiles - t0), t0 == 0);
        if (rc != QM_OK) return rc;
    }
    return QM_OK;
}

// The sweeps of tiles [t0, t0 + nt) of one code; profile: time the middle
// sweeps (the first batch of a batched decode). With tile groups, each group
// of consecutive tiles runs its own layer sequence on its own stream (frames
// never depend on other frames), so one group's launch can fill the
// ramp-down of another's.
int enqueue_sweeps_tiles(qm_decoder &d, Slot &s, int32_t iters, hipStream_t st, int t0, int nt, bool profile) {
    const int msgk = msg_kind(d);
    const size_t msg = msg_bytes(d);
    const RowDesc *rows = slot_bufs(d, s).rows;
    LayerArgs la = layer_args(d, s);
    la.A += (int64_t)t0 * la.strideA;
    la.R = static_cast<char *>(la.R) + (int64_t)t0 * la.strideR * (int64_t)msg;
    la.K += (int64_t)t0 * la.strideK;
    la.ntiles = nt;
    // share of the code's frames in these tiles (padding frames excluded)
    const int ft = 1 << la.ft_log2;
    const double share = (double)std::max(0, std::min(nt * ft, s.F - t0 * ft)) / (double)std::max(s.F, 1);
    const int G = (int)s.gptr.size() - 1;
    const int ng = tile_groups(d, nt);
    std::vector<LayerArgs> lg(ng, la);
    std::vector<hipStream_t> gs(ng, st);
    if (ng > 1) {
        if ((int)d.gstreams.size() < ng - 1 || !d.gfork) return fail(QM_ERR_STATE, "tile-group streams missing");
        const int tpg = la.ntiles / ng;
        for (int g = 0; g < ng; ++g) {
            lg[g].A = la.A + (int64_t)g * tpg * la.strideA;
            lg[g].R = static_cast<char *>(la.R) + (int64_t)g * tpg * la.strideR * (int64_t)msg;
            lg[g].K = la.K + (int64_t)g * tpg * la.strideK;
            lg[g].ntiles = tpg;
            if (g > 0) gs[g] = d.gstreams[g - 1];
        }
        QM_HIP(hipEventRecord(d.gfork, st));
        for (int g = 1; g < ng; ++g) QM_HIP(hipStreamWaitEvent(gs[g], d.gfork, 0));
    }
    // profiled: up to 4 sweeps from the middle of the decode, never the last
    // (which also forms the degree-1 APPs); one event pair per sweep, so no
    // event sits between two layer launches
    const int t0p = (iters - 1) / 2, t1p = (d.profiling && profile) ? std::min(t0p + 4, iters - 1) : -1;
    for (int t = 0; t < iters; ++t) {
        const bool prof = t >= t0p && t < t1p;
        // with tile groups the window is timed on the decode stream, where
        // group 0 runs; the groups proceed concurrently with the same work
        ProfScope sweep(d, st, prof);
        int rc = sweep.begin();
        if (rc != QM_OK) return rc;
        double bytes = 0.0, checks = 0.0;
        int launches = 0;
        for (int gi = 0; gi < G; ++gi) {
            const int p_lo = s.gptr[gi], p_hi = s.gptr[gi + 1];
            const int step = d.tun.merge ? (p_hi - p_lo) : 1;
            for (int p = p_lo; p < p_hi; p += step) {
                for (int g = 0; g < ng; ++g) {
                    lg[g].last = (t == iters - 1) ? 1 : 0;
                    lg[g].rows = rows + p;
                    lg[g].nrows = step;
                    QM_HIP(qm_launch_layer(lg[g], msgk, s.maxd_t, la.fpl, d.tun.block, d.tun.stream_hint, gs[g]));
                }
                double b, ch;
                layer_work(s, s.hrows.data() + p, step, msg, &b, &ch);
                bytes += b * share;
                checks += ch * share;
                ++launches;
            }
        }
        if ((rc = sweep.end(bytes, checks, launches)) != QM_OK) return rc;
    }
    for (int g = 1; g < ng; ++g) {
        QM_HIP(hipEventRecord(d.gjoin[g - 1], gs[g]));
        QM_HIP(hipStreamWaitEvent(st, d.gjoin[g - 1], 0));
    }
    return QM_OK;
}

// Sweeps of every code in fused launches: step k runs layer (k mod G_c) of
// iteration k / G_c of each code c that still has sweeps left.
int enqueue_sweeps_fused(qm_decoder &d, int32_t iters, hipStream_t st) {
    const int msgk = msg_kind(d);
    const size_t msg = msg_bytes(d);
    std::vector<Slot *> act;
    for (Slot &s : d.slots)
        if (s.F > 0 && !lds_slot(d, s)) act.push_back(&s);
    // the code with the longest chain of layers is placed first in every
    // launch, so its (latency-bound) blocks are dispatched first and overlap
    // with the other codes' blocks instead of trailing them
    std::stable_sort(act.begin(), act.end(),
                     [](const Slot *a, const Slot *b) { return a->gptr.size() > b->gptr.size(); });
    const int nc = (int)act.size();
    std::vector<LayerArgs> base(nc);
    std::vector<int> G(nc);
    int64_t steps = 0;
    int maxd = 2;
    for (int c = 0; c < nc; ++c) {
        base[c] = layer_args(d, *act[c]);
        G[c] = (int)act[c]->gptr.size() - 1;
        steps = std::max<int64_t>(steps, (int64_t)iters * G[c]);
        maxd = std::max(maxd, act[c]->maxd_t);
    }
    // one lane width for the whole launch: no wider than any code's tile
    int fpl = d.tun.frames_per_lane;
    for (int c = 0; c < nc; ++c) fpl = std::min(fpl, 1 << base[c].ft_log2);
    for (int c = 0; c < nc; ++c) {
        base[c].fpl = fpl;
        const int lanes = (base[c].Z << base[c].ft_log2) / fpl;
        base[c].chunks = (lanes + d.tun.block - 1) / d.tun.block;
    }
    // profiled: the steps of one sweep of the code with the most layers,
    // from the middle of the decode (never its last sweep)
    int gmax = 1;
    for (int c = 0; c < nc; ++c) gmax = std::max(gmax, G[c]);
    const int64_t kprof = (d.profiling && steps >= 2 * gmax) ? (steps / 2 / gmax) * gmax - gmax : -1;
    ProfScope window(d, st, kprof >= 0);
    double wbytes = 0.0, wchecks = 0.0;
    for (int64_t k = 0; k < steps; ++k) {
        const bool in_window = kprof >= 0 && k >= kprof && k < kprof + gmax;
        if (k == kprof) {
            const int rc = window.begin();
            if (rc != QM_OK) return rc;
        }
        MultiLayerArgs m;
        std::memset(&m, 0, sizeof(m));
        m.ncodes = nc;
        double bytes = 0.0, checks = 0.0;
        int32_t off = 0;
        for (int c = 0; c < nc; ++c) {
            m.block_off[c] = off;
            LayerArgs la = base[c];
            // code c runs its layer number j (of N = iters * G[c]) at this
            // step: spread, at the steps where floor(k N / steps) advances
            // (every step for the longest code); else at step j itself
            const int64_t N = (int64_t)iters * G[c];
            int64_t j = -1;
            if (d.tun.spread_codes) {
                const int64_t j0 = k * N / steps, j1 = (k + 1) * N / steps;
                if (j1 > j0) j = j0;
            } else if (k < N) {
                j = k;
            }
            if (j >= 0) {
                const int t = (int)(j / G[c]), gi = (int)(j % G[c]);
                const Slot &s = *act[c];
                la.last = (t == iters - 1) ? 1 : 0;
                la.rows = slot_bufs(d, s).rows + s.gptr[gi];
                la.nrows = s.gptr[gi + 1] - s.gptr[gi];
                off += la.ntiles * la.nrows * la.chunks;
                double b, ch;
                layer_work(s, s.hrows.data() + s.gptr[gi], la.nrows, msg, &b, &ch);
                bytes += b;
                checks += ch;
            } else {
                la.nrows = 0;
            }
            m.code[c] = la;
        }
        m.block_off[nc] = off;
        QM_HIP(qm_launch_layer_multi(m, msgk, maxd, fpl, d.tun.block, d.tun.stream_hint, st));
        if (in_window) {
            wbytes += bytes;
            wchecks += checks;
        }
        if (kprof >= 0 && k == kprof + gmax - 1) {
            const int rc = window.end(wbytes, wchecks, gmax);
            if (rc != QM_OK) return rc;
        }
    }
    return QM_OK;
}

// Flooding schedule: per iteration, every check from the previous
// iteration's APPs (one launch over all rows), then every degree>=2
// variable: APP = LLR + its messages in ascending row order.
int enqueue_flood_slot(qm_decoder &d, Slot &s, int32_t iters, hipStream_t st) {
    const TileGeom g = geom(d, s);
    const SlotBufs b = slot_bufs(d, s);
    const int msgk = msg_kind(d);
    const size_t msg = msg_bytes(d);
    float *Lam = reinterpret_cast<float *>(d.ws + s.oLam);
    const ColDesc *cols = reinterpret_cast<const ColDesc *>(d.ws + s.oColD);
    const int ncols1 = (int)s.cols1.size();
    QM_HIP(qm_launch_copy_cols(b.A, Lam, reinterpret_cast<const int32_t *>(d.ws + s.oCols1), ncols1, g, st));
    LayerArgs la = layer_args(d, s);
    la.rows = b.rows;
    la.nrows = s.code->mb;
    // algorithmic bytes of one iteration: checks read APP and message and
    // write the message per edge, read K per check; variables read the
    // message per edge, read the LLR and write the APP per variable
    double it_bytes = 0.0, checks = 0.0;
    for (const RowDesc &r : s.hrows) it_bytes += (4.0 + 2.0 * msg) * r.d + 4.0;
    for (const ColDesc &cd : s.hcols) it_bytes += (double)msg * cd.deg + 8.0;
    it_bytes *= (double)s.F * s.code->Z;
    checks = (double)s.code->mb * s.F * s.code->Z;
    const int t0p = (iters - 1) / 2, t1p = d.profiling ? std::min(t0p + 4, iters - 1) : -1;
    for (int t = 0; t < iters; ++t) {
        la.last = (t == iters - 1) ? 1 : 0;
        ProfScope it(d, st, t >= t0p && t < t1p);
        int rc = it.begin();
        if (rc != QM_OK) return rc;
        QM_HIP(qm_launch_layer_flood(la, msgk, s.maxd_t, la.fpl, d.tun.block, d.tun.stream_hint, st));
        QM_HIP(qm_launch_flood_vars(b.A, Lam, b.R, cols, ncols1, msgk, la.fpl, d.tun.block, g, st));
        if ((rc = it.end(it_bytes, checks, 1)) != QM_OK) return rc;  // one timed unit = one iteration
    }
    return QM_OK;
}

// All sweeps of one code in one launch of the LDS-resident kernel.
int ensure_side_stream(qm_decoder &d) {
    if (!d.side) QM_HIP(hipStreamCreateWithFlags(&d.side, hipStreamNonBlocking));
    if (!d.ev_fork) QM_HIP(hipEventCreateWithFlags(&d.ev_fork, hipEventDisableTiming));
    if (!d.ev_join) QM_HIP(hipEventCreateWithFlags(&d.ev_join, hipEventDisableTiming));
    return QM_OK;
}

int enqueue_sweeps_lds(qm_decoder &d, Slot &s, int32_t iters, hipStream_t st) {
    const SlotBufs b = slot_bufs(d, s);
    LdsArgs a;
    std::memset(&a, 0, sizeof(a));
    a.A = b.A;
    a.R = b.R;
    a.K = b.K;
    a.rows = b.rows;
    a.gptr = reinterpret_cast<const int32_t *>(d.ws + s.oGptr);
    a.cols1 = reinterpret_cast<const int32_t *>(d.ws + s.oCols1);
    a.G = (int)s.gptr.size() - 1;
    a.Z = s.code->Z;
    a.T = iters;
    a.ncols1 = (int)s.cols1.size();
    a.n = s.n;
    a.m = s.m;
    a.nr = (int64_t)s.code->nent1 * s.code->Z;
    const bool prof = d.profiling && iters > 0;
    size_t i0 = 0, i1 = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof) {
        int rc = take_event(d, &e0, &i0);
        if (rc != QM_OK) return rc;
        QM_HIP(hipEventRecord(e0, st));
    }
    QM_HIP(qm_launch_sweeps_lds(a, s.F, msg_kind(d), s.maxd_t, st));
    if (prof) {
        int rc = take_event(d, &e1, &i1);
        if (rc != QM_OK) return rc;
        QM_HIP(hipEventRecord(e1, st));
        // per sweep: messages read + written and K per check; once: the APPs in and out
        double per_sweep = 0.0;
        const double msg = (double)msg_bytes(d);
        for (const RowDesc &r : s.hrows) per_sweep += 2.0 * msg * r.d + 4.0;
        const double bytes = (double)s.F * s.code->Z * per_sweep * iters + 8.0 * (double)s.F * s.cols1.size() * s.code->Z;
        d.lds_pending.push_back(qm_decoder::LdsPending{i0, i1, bytes});
    }
    return QM_OK;
}

int tiled_codes(const qm_decoder &d) {
    int nc = 0;
    for (const Slot &s : d.slots) nc += (s.F > 0 && !lds_slot(d, s)) ? 1 : 0;
    return nc;
}

bool fused_path(const qm_decoder &d) {
    const int nc = tiled_codes(d);
    return nc >= 2 && nc <= QM_MAX_CODES && d.tun.fuse_codes == 1 && d.tun.merge;
}

bool streams_path(const qm_decoder &d) {
    const int nc = tiled_codes(d);
    return nc >= 2 && nc <= QM_MAX_CODES && d.tun.fuse_codes == 2 && d.tun.merge;
}

// Codes on their own streams (tuning fuse_codes = 2): each tiled code runs
// its own layer sequence on its own stream, forked from and joined to the
// decode stream, so the launches of different codes overlap on the device.
// Launches are enqueued round-robin, each code's layers spread evenly over
// the steps of the longest code (as spread_codes), so every stream is fed.
int enqueue_sweeps_streams(qm_decoder &d, int32_t iters, hipStream_t st) {
    const int msgk = msg_kind(d);
    const size_t msg = msg_bytes(d);
    std::vector<Slot *> act;
    for (Slot &s : d.slots)
        if (s.F > 0 && !lds_slot(d, s)) act.push_back(&s);
    std::stable_sort(act.begin(), act.end(),
                     [](const Slot *a, const Slot *b) { return a->gptr.size() > b->gptr.size(); });
    const int nc = (int)act.size();
    if ((int)d.gstreams.size() < nc - 1 || !d.gfork) return fail(QM_ERR_STATE, "code streams missing");
    std::vector<hipStream_t> cs(nc, st);
    std::vector<LayerArgs> base(nc);
    std::vector<int> G(nc);
    int64_t steps = 0;
    // every chain but the longest (act[0]) holds at most resident_cap
    // workgroups per compute unit, through an unused dynamic LDS request
    const uint32_t cap_lds =
        d.tun.resident_cap > 0 ? (uint32_t)std::min(d.lds_per_cu / d.tun.resident_cap, d.lds_limit) : 0u;
    for (int c = 0; c < nc; ++c) {
        if (c > 0) cs[c] = d.gstreams[c - 1];
        base[c] = layer_args(d, *act[c]);
        base[c].shmem = c > 0 ? cap_lds : 0u;
        G[c] = (int)act[c]->gptr.size() - 1;
        steps = std::max<int64_t>(steps, (int64_t)iters * G[c]);
    }
    QM_HIP(hipEventRecord(d.gfork, st));
    for (int c = 1; c < nc; ++c) QM_HIP(hipStreamWaitEvent(cs[c], d.gfork, 0));
    // profiled: one sweep of the longest code (on the decode stream) from
    // the middle of the decode; its launches overlap the other codes'
    const int64_t kprof = (d.profiling && iters >= 2) ? (int64_t)((iters - 1) / 2) * G[0] : -1;
    ProfScope window(d, st, kprof >= 0);
    double wbytes = 0.0, wchecks = 0.0;
    for (int64_t k = 0; k < steps; ++k) {
        if (k == kprof) {
            const int rc = window.begin();
            if (rc != QM_OK) return rc;
        }
        for (int c = 0; c < nc; ++c) {
            const int64_t N = (int64_t)iters * G[c];
            const int64_t j0 = k * N / steps, j1 = (k + 1) * N / steps;
            if (j1 <= j0) continue;
            const Slot &s = *act[c];
            const int t = (int)(j0 / G[c]), gi = (int)(j0 % G[c]);
            LayerArgs la = base[c];
            la.last = (t == iters - 1) ? 1 : 0;
            la.rows = slot_bufs(d, s).rows + s.gptr[gi];
            la.nrows = s.gptr[gi + 1] - s.gptr[gi];
            QM_HIP(qm_launch_layer(la, msgk, s.maxd_t, la.fpl, d.tun.block, d.tun.stream_hint, cs[c]));
            if (c == 0 && kprof >= 0 && k >= kprof && k < kprof + G[0]) {
                double b, ch;
                layer_work(s, s.hrows.data() + s.gptr[gi], la.nrows, msg, &b, &ch);
                wbytes += b;
                wchecks += ch;
            }
        }
        if (kprof >= 0 && k == kprof + G[0] - 1) {
            const int rc = window.end(wbytes, wchecks, G[0]);
            if (rc != QM_OK) return rc;
        }
    }
    for (int c = 1; c < nc; ++c) {
        QM_HIP(hipEventRecord(d.gjoin[c - 1], cs[c]));
        QM_HIP(hipStreamWaitEvent(st, d.gjoin[c - 1], 0));
    }
    return QM_OK;
}

// The launch sequence of one decode (no host synchronisation: capturable).
int enqueue_decode(qm_decoder &d, const float *llr, const uint8_t *syn, int32_t iters, uint8_t *hard, float *app,
                   uint8_t *flags, hipStream_t st) {
    int rc = enqueue_init(d, llr, syn, st);
    if (rc != QM_OK) return rc;
    if (d.flags & QM_FLOODING) {
        for (Slot &s : d.slots) {
            if (s.F == 0) continue;
            if ((rc = enqueue_flood_slot(d, s, iters, st)) != QM_OK) return rc;
        }
        return enqueue_finalize(d, hard, app, flags, st);
    }
    bool any_lds = false, any_tiled = false;
    for (const Slot &s : d.slots) {
        if (s.F == 0) continue;
        (lds_slot(d, s) ? any_lds : any_tiled) = true;
    }
    // LDS-resident codes next to tiled ones run concurrently on the side stream
    const bool fork = any_lds && any_tiled;
    hipStream_t ls = st;
    if (fork) {
        if (!d.side) return fail(QM_ERR_STATE, "side stream missing");
        QM_HIP(hipEventRecord(d.ev_fork, st));
        QM_HIP(hipStreamWaitEvent(d.side, d.ev_fork, 0));
        ls = d.side;
    }
    for (Slot &s : d.slots) {
        if (!lds_slot(d, s)) continue;
        rc = enqueue_sweeps_lds(d, s, iters, ls);
        if (rc != QM_OK) return rc;
    }
    if (fork) QM_HIP(hipEventRecord(d.ev_join, d.side));
    if (fused_path(d)) {
        rc = enqueue_sweeps_fused(d, iters, st);
    } else if (streams_path(d)) {
        rc = enqueue_sweeps_streams(d, iters, st);
    } else {
        for (Slot &s : d.slots) {
            if (s.F == 0 || lds_slot(d, s)) continue;
            rc = enqueue_sweeps_slot(d, s, iters, st);
            if (rc != QM_OK) break;
        }
    }
    if (rc != QM_OK) return rc;
    if (fork) QM_HIP(hipStreamWaitEvent(st, d.ev_join, 0));
    return enqueue_finalize(d, hard, app, flags, st);
}

// ------------------------------------------------------ early termination --

// Sweeps of one code until every frame has met its syndrome or T sweeps
// have run (Results, Table tabearly): after each sweep the frames still
// decoding are tested, those that pass stop and their outputs are written,
// and the frames still decoding are gathered into the leading tiles when
// that frees a tile.  The host stops enqueueing once a poll (every
// kPollEvery sweeps, read one poll late so the queue never drains) shows no
// frame left.  When a
// poll shows that the frames still decoding fit in half a tile, their state
// is copied into a narrower tile (in a tile region whose frames have all
// stopped) and the sweeps go on there: a few frames in a wide tile make
// latency-bound launches that narrow tiles shorten.
constexpr int kPollEvery = 2;  // sweeps between host polls of an early-terminating decode

int enqueue_early_slot(qm_decoder &d, Slot &s, int32_t T, uint8_t *hard, float *app, uint8_t *flags,
                       int32_t *iters_out, hipStream_t st) {
    const qm_code &c = *s.code;
    const TileGeom g0 = geom(d, s);
    const SlotBufs b = slot_bufs(d, s);
    const int msgk = msg_kind(d);
    const size_t msg = msg_bytes(d);
    float *Ad0 = reinterpret_cast<float *>(d.ws + s.oAd);
    uint32_t *act = reinterpret_cast<uint32_t *>(d.ws + s.oAct);
    uint64_t *tmask = reinterpret_cast<uint64_t *>(d.ws + s.oTmask);
    int32_t *map = reinterpret_cast<int32_t *>(d.ws + s.oMap);
    int32_t *perm = reinterpret_cast<int32_t *>(d.ws + s.oPerm);
    int32_t *it = reinterpret_cast<int32_t *>(d.ws + s.oIt);
    int32_t *ctl = reinterpret_cast<int32_t *>(d.ws + s.oCtl);
    int32_t *emit = reinterpret_cast<int32_t *>(d.ws + s.oEmit);
    uint8_t *PA = reinterpret_cast<uint8_t *>(d.ws + s.oPA);
    uint8_t *Pd = reinterpret_cast<uint8_t *>(d.ws + s.oPd);
    uint8_t *PS = reinterpret_cast<uint8_t *>(d.ws + s.oPS);
    const int32_t *cols1 = reinterpret_cast<const int32_t *>(d.ws + s.oCols1);
    const int32_t *d1row = reinterpret_cast<const int32_t *>(d.ws + s.oD1Row);
    const int64_t nR = (int64_t)c.nent1 * c.Z;  // message nodes

    // The current frame-tile geometry and per-node arrays (A, R, S, Ad).
    // g.ntiles is an upper bound of ctl[1] known to the host (the live-tile
    // count only falls, so any count read back earlier in stream order
    // bounds it); grids cover those tiles alone.
    TileGeom g = g0;
    int Fpad = s.Fpad;
    float *A = b.A, *Ad = Ad0, *K = b.K;
    char *R = static_cast<char *>(b.R);
    uint8_t *S = b.S;
    int region = 0;  // tile of the original layout that holds the state once narrowed
    LayerArgs la = layer_args(d, s);
    la.Ad = Ad;
    la.tmask = tmask;
    la.ctl = ctl;
    la.Pd = Pd;
    la.PS = PS;
    la.last = 0;

    QM_HIP(qm_launch_et_init(act, tmask, map, it, ctl, Fpad, g.ntiles, g.ft_log2, st));
    QM_HIP(qm_launch_commit_d1(A, Ad, 0, b.rows, c.mb, g, st));  // Ad = LLR_d
    // packed hard decisions (the degree>=2 variables' before every test, the
    // degree-1 ones here and then by every sweep) and syndrome bits (here,
    // after every compaction and after narrowing)
    QM_HIP(qm_launch_pack_signs(Ad, Pd, s.m, la.fpl, g, st));
    QM_HIP(qm_launch_pack_syndrome(S, PS, nullptr, 0, la.fpl, g, st));
    auto test = [&](int t) -> int {
        // the per-node state of a decoding frame
        const CompactArray arr[] = {{A, s.n, 4}, {R, nR, (int32_t)msg}, {S, s.m, 1}, {Ad, s.m, 4}, {K, s.m, 4}};
        const int narr = (int)(sizeof(arr) / sizeof(arr[0]));
        QM_HIP(qm_launch_pack_cols(A, PA, cols1, (int)s.cols1.size(), ctl, la.fpl, g, st));
        QM_HIP(qm_launch_syndrome_packed(PA, Pd, PS, b.rows, c.mb, b.fail, ctl, la.fpl, g, st));
        QM_HIP(qm_launch_et_plan(b.fail, act, tmask, map, perm, it, emit, flags, s.F, ctl, Fpad, g.ft_log2, t, 0, st));
        QM_HIP(qm_launch_emit(A, Ad, emit, ctl, it, b.rows, d1row, msgk, app, hard, g, st));
        if (g.ntiles > 1) {  // with one tile left no compaction can be planned
            QM_HIP(qm_launch_compact(arr, narr, perm, ctl, g.ft_log2, st));
            QM_HIP(qm_launch_pack_syndrome(S, PS, ctl, 1, la.fpl, g, st));
        }
        return QM_OK;
    };
    // Gather the frames still decoding (all in tile 0 of the current
    // layout) into the first slots of a one-tile layout of 2^ftl frames in
    // the other region; the slot -> frame map, flags and masks follow.
    auto narrow = [&](int ftl) -> int {
        region ^= 1;
        float *A2 = b.A + (int64_t)region * (s.n << g0.ft_log2);
        char *R2 = static_cast<char *>(b.R) + (int64_t)region * (nR << g0.ft_log2) * (int64_t)msg;
        uint8_t *S2 = b.S + (int64_t)region * (s.m << g0.ft_log2);
        float *Ad2 = Ad0 + (int64_t)region * (s.m << g0.ft_log2);
        float *K2 = b.K + (int64_t)region * (s.m << g0.ft_log2);
        QM_HIP(qm_launch_et_narrow_plan(act, tmask, map, perm, ctl, g.ft_log2, ftl, st));
        QM_HIP(qm_launch_narrow(A, A2, perm, s.n, 4, g.ft_log2, ftl, st));
        QM_HIP(qm_launch_narrow(R, R2, perm, nR, (int)msg, g.ft_log2, ftl, st));
        QM_HIP(qm_launch_narrow(S, S2, perm, s.m, 1, g.ft_log2, ftl, st));
        QM_HIP(qm_launch_narrow(Ad, Ad2, perm, s.m, 4, g.ft_log2, ftl, st));
        QM_HIP(qm_launch_narrow(K, K2, perm, s.m, 4, g.ft_log2, ftl, st));
        A = A2;
        R = R2;
        S = S2;
        Ad = Ad2;
        K = K2;
        g.ft_log2 = ftl;
        g.ntiles = 1;
        Fpad = 1 << ftl;
        la.A = A;
        la.R = R;
        la.Ad = Ad;
        la.K = K;
        la.ft_log2 = ftl;
        // one frame per lane in the narrowed tile: its launches are short and
        // bound by each lane's chain of dependent loads, which a lane with one
        // frame finishes sooner (8 frames, one-row layer: 5.5 against 6.6 us);
        // the packed layouts follow fpl, and every packed array the next test
        // reads is rewritten under it (PS here, Pd by the sweep, PA by the test)
        la.fpl = 1;
        la.chunks = ((c.Z << ftl) / la.fpl + d.tun.block - 1) / d.tun.block;
        la.strideA = s.n << ftl;
        la.strideR = nR << ftl;
        la.strideK = s.m << ftl;
        QM_HIP(qm_launch_pack_syndrome(S, PS, nullptr, 0, la.fpl, g, st));
        ++d.et_narrowings;
        return QM_OK;
    };
    int rc = test(0);
    if (rc != QM_OK) return rc;
    const RowDesc *rows = b.rows;
    const int G = (int)s.gptr.size() - 1;
    int pending = -1;
    for (int t = 0; t < T; ++t) {
        // profiled: the first sweep, while every tile still decodes (frames
        // whose channel decisions already pass are the exception)
        ProfScope sweep(d, st, d.profiling && t == 0);
        if ((rc = sweep.begin()) != QM_OK) return rc;
        double bytes = 0.0, checks = 0.0;
        int launches = 0;
        for (int gi = 0; gi < G; ++gi) {
            const int p_lo = s.gptr[gi], p_hi = s.gptr[gi + 1];
            const int step = d.tun.merge ? (p_hi - p_lo) : 1;
            for (int p = p_lo; p < p_hi; p += step) {
                la.rows = rows + p;
                la.nrows = step;
                la.ntiles = g.ntiles;
                QM_HIP(qm_launch_layer_et(la, msgk, s.maxd_t, la.fpl, d.tun.block, d.tun.stream_hint, st));
                double bb, ch;
                layer_work(s, s.hrows.data() + p, step, msg, &bb, &ch, true);
                bytes += bb;
                checks += ch;
                ++launches;
            }
        }
        if ((rc = sweep.end(bytes, checks, launches)) != QM_OK) return rc;
        if ((rc = test(t + 1)) != QM_OK) return rc;
        if ((t + 1) % kPollEvery == 0 && t + 1 < T) {
            if (pending >= 0) {
                QM_HIP(hipEventSynchronize(d.poll_ev[pending]));
                const int32_t *pc = d.h_poll + pending * QM_ET_CTL_WORDS;  // ctl as of that poll
                const int32_t alive = pc[5];
                if (alive == 0) break;
                g.ntiles = std::min(g.ntiles, pc[1]);
                int ftl = 0;
                while ((1 << ftl) < alive) ++ftl;
                if (g0.ntiles >= 2 && g.ntiles == 1 && ftl < g.ft_log2) {
                    if ((rc = narrow(ftl)) != QM_OK) return rc;
                }
            }
            pending = pending < 0 ? 0 : 1 - pending;
            QM_HIP(hipMemcpyAsync(d.h_poll + pending * QM_ET_CTL_WORDS, ctl, QM_ET_CTL_WORDS * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, st));
            QM_HIP(hipEventRecord(d.poll_ev[pending], st));
        }
    }
    // frames still decoding ran all T sweeps and failed the last test
    QM_HIP(qm_launch_et_plan(b.fail, act, tmask, map, perm, it, emit, flags, s.F, ctl, Fpad, g.ft_log2, T, 1, st));
    QM_HIP(qm_launch_emit(A, Ad, emit, ctl, it, b.rows, d1row, msgk, app, hard, g, st));
    if (iters_out && s.F > 0)
        QM_HIP(hipMemcpyAsync(iters_out, it, (size_t)s.F * 4, hipMemcpyDeviceToDevice, st));
    return QM_OK;
}

int validate_inputs(qm_decoder &d, const float *llr, const uint8_t *syn, hipStream_t st) {
    size_t nl = 0, ns = 0;
    for (const Slot &s : d.slots) {
        nl += (size_t)s.F * s.n;
        ns += (size_t)s.F * s.m;
    }
    uint32_t *err = reinterpret_cast<uint32_t *>(d.ws + d.oErr);
    QM_HIP(qm_launch_fill_u32(err, 0u, 1, st));
    QM_HIP(qm_launch_validate(llr, nl, syn, ns, err, st));
    uint32_t h = 0;
    QM_HIP(hipMemcpyAsync(&h, err, 4, hipMemcpyDeviceToHost, st));
    QM_HIP(hipStreamSynchronize(st));
    if (h & 1u) return fail(QM_ERR_INPUT, "non-finite channel LLR");
    if (h & 2u) return fail(QM_ERR_INPUT, "syndrome value other than 0/1");
    return QM_OK;
}

// ---------------------------------------------------------- learned decoder --

int nms_slot(qm_decoder &d, Slot **out) {
    Slot *only = nullptr;
    int n = 0;
    for (Slot &s : d.slots)
        if (s.F > 0) {
            only = &s;
            ++n;
        }
    if (n != 1) return fail(QM_ERR_UNSUPPORTED, "the min-sum decoder takes a decoder with exactly one code");
    if (d.flags & (QM_MSG_FP16 | QM_MSG_FP8))
        return fail(QM_ERR_UNSUPPORTED, "the min-sum decoder keeps float32 messages");
    if (d.flags & QM_FLOODING) return fail(QM_ERR_UNSUPPORTED, "the min-sum decoder is built for the layered schedule");
    *out = only;
    return QM_OK;
}

// Loss terms of a training call whose reverse sweeps may run at once, each
// on its own stream with its own adjoints and partial sums (the reverse
// sweeps of a term read only K, the degree-1 LLRs, the weights and the
// recorded q's, none of which a later forward sweep changes).
constexpr int kAdjSets = 2;

void nms_layout(qm_decoder &d, const Slot &s, int32_t T, int32_t train) {
    const size_t fp = (size_t)s.Fpad, n = (size_t)s.n, m = (size_t)s.m;
    const size_t e = (size_t)s.code->nent1 * s.code->Z;
    size_t off = 0;
    d.oAd = off; off = align_up(off + fp * m * 4);
    d.oAct = off; off = align_up(off + fp * 4);
    d.oTmask = off; off = align_up(off + fp * 8);  // one word per tile (at most Fpad tiles)
    d.oIt = off; off = align_up(off + fp * 4);
    d.oCols = off; off = align_up(off + (size_t)s.code->nb * 4);
    // partial loss sums: one per workgroup of the loss kernel (256 lanes)
    const size_t bce_blocks = (size_t)(s.code->nb + s.code->mb) * (fp * s.code->Z / 256 + fp + 1);
    d.oLossP = off; off = align_up(off + bce_blocks * 4);
    d.oLoss = off; off = align_up(off + 4);
    if (train) {
        d.oX = off; off = align_up(off + fp * n);
        // kAdjSets sets of adjoints (gA, gAd, gR), one per loss term whose
        // reverse sweeps may run at once
        d.ogA = off;
        d.ogAd = d.ogA + align_up(fp * n * 4);
        d.ogR = d.ogAd + align_up(fp * m * 4);
        d.adjSet = d.ogR + align_up(fp * e * 4) - d.ogA;
        off += kAdjSets * d.adjSet;
        // the q's of every sweep inside a backward window (at most T),
        // recorded by the forward sweeps: the reverse sweeps need nothing else
        d.oQ = off; off = align_up(off + (size_t)T * fp * e * 4);
        // per-workgroup gradient sums of the reverse sweep: at most
        // Fpad*Z/64 + Fpad workgroups per (sweep, row)
        d.partSet = align_up((size_t)T * s.code->mb * (fp * s.code->Z / 64 + fp + 1) * 16);
        d.oPart = off; off += kAdjSets * d.partSet;
        d.oClamp = off; off = align_up(off + 4);
    }
    d.nTotal = off;
}

template <typename T>
T *nws_ptr(const qm_decoder &d, size_t off) { return reinterpret_cast<T *>(d.nws + off); }

NmsLayerArgs nms_args(qm_decoder &d, Slot &s) {
    NmsLayerArgs na;
    std::memset(&na, 0, sizeof(na));
    na.L = layer_args(d, s);
    na.Ad = nws_ptr<float>(d, d.oAd);
    return na;
}

// initial state of a min-sum decode: frame tiles, K = |LLR_d| with sign
// s ^ [LLR_d < 0], r = 0, Ad = LLR_d, every frame active
int nms_init(qm_decoder &d, Slot &s, const float *llr, const uint8_t *syn, hipStream_t st) {
    const qm_code &c = *s.code;
    const TileGeom g = geom(d, s);
    const SlotBufs b = slot_bufs(d, s);
    QM_HIP(qm_launch_to_tiles_f32(llr, b.A, s.F, s.n, g.ft_log2, g.ntiles, st));
    QM_HIP(qm_launch_to_tiles_u8(syn, b.S, s.F, s.m, g.ft_log2, g.ntiles, st));
    QM_HIP(qm_launch_nms_kappa(b.A, b.S, b.K, b.rows, c.mb, g, st));
    QM_HIP(qm_launch_fill_u32(reinterpret_cast<uint32_t *>(b.R), 0u, align_up((size_t)s.Fpad * c.nent1 * c.Z * 4) / 4, st));
    QM_HIP(qm_launch_fill_u32(b.fail, 0u, (size_t)s.Fpad, st));
    QM_HIP(qm_launch_commit_d1(b.A, nws_ptr<float>(d, d.oAd), 0, b.rows, c.mb, g, st));
    QM_HIP(qm_launch_fill_u32(nws_ptr<uint32_t>(d, d.oAct), 1u, (size_t)s.Fpad, st));
    QM_HIP(qm_launch_tile_masks(nws_ptr<uint32_t>(d, d.oAct), nws_ptr<uint64_t>(d, d.oTmask), s.Fpad, g.ft_log2, st));
    QM_HIP(qm_launch_fill_u32(nws_ptr<uint32_t>(d, d.oIt), 0u, (size_t)s.Fpad, st));
    return QM_OK;
}

// one sweep t of min-sum layers
int nms_sweep(qm_decoder &d, Slot &s, const float *W, int t, int last, const uint32_t *act, float *Q, hipStream_t st) {
    const RowDesc *rows = slot_bufs(d, s).rows;
    NmsLayerArgs na = nms_args(d, s);
    na.L.last = last;
    na.W = W + (size_t)t * s.code->mb * 4;
    na.act = act;
    na.tmask = act ? nws_ptr<uint64_t>(d, d.oTmask) : nullptr;
    na.Q = Q;
    const int G = (int)s.gptr.size() - 1;
    for (int gi = 0; gi < G; ++gi) {
        const int p_lo = s.gptr[gi], p_hi = s.gptr[gi + 1];
        const int step = d.tun.merge ? (p_hi - p_lo) : 1;
        for (int p = p_lo; p < p_hi; p += step) {
            na.L.rows = rows + p;
            na.L.nrows = step;
            QM_HIP(qm_launch_nms_layer(na, s.maxd_t, na.L.fpl, d.tun.block, st));
        }
    }
    return QM_OK;
}

}  // namespace

extern "C" {

int qm_abi_version(void) { return QM_ABI_VERSION; }

const char *qm_last_error(void) { return g_err.c_str(); }

int qm_code_create(int32_t mb, int32_t nb, int32_t Z, const int32_t *shifts, qm_code **out) {
    if (!out) return fail(QM_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!shifts) return fail(QM_ERR_INVALID_ARG, "shifts is NULL");
    if (mb <= 0 || nb <= 0 || Z <= 0) return fail(QM_ERR_INVALID_ARG, "mb, nb and Z must be positive");
    if ((int64_t)mb * Z > (1 << 30) || (int64_t)nb * Z > (1 << 30))
        return fail(QM_ERR_UNSUPPORTED, "code too large (n or m above 2^30)");
    qm_code *c = new (std::nothrow) qm_code;
    if (!c) return fail(QM_ERR_OOM, "out of host memory");
    c->mb = mb;
    c->nb = nb;
    c->Z = Z;
    c->sh.assign(shifts, shifts + (size_t)mb * nb);
    c->col_deg.assign(nb, 0);
    c->ent.assign((size_t)mb * nb, -1);
    for (int i = 0; i < mb; ++i)
        for (int j = 0; j < nb; ++j) {
            const int a = c->sh[i * nb + j];
            if (a < -1 || a >= Z) {
                delete c;
                return fail(QM_ERR_INVALID_ARG, "shift out of range at (" + std::to_string(i) + "," +
                                                    std::to_string(j) + ")");
            }
            if (a >= 0) {
                c->col_deg[j]++;
                c->edges += Z;
            }
        }
    for (int j = 0; j < nb; ++j) {
        if (c->col_deg[j] == 1) c->ndeg1++;
        if (c->col_deg[j] >= 2) c->ntype1++;
    }
    for (int i = 0; i < mb; ++i) {
        int d = 0, d1 = 0;
        for (int j = 0; j < nb; ++j) {
            if (c->sh[i * nb + j] < 0) continue;
            if (c->col_deg[j] == 1) {
                d1++;
            } else {
                c->ent[i * nb + j] = c->nent1++;
                d++;
            }
        }
        if (d1 > 1) {
            delete c;
            return fail(QM_ERR_UNSUPPORTED, "row " + std::to_string(i) + " holds more than one degree-1 column");
        }
        if (d > QM_MAXD) {
            delete c;
            return fail(QM_ERR_UNSUPPORTED, "row " + std::to_string(i) + " holds more than 16 entries in degree>=2 columns");
        }
        c->max_d = std::max(c->max_d, d);
    }
    greedy_schedule(*c, c->gptr, c->rows);
    *out = c;
    return QM_OK;
}

int qm_code_destroy(qm_code *code) {
    delete code;
    return QM_OK;
}

int qm_code_get_info(const qm_code *c, qm_code_info *info) {
    if (!c || !info) return fail(QM_ERR_INVALID_ARG, "NULL argument");
    info->mb = c->mb;
    info->nb = c->nb;
    info->Z = c->Z;
    info->n = (int64_t)c->nb * c->Z;
    info->m = (int64_t)c->mb * c->Z;
    info->n_type1_cols = c->ntype1;
    info->n_deg1_cols = c->ndeg1;
    info->n_type1_entries = c->nent1;
    info->max_row_type1 = c->max_d;
    info->edges = c->edges;
    info->G = (int32_t)c->gptr.size() - 1;
    return QM_OK;
}

int qm_code_set_schedule(qm_code *c, int32_t G, const int32_t *group_ptr, const int32_t *rows) {
    if (!c || !group_ptr || !rows) return fail(QM_ERR_INVALID_ARG, "NULL argument");
    const int rc = check_schedule(*c, G, group_ptr, rows);
    if (rc != QM_OK) return rc;
    c->gptr.assign(group_ptr, group_ptr + G + 1);
    c->rows.assign(rows, rows + c->mb);
    return QM_OK;
}

int qm_code_get_schedule(const qm_code *c, int32_t *G, int32_t *group_ptr, int32_t *rows) {
    if (!c || !G) return fail(QM_ERR_INVALID_ARG, "NULL argument");
    *G = (int32_t)c->gptr.size() - 1;
    if (group_ptr) std::copy(c->gptr.begin(), c->gptr.end(), group_ptr);
    if (rows) std::copy(c->rows.begin(), c->rows.end(), rows);
    return QM_OK;
}

int qm_decoder_create(const qm_code *const *codes, int32_t ncodes, const int32_t *frames_per_code, int32_t flags,
                      qm_decoder **out) {
    if (!out) return fail(QM_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!codes || !frames_per_code || ncodes <= 0) return fail(QM_ERR_INVALID_ARG, "need at least one code");
    if (flags & ~(QM_MSG_FP16 | QM_MSG_FP8 | QM_VALIDATE | QM_GRAPH | QM_EARLY_STOP | QM_FLOODING))
        return fail(QM_ERR_INVALID_ARG, "unknown flag bits");
    if ((flags & QM_FLOODING) && (flags & QM_EARLY_STOP))
        return fail(QM_ERR_UNSUPPORTED, "early termination is built for the layered schedule only");
    if ((flags & QM_MSG_FP16) && (flags & QM_MSG_FP8))
        return fail(QM_ERR_INVALID_ARG, "QM_MSG_FP16 and QM_MSG_FP8 exclude each other");
    qm_decoder *d = new (std::nothrow) qm_decoder;
    if (!d) return fail(QM_ERR_OOM, "out of host memory");
    d->flags = flags;
    for (int c = 0; c < ncodes; ++c) {
        if (!codes[c] || frames_per_code[c] < 0) {
            delete d;
            return fail(QM_ERR_INVALID_ARG, "bad code or frame count at index " + std::to_string(c));
        }
        Slot s;
        s.code = codes[c];
        s.F = frames_per_code[c];
        if (s.F >= 64) {
            s.Fpad = (s.F + 63) / 64 * 64;
        } else {
            s.Fpad = 0;
            if (s.F > 0) {
                s.Fpad = 1;
                while (s.Fpad < s.F) s.Fpad <<= 1;
            }
        }
        if ((flags & QM_EARLY_STOP) && s.Fpad > QM_ET_MAXF) {
            delete d;
            return fail(QM_ERR_UNSUPPORTED, "early termination takes at most " + std::to_string(QM_ET_MAXF) +
                                                " frames per code");
        }
        s.n = (int64_t)s.code->nb * s.code->Z;
        s.m = (int64_t)s.code->mb * s.code->Z;
        const int64_t widest = std::max<int64_t>(std::max<int64_t>(s.n, s.m), (int64_t)s.code->nent1 * s.code->Z);
        if (widest * 64 * 4 >= (int64_t)1 << 32) {
            delete d;
            return fail(QM_ERR_UNSUPPORTED, "code too wide for 32-bit in-tile byte offsets");
        }
        for (int i : s.code->rows) s.hrows.push_back(make_desc(*s.code, i));
        s.d1row.assign(s.code->nb, -1);
        for (size_t r = 0; r < s.hrows.size(); ++r)
            if (s.hrows[r].d1col >= 0) s.d1row[s.hrows[r].d1col] = (int32_t)r;
        s.gptr = s.code->gptr;
        for (int j = 0; j < s.code->nb; ++j)
            if (s.code->col_deg[j] >= 2) s.cols1.push_back(j);
        if (flags & QM_FLOODING) {
            for (int j : s.cols1) {
                ColDesc cd;
                std::memset(&cd, 0, sizeof(cd));
                cd.col = j;
                for (int i = 0; i < s.code->mb; ++i) {
                    const int a = s.code->sh[i * s.code->nb + j];
                    if (a < 0) continue;
                    if (cd.deg == QM_MAXCD) {
                        delete d;
                        return fail(QM_ERR_UNSUPPORTED, "flooding: a column has more than " +
                                                            std::to_string(QM_MAXCD) + " entries");
                    }
                    cd.ent[cd.deg] = s.code->ent[i * s.code->nb + j];
                    cd.shift[cd.deg] = a;
                    cd.deg++;
                }
                s.hcols.push_back(cd);
            }
        }
        {
            const int md = s.code->max_d;
            s.maxd_t = md <= 2 ? 2 : md <= 6 ? md : md <= 8 ? 8 : 16;
        }
        d->slots.push_back(std::move(s));
    }
    d->tun.frames_per_tile = 16;
    d->tun.block = 128;
    d->tun.merge = 1;
    d->tun.graph = (flags & QM_GRAPH) ? 1 : 0;
    d->tun.frames_per_lane = 2;
    d->tun.fuse_codes = 2;
    d->tun.stream_hint = 1;
    d->tun.tile_groups = 1;
    d->tun.spread_codes = 1;
    d->tun.lds_resident = 2;
    d->tun.frames_per_batch = 0;
    d->tun.resident_cap = 10;
    layout(*d);
    *out = d;
    return QM_OK;
}

int qm_decoder_destroy(qm_decoder *d) {
    if (!d) return QM_OK;
    drop_graph(*d);
    if (d->cap) (void)hipStreamDestroy(d->cap);
    for (hipEvent_t e : d->ev_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : d->poll_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t g : d->gstreams) (void)hipStreamDestroy(g);
    for (hipEvent_t e : d->gjoin) (void)hipEventDestroy(e);
    if (d->gfork) (void)hipEventDestroy(d->gfork);
    for (hipEvent_t e : d->term_done) (void)hipEventDestroy(e);
    if (d->term_fwd) (void)hipEventDestroy(d->term_fwd);
    if (d->ev_fork) (void)hipEventDestroy(d->ev_fork);
    if (d->ev_join) (void)hipEventDestroy(d->ev_join);
    if (d->side) (void)hipStreamDestroy(d->side);
    if (d->h_poll) (void)hipHostFree(d->h_poll);
    delete d;
    return QM_OK;
}

size_t qm_decoder_workspace_bytes(const qm_decoder *d) { return d ? d->total : 0; }

int qm_decoder_bind_workspace(qm_decoder *d, void *dev, size_t bytes) {
    if (!d || !dev) return fail(QM_ERR_INVALID_ARG, "NULL argument");
    if ((reinterpret_cast<uintptr_t>(dev) % kAlign) != 0) return fail(QM_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    if (bytes < d->total)
        return fail(QM_ERR_NO_WORKSPACE, "workspace too small: need " + std::to_string(d->total) + " bytes");
    d->ws = static_cast<char *>(dev);
    d->ws_bytes = bytes;
    drop_graph(*d);
    for (Slot &s : d->slots) {
        QM_HIP(hipMemcpy(d->ws + s.oRows, s.hrows.data(), s.hrows.size() * sizeof(RowDesc), hipMemcpyHostToDevice));
        QM_HIP(hipMemcpy(d->ws + s.oGptr, s.gptr.data(), s.gptr.size() * 4, hipMemcpyHostToDevice));
        if (d->flags & QM_EARLY_STOP)
            QM_HIP(hipMemcpy(d->ws + s.oD1Row, s.d1row.data(), s.d1row.size() * 4, hipMemcpyHostToDevice));
        if (!s.cols1.empty())
            QM_HIP(hipMemcpy(d->ws + s.oCols1, s.cols1.data(), s.cols1.size() * 4, hipMemcpyHostToDevice));
        if (!s.hcols.empty())
            QM_HIP(hipMemcpy(d->ws + s.oColD, s.hcols.data(), s.hcols.size() * sizeof(ColDesc), hipMemcpyHostToDevice));
    }
    int device = 0, lds = 0;
    QM_HIP(hipGetDevice(&device));
    QM_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    d->lds_limit = lds;
    QM_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device));
    d->lds_per_cu = lds;
    QM_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMultiprocessorCount, device));
    d->ncu = lds;
    d->bound = true;
    return QM_OK;
}

int qm_decoder_set_tuning(qm_decoder *d, const qm_tuning *t) {
    if (!d || !t) return fail(QM_ERR_INVALID_ARG, "NULL argument");
    qm_tuning n = *t;
    if (n.frames_per_tile == 0) n.frames_per_tile = 16;
    if (!is_pow2(n.frames_per_tile) || n.frames_per_tile > 64)
        return fail(QM_ERR_INVALID_ARG, "frames_per_tile must be a power of two <= 64");
    if (n.block == 0) n.block = 128;
    if (n.block < 64 || n.block > 256 || n.block % 64)
        return fail(QM_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 256]");
    if (n.frames_per_lane == 0) n.frames_per_lane = 2;
    if (n.frames_per_lane == 4)
        return fail(QM_ERR_UNSUPPORTED, "frames_per_lane 4 (128-bit buffer accesses) is switched off: it gave "
                                        "run-to-run varying results at Z = 20000 whose cause is not established");
    if (n.frames_per_lane != 1 && n.frames_per_lane != 2)
        return fail(QM_ERR_INVALID_ARG, "frames_per_lane must be 1 or 2");
    n.merge = n.merge ? 1 : 0;
    n.graph = n.graph ? 1 : 0;
    if (n.fuse_codes < 0 || n.fuse_codes > 2) return fail(QM_ERR_INVALID_ARG, "fuse_codes must be 0, 1 or 2");
    n.stream_hint = n.stream_hint ? 1 : 0;
    if (n.lds_resident < 0 || n.lds_resident > 2) return fail(QM_ERR_INVALID_ARG, "lds_resident must be 0, 1 or 2");
    n.spread_codes = n.spread_codes ? 1 : 0;
    if (n.frames_per_batch < 0) return fail(QM_ERR_INVALID_ARG, "frames_per_batch must be >= 0");
    if (n.resident_cap != 0 && (n.resident_cap < 3 || n.resident_cap > 64))
        return fail(QM_ERR_INVALID_ARG, "resident_cap must be 0 or in [3, 64]");
    if (n.tile_groups == 0) n.tile_groups = 1;
    if (n.tile_groups != 1 && n.tile_groups != 2 && n.tile_groups != 4 && n.tile_groups != 8)
        return fail(QM_ERR_INVALID_ARG, "tile_groups must be 1, 2, 4 or 8");
    d->tun = n;
    drop_graph(*d);
    return QM_OK;
}

int qm_decoder_get_tuning(const qm_decoder *d, qm_tuning *t) {
    if (!d || !t) return fail(QM_ERR_INVALID_ARG, "NULL argument");
    *t = d->tun;
    return QM_OK;
}

int qm_decode(qm_decoder *d, const float *llr, const uint8_t *syn, int32_t iters, uint8_t *hard, float *app,
              uint8_t *flags, void *stream) {
    if (!d) return fail(QM_ERR_INVALID_ARG, "decoder is NULL");
    if (!d->bound) return fail(QM_ERR_NO_WORKSPACE, "no workspace bound");
    if (iters < 0) return fail(QM_ERR_INVALID_ARG, "iters must be >= 0");
    if (total_frames(*d) == 0) return QM_OK;  // nothing to decode; the buffers may be NULL
    if (!llr || !syn || !hard || !flags) return fail(QM_ERR_INVALID_ARG, "NULL buffer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (d->flags & QM_VALIDATE) {
        const int rc = validate_inputs(*d, llr, syn, st);
        if (rc != QM_OK) return rc;
    }
    if (d->tun.lds_resident) {
        const int rc = ensure_side_stream(*d);
        if (rc != QM_OK) return rc;
    }
    if (d->tun.tile_groups > 1 || d->tun.fuse_codes == 2) {
        const int rc = ensure_group_streams(
            *d, d->tun.fuse_codes == 2 ? std::max<int>(d->tun.tile_groups, QM_MAX_CODES) : d->tun.tile_groups);
        if (rc != QM_OK) return rc;
    }
    if (!d->tun.graph || d->profiling) return enqueue_decode(*d, llr, syn, iters, hard, app, flags, st);

    const void *key[7] = {llr, syn, hard, app, flags, stream, d->ws};
    if (!d->gexec || d->giters != iters || std::memcmp(key, d->gkey, sizeof(key)) != 0) {
        drop_graph(*d);
        // capture on a private stream (the caller's may be the null stream,
        // which cannot be captured); the graph is replayed on the caller's
        if (!d->cap) QM_HIP(hipStreamCreateWithFlags(&d->cap, hipStreamNonBlocking));
        QM_HIP(hipStreamBeginCapture(d->cap, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue_decode(*d, llr, syn, iters, hard, app, flags, d->cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(d->cap, &g);
        if (rc != QM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(QM_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        d->graph = g;
        QM_HIP(hipGraphInstantiate(&d->gexec, d->graph, nullptr, nullptr, 0));
        std::memcpy(d->gkey, key, sizeof(key));
        d->giters = iters;
    }
    QM_HIP(hipGraphLaunch(d->gexec, st));
    return QM_OK;
}

}  // extern "C"

int qm_set_error(int code, const char *msg) { return fail(code, msg); }

// One fixed-sweep decode with `ws` as the decoder's workspace for this call
// only (the allocation-free entry point passes its static scratch array).
// Nothing here allocates: the row, group and column descriptors are copied
// into `ws` on the stream, every kernel argument is a plain pointer into it,
// and the call takes the single-stream launch sequence (no graph, no side or
// group streams, no profiling events).  The tuning switches that would need
// those resources are overridden for the call; each alternative they select
// gives bit-identical outputs.  The decoder's own workspace binding, tuning
// and cached graph are left as they were.
int qm_decode_on_workspace(qm_decoder *d, char *ws, size_t ws_bytes, const float *llr, const uint8_t *syn,
                           int32_t iters, uint8_t *hard, float *app, uint8_t *flags, hipStream_t st) {
    if (!d) return fail(QM_ERR_INVALID_ARG, "decoder is NULL");
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0)
        return fail(QM_ERR_INVALID_ARG, "scratch missing or not 256-byte aligned");
    if (iters < 0) return fail(QM_ERR_INVALID_ARG, "iters must be >= 0");
    if (d->flags & (QM_EARLY_STOP | QM_FLOODING))
        return fail(QM_ERR_UNSUPPORTED, "the allocation-free decode takes fixed-sweep layered decoders only");
    if (d->total > ws_bytes)
        return fail(QM_ERR_NO_WORKSPACE, "the decoder needs " + std::to_string(d->total) +
                                             " workspace bytes; the static scratch holds " + std::to_string(ws_bytes));
    if (total_frames(*d) == 0) return QM_OK;
    if (!llr || !syn || !hard || !flags) return fail(QM_ERR_INVALID_ARG, "NULL buffer");
    int device = 0, v = 0;
    QM_HIP(hipGetDevice(&device));
    // the decoder's state that this call swaps out, restored on every return
    struct Saved {
        qm_decoder *d;
        char *ws;
        size_t ws_bytes;
        bool bound;
        qm_tuning tun;
        int32_t profiling;
        int64_t lds_limit, lds_per_cu;
        int32_t ncu;
        ~Saved() {
            d->ws = ws;
            d->ws_bytes = ws_bytes;
            d->bound = bound;
            d->tun = tun;
            d->profiling = profiling;
            d->lds_limit = lds_limit;
            d->lds_per_cu = lds_per_cu;
            d->ncu = ncu;
        }
    } saved{d, d->ws, d->ws_bytes, d->bound, d->tun, d->profiling, d->lds_limit, d->lds_per_cu, d->ncu};
    d->ws = ws;
    d->ws_bytes = ws_bytes;
    d->bound = true;
    d->profiling = 0;
    d->tun.graph = 0;
    d->tun.tile_groups = 1;
    d->tun.lds_resident = 0;
    if (d->tun.fuse_codes == 2) d->tun.fuse_codes = 1;
    QM_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    d->lds_limit = v;
    QM_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device));
    d->lds_per_cu = v;
    QM_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device));
    d->ncu = v;
    // the scratch keeps whatever the previous call on this device left there
    for (const Slot &s : d->slots) {
        QM_HIP(hipMemcpyAsync(ws + s.oRows, s.hrows.data(), s.hrows.size() * sizeof(RowDesc), hipMemcpyHostToDevice,
                              st));
        QM_HIP(hipMemcpyAsync(ws + s.oGptr, s.gptr.data(), s.gptr.size() * 4, hipMemcpyHostToDevice, st));
        if (d->flags & QM_EARLY_STOP)
            QM_HIP(hipMemcpyAsync(ws + s.oD1Row, s.d1row.data(), s.d1row.size() * 4, hipMemcpyHostToDevice, st));
        if (!s.cols1.empty())
            QM_HIP(hipMemcpyAsync(ws + s.oCols1, s.cols1.data(), s.cols1.size() * 4, hipMemcpyHostToDevice, st));
        if (!s.hcols.empty())
            QM_HIP(hipMemcpyAsync(ws + s.oColD, s.hcols.data(), s.hcols.size() * sizeof(ColDesc),
                                  hipMemcpyHostToDevice, st));
    }
    if (d->flags & QM_VALIDATE) {
        const int rc = validate_inputs(*d, llr, syn, st);
        if (rc != QM_OK) return rc;
    }
    return enqueue_decode(*d, llr, syn, iters, hard, app, flags, st);
}

extern "C" {

int qm_decode_early(qm_decoder *d, const float *llr, const uint8_t *syn, int32_t max_iters, uint8_t *hard,
                    float *app, uint8_t *flags, int32_t *iters_used, void *stream) {
    if (!d) return fail(QM_ERR_INVALID_ARG, "decoder is NULL");
    if (!(d->flags & QM_EARLY_STOP)) return fail(QM_ERR_UNSUPPORTED, "decoder was not created with QM_EARLY_STOP");
    if (!d->bound) return fail(QM_ERR_NO_WORKSPACE, "no workspace bound");
    if (max_iters < 0) return fail(QM_ERR_INVALID_ARG, "max_iters must be >= 0");
    if (total_frames(*d) == 0) return QM_OK;  // nothing to decode; the buffers may be NULL
    if (!llr || !syn || !hard || !flags) return fail(QM_ERR_INVALID_ARG, "NULL buffer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (d->flags & QM_VALIDATE) {
        const int rc = validate_inputs(*d, llr, syn, st);
        if (rc != QM_OK) return rc;
    }
    if (!d->h_poll) {
        void *p = nullptr;
        QM_HIP(hipHostMalloc(&p, 2 * QM_ET_CTL_WORDS * sizeof(int32_t), hipHostMallocDefault));
        d->h_poll = static_cast<int32_t *>(p);
        QM_HIP(hipEventCreateWithFlags(&d->poll_ev[0], hipEventDisableTiming));
        QM_HIP(hipEventCreateWithFlags(&d->poll_ev[1], hipEventDisableTiming));
    }
    int rc = enqueue_init(*d, llr, syn, st);
    if (rc != QM_OK) return rc;
    size_t on = 0, of = 0;
    for (Slot &s : d->slots) {
        if (s.F == 0) continue;
        rc = enqueue_early_slot(*d, s, max_iters, hard + on, app ? app + on : nullptr, flags + of,
                                iters_used ? iters_used + of : nullptr, st);
        if (rc != QM_OK) return rc;
        on += (size_t)s.F * s.n;
        of += (size_t)s.F;
    }
    return QM_OK;
}

int qm_decoder_set_profiling(qm_decoder *d, int32_t enable) {
    if (!d) return fail(QM_ERR_INVALID_ARG, "decoder is NULL");
    d->profiling = enable ? 1 : 0;
    return QM_OK;
}

int qm_decoder_get_profile(qm_decoder *d, qm_profile *out, int32_t reset) {
    if (!d || !out) return fail(QM_ERR_INVALID_ARG, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    for (const auto &p : d->pending) {
        QM_HIP(hipEventSynchronize(d->ev_pool[p.b]));
        float ms = 0.0f;
        QM_HIP(hipEventElapsedTime(&ms, d->ev_pool[p.a], d->ev_pool[p.b]));
        out->launches += p.launches;
        out->sweeps++;
        out->layer_ms += ms;
        out->layer_bytes += p.bytes;
        out->checks += p.checks;
    }
    for (const auto &p : d->lds_pending) {
        QM_HIP(hipEventSynchronize(d->ev_pool[p.b]));
        float ms = 0.0f;
        QM_HIP(hipEventElapsedTime(&ms, d->ev_pool[p.a], d->ev_pool[p.b]));
        out->lds_launches++;
        out->lds_ms += ms;
        out->lds_bytes += p.bytes;
    }
    out->et_narrowings = d->et_narrowings;
    if (reset) {
        d->pending.clear();
        d->lds_pending.clear();
        d->ev_used = 0;
        d->et_narrowings = 0;
    }
    return QM_OK;
}

size_t qm_nms_workspace_bytes(const qm_decoder *dc, int32_t T, int32_t train) {
    if (!dc || T < 0) return 0;
    qm_decoder &d = const_cast<qm_decoder &>(*dc);
    Slot *s = nullptr;
    if (nms_slot(d, &s) != QM_OK) return 0;
    qm_decoder tmp;
    nms_layout(tmp, *s, T, train);
    return tmp.nTotal;
}

int qm_nms_bind_workspace(qm_decoder *d, void *dev, size_t bytes, int32_t T, int32_t train) {
    if (!d || !dev || T < 0) return fail(QM_ERR_INVALID_ARG, "bad argument");
    if ((reinterpret_cast<uintptr_t>(dev) % kAlign) != 0) return fail(QM_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    Slot *s = nullptr;
    int rc = nms_slot(*d, &s);
    if (rc != QM_OK) return rc;
    nms_layout(*d, *s, T, train);
    if (bytes < d->nTotal)
        return fail(QM_ERR_NO_WORKSPACE, "min-sum workspace too small: need " + std::to_string(d->nTotal) + " bytes");
    // a bound min-sum workspace keeps every code on the layer kernels (the
    // LDS-resident engine is not taken), so a graph captured before differs
    drop_graph(*d);
    d->nws = static_cast<char *>(dev);
    d->nws_bytes = bytes;
    d->nT = T;
    d->ntrain = train ? 1 : 0;
    d->acols.clear();
    for (int j = 0; j < s->code->nb; ++j)
        if (s->code->col_deg[j] != 1) d->acols.push_back(j);
    if (!d->acols.empty())
        QM_HIP(hipMemcpy(d->nws + d->oCols, d->acols.data(), d->acols.size() * 4, hipMemcpyHostToDevice));
    return QM_OK;
}

int qm_nms_decode(qm_decoder *d, const float *W, const float *llr, const uint8_t *syn, int32_t T, int32_t early_stop,
                  uint8_t *hard, float *app, uint8_t *flags, int32_t *iters_used, void *stream) {
    if (!d || !W || !llr || !syn || !hard || !flags) return fail(QM_ERR_INVALID_ARG, "NULL argument");
    if (!d->bound || !d->nws) return fail(QM_ERR_NO_WORKSPACE, "decoder or min-sum workspace not bound");
    if (T < 0 || T > d->nT) return fail(QM_ERR_INVALID_ARG, "T must be in [0, T of the bound min-sum workspace]");
    Slot *s = nullptr;
    int rc = nms_slot(*d, &s);
    if (rc != QM_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const qm_code &c = *s->code;
    const TileGeom g = geom(*d, *s);
    const SlotBufs b = slot_bufs(*d, *s);
    float *Ad = nws_ptr<float>(*d, d->oAd);
    uint32_t *act = nws_ptr<uint32_t>(*d, d->oAct);
    int32_t *it = nws_ptr<int32_t>(*d, d->oIt);
    if ((rc = nms_init(*d, *s, llr, syn, st)) != QM_OK) return rc;
    if (early_stop) {
        // frames whose channel decisions already satisfy H c = s stop at 0
        QM_HIP(qm_launch_syndrome(b.A, Ad, b.S, b.rows, c.mb, b.fail, g, st));
        QM_HIP(qm_launch_et_update(b.fail, act, nws_ptr<uint64_t>(*d, d->oTmask), it, s->Fpad, g.ft_log2, 0, st));
    }
    for (int t = 0; t < T; ++t) {
        const int last = early_stop ? 1 : (t == T - 1);
        if ((rc = nms_sweep(*d, *s, W, t, last, early_stop ? act : nullptr, nullptr, st)) != QM_OK) return rc;
        if (early_stop) {
            QM_HIP(qm_launch_syndrome(b.A, Ad, b.S, b.rows, c.mb, b.fail, g, st));
            QM_HIP(qm_launch_et_update(b.fail, act, nws_ptr<uint64_t>(*d, d->oTmask), it, s->Fpad, g.ft_log2, t + 1, st));
        }
    }
    if (early_stop) {
        QM_HIP(qm_launch_et_final(act, it, s->Fpad, T, st));
    } else {
        QM_HIP(qm_launch_fill_u32(reinterpret_cast<uint32_t *>(it), (uint32_t)T, (size_t)s->Fpad, st));
    }
    QM_HIP(qm_launch_commit_d1(b.A, Ad, 1, b.rows, c.mb, g, st));
    QM_HIP(qm_launch_fill_u32(b.fail, 0u, (size_t)s->Fpad, st));
    QM_HIP(qm_launch_syndrome(b.A, nullptr, b.S, b.rows, c.mb, b.fail, g, st));
    QM_HIP(qm_launch_finalize(b.A, b.fail, app, hard, flags, s->F, g, st));
    if (iters_used) QM_HIP(hipMemcpyAsync(iters_used, it, (size_t)s->F * 4, hipMemcpyDeviceToDevice, st));
    return QM_OK;
}

int qm_nms_train_grad(qm_decoder *d, const float *W, const float *llr, const uint8_t *syn, const uint8_t *x,
                      int32_t T, int32_t every_sweep, int32_t window, float *loss, float *grad, int32_t *clamped,
                      void *stream) {
    if (!d || !W || !llr || !syn || !x || !loss || !grad) return fail(QM_ERR_INVALID_ARG, "NULL argument");
    if (!d->bound || !d->nws || !d->ntrain) return fail(QM_ERR_NO_WORKSPACE, "training workspace not bound");
    if (T < 1 || T > d->nT) return fail(QM_ERR_INVALID_ARG, "T must be in [1, T of the bound workspace]");
    if (window == 0) window = T;
    if (window < 1 || window > T) return fail(QM_ERR_INVALID_ARG, "window must be 0 or in [1, T]");
    Slot *s = nullptr;
    int rc = nms_slot(*d, &s);
    if (rc != QM_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const qm_code &c = *s->code;
    const TileGeom g = geom(*d, *s);
    const SlotBufs b = slot_bufs(*d, *s);
    const size_t fp = (size_t)s->Fpad;
    const size_t qsz = fp * (size_t)c.nent1 * c.Z;  // floats of one sweep's q record
    float *Ad = nws_ptr<float>(*d, d->oAd), *Q = nws_ptr<float>(*d, d->oQ);
    int32_t *clamps = nws_ptr<int32_t>(*d, d->oClamp);
    uint8_t *X = nws_ptr<uint8_t>(*d, d->oX);
    // With a loss term in every sweep, consecutive terms' reverse sweeps run
    // on kAdjSets streams at once (term t on set t % kAdjSets), beside the
    // forward sweeps on the caller's stream.  Forward sweep t records its
    // q's in slot t % nq of a ring of nq = window + kAdjSets slots, so it
    // first waits for the last term that reads the slot it overwrites (term
    // t - kAdjSets - 1); term t's loss kernel writes set t % kAdjSets after
    // term t - kAdjSets is done with it.
    const int nsets = (every_sweep && T > 1) ? kAdjSets : 1;
    const int nq = nsets > 1 ? std::min(T, window + nsets) : window;
    const int nev = nsets + 2;  // term events, cycled: a wait never names a re-recorded one
    if (nsets > 1) {
        if ((rc = ensure_group_streams(*d, nsets + 1)) != QM_OK) return rc;
        while ((int)d->term_done.size() < nev) {
            hipEvent_t e = nullptr;
            QM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            d->term_done.push_back(e);
        }
        if (!d->term_fwd) QM_HIP(hipEventCreateWithFlags(&d->term_fwd, hipEventDisableTiming));
    }
    auto gA_of = [&](int k) { return nws_ptr<float>(*d, d->ogA + (size_t)k * d->adjSet); };
    auto gAd_of = [&](int k) { return nws_ptr<float>(*d, d->ogAd + (size_t)k * d->adjSet); };
    auto gR_of = [&](int k) { return nws_ptr<float>(*d, d->ogR + (size_t)k * d->adjSet); };

    if ((rc = nms_init(*d, *s, llr, syn, st)) != QM_OK) return rc;
    QM_HIP(qm_launch_to_tiles_u8(x, X, s->F, s->n, g.ft_log2, g.ntiles, st));
    const RowDesc *rows = b.rows;
    NmsBwdArgs ba;
    std::memset(&ba, 0, sizeof(ba));
    ba.L = layer_args(*d, *s);
    ba.clamps = clamps;
    ba.mb = c.mb;
    const int per_row = ba.L.ntiles * ba.L.chunks;
    const size_t part_floats = (size_t)T * c.mb * per_row * 4;  // one set's partial sums
    float *part = nws_ptr<float>(*d, d->oPart);
    QM_HIP(qm_launch_fill_u32(reinterpret_cast<uint32_t *>(part), 0u, (size_t)nsets * part_floats, st));
    QM_HIP(qm_launch_fill_u32(reinterpret_cast<uint32_t *>(clamps), 0u, 1, st));
    if (nsets > 1) {
        QM_HIP(hipEventRecord(d->term_fwd, st));
        for (int k = 0; k < nsets; ++k) QM_HIP(hipStreamWaitEvent(d->gstreams[k], d->term_fwd, 0));
    }
    const int G = (int)s->gptr.size() - 1;
    const float weight = every_sweep ? 1.0f / (float)T : 1.0f;
    bool first_term = true;
    for (int t = 0; t < T; ++t) {
        // forward sweep t, recording its q's in the ring; the degree-1 APPs
        // are formed in every sweep that ends a loss term
        if (nsets > 1 && t - nsets - 1 >= 0)
            QM_HIP(hipStreamWaitEvent(st, d->term_done[(t - nsets - 1) % nev], 0));
        const bool term = every_sweep || t == T - 1;
        if ((rc = nms_sweep(*d, *s, W, t, term ? 1 : 0, nullptr, Q + (size_t)(t % nq) * qsz, st)) != QM_OK)
            return rc;
        if (!term) continue;
        const int k = t % nsets;
        float *gA = gA_of(k), *gAd = gAd_of(k), *gR = gR_of(k);
        if (nsets > 1 && t - nsets >= 0) QM_HIP(hipStreamWaitEvent(st, d->term_done[(t - nsets) % nev], 0));
        // this sweep's loss term and dL/dAPP; nothing flows back through
        // the messages it wrote
        QM_HIP(qm_launch_bce(b.A, Ad, X, gA, gAd, nws_ptr<float>(*d, d->oLossP), nws_ptr<int32_t>(*d, d->oCols),
                             (int)d->acols.size(), b.rows, c.mb, g, s->F, weight, first_term ? 0 : 1, loss, st));
        first_term = false;
        hipStream_t bs = st;
        if (nsets > 1) {
            bs = d->gstreams[k];
            QM_HIP(hipEventRecord(d->term_fwd, st));
            QM_HIP(hipStreamWaitEvent(bs, d->term_fwd, 0));
        }
        ba.gA = gA;
        ba.gR = gR;
        ba.gAd = gAd;
        ba.part = part + (size_t)k * part_floats;
        // reverse sweeps t, t-1, ... down to the window's first, each from
        // its recorded q's; the degree-1 edges are targets only in sweep t
        for (int u = t; u >= 0 && u > t - window; --u) {
            ba.t = u;
            ba.Q = Q + (size_t)(u % nq) * qsz;
            ba.L.last = (u == t) ? 1 : 0;
            ba.W = W + (size_t)u * c.mb * 4;
            for (int gi = G - 1; gi >= 0; --gi) {
                ba.L.rows = rows + s->gptr[gi];
                ba.L.nrows = s->gptr[gi + 1] - s->gptr[gi];
                QM_HIP(qm_launch_nms_bwd(ba, s->maxd_t, ba.L.fpl, d->tun.block, bs));
            }
        }
        if (nsets > 1) QM_HIP(hipEventRecord(d->term_done[t % nev], bs));
    }
    // join the reverse streams (their last terms), then sum the sets'
    // partials per (sweep, row, component)
    for (int t = std::max(0, T - nsets); nsets > 1 && t < T; ++t)
        QM_HIP(hipStreamWaitEvent(st, d->term_done[t % nev], 0));
    QM_HIP(qm_launch_grad_reduce(part, grad, T, c.mb, per_row, nsets, part_floats, st));
    if (clamped) QM_HIP(hipMemcpyAsync(clamped, clamps, 4, hipMemcpyDeviceToDevice, st));
    return QM_OK;
}

int qm_nms_loss_grad(qm_decoder *d, const float *W, const float *llr, const uint8_t *syn, const uint8_t *x,
                     int32_t T, float *loss, float *grad, void *stream) {
    return qm_nms_train_grad(d, W, llr, syn, x, T, 0, T, loss, grad, nullptr, stream);
}

int qm_generate_frames(qm_decoder *d, int32_t code_index, uint64_t seed, uint64_t first_frame, float snr, int32_t F,
                       uint8_t *x, float *llr, uint8_t *syn, void *stream) {
    if (!d || !x || !llr || !syn || F < 0 || !(snr > 0.0f)) return fail(QM_ERR_INVALID_ARG, "bad argument");
    if (!d->bound) return fail(QM_ERR_NO_WORKSPACE, "no workspace bound");
    if (code_index < 0 || code_index >= (int)d->slots.size()) return fail(QM_ERR_INVALID_ARG, "code_index out of range");
    const Slot &s = d->slots[code_index];
    QM_HIP(qm_launch_framegen(x, llr, syn, slot_bufs(*d, s).rows, s.code->mb, s.code->Z, s.n, s.m, F, seed,
                              first_frame, snr, static_cast<hipStream_t>(stream)));
    return QM_OK;
}

int qm_adam_step(float *w, const float *g, float *m, float *v, int32_t count, float lr, float b1, float b2, float eps,
                 int32_t step, void *stream) {
    if (!w || !g || !m || !v || count < 0 || step < 1) return fail(QM_ERR_INVALID_ARG, "bad argument");
    if (count == 0) return QM_OK;
    QM_HIP(qm_launch_adam(w, g, m, v, count, lr, b1, b2, eps, step, static_cast<hipStream_t>(stream)));
    return QM_OK;
}

int qm_autotune(qm_decoder *d, const float *llr, const uint8_t *syn, int32_t iters, uint8_t *hard, float *app,
                uint8_t *flags, const char *cache_path, void *stream) {
    if (!d) return fail(QM_ERR_INVALID_ARG, "decoder is NULL");
    if (!d->bound) return fail(QM_ERR_NO_WORKSPACE, "no workspace bound");
    if (!llr || !syn || !hard || !flags) return fail(QM_ERR_INVALID_ARG, "NULL buffer");
    if (iters < 1) return fail(QM_ERR_INVALID_ARG, "iters must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int probe = std::min<int>(iters, 8);
    const int saved_prof = d->profiling;
    const int32_t saved_flags = d->flags;
    d->profiling = 0;
    d->flags &= ~QM_VALIDATE;
    hipEvent_t e0, e1;
    QM_HIP(hipEventCreate(&e0));
    QM_HIP(hipEventCreate(&e1));
    FILE *log = cache_path ? std::fopen(cache_path, "a") : nullptr;
    int ncodes = 0;
    for (const Slot &s : d->slots) ncodes += s.F > 0 ? 1 : 0;

    auto trial = [&](const qm_tuning &t, float *ms, int n) -> int {
        d->tun = t;
        drop_graph(*d);
        int rc = qm_decode(d, llr, syn, n, hard, app, flags, stream);  // warm-up (and capture)
        if (rc != QM_OK) return rc;
        QM_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < 2 && rc == QM_OK; ++r) rc = qm_decode(d, llr, syn, n, hard, app, flags, stream);
        if (rc != QM_OK) return rc;
        QM_HIP(hipEventRecord(e1, st));
        QM_HIP(hipEventSynchronize(e1));
        float el = 0.0f;
        QM_HIP(hipEventElapsedTime(&el, e0, e1));
        *ms = el / 2.0f;
        if (log)
            std::fprintf(log,
                         "{\"frames_per_tile\": %d, \"frames_per_lane\": %d, \"block\": %d, \"merge\": %d, "
                         "\"fuse_codes\": %d, \"graph\": %d, \"stream_hint\": %d, \"lds_resident\": %d, "
                         "\"tile_groups\": %d, \"spread_codes\": %d, \"resident_cap\": %d, \"iters\": %d, "
                         "\"ms\": %.4f}\n",
                         t.frames_per_tile, t.frames_per_lane, t.block, t.merge, t.fuse_codes, t.graph,
                         t.stream_hint, t.lds_resident, t.tile_groups, t.spread_codes, t.resident_cap, n, *ms);
        return QM_OK;
    };

    qm_tuning best = d->tun;
    float best_ms = 1e30f;
    int rc = QM_OK;
    const int fts[3] = {16, 32, 64}, fpls[2] = {1, 2}, blocks[2] = {128, 256};
    for (int a = 0; a < 3 && rc == QM_OK; ++a)
        for (int b = 0; b < 2 && rc == QM_OK; ++b)
            for (int c = 0; c < 2 && rc == QM_OK; ++c) {
                qm_tuning t = d->tun;
                t.frames_per_tile = fts[a];
                t.frames_per_lane = fpls[b];
                t.block = blocks[c];
                t.merge = 1;
                t.graph = 0;
                // the launch shape only matters to the layer kernels: time
                // those (the LDS-resident engine is a structural variant)
                t.lds_resident = 0;
                float ms = 0.0f;
                rc = trial(t, &ms, probe);
                if (rc == QM_OK && ms < best_ms) {
                    best_ms = ms;
                    best = t;
                }
            }
    // could a code use the LDS-resident kernel?
    bool lds_candidate = false;
    {
        const qm_tuning keep = d->tun;
        d->tun.lds_resident = 1;
        for (const Slot &s : d->slots) lds_candidate = lds_candidate || lds_slot(*d, s);
        d->tun = keep;
    }
    // structural variants on top of the best launch shape, timed over the
    // full sweep count (at most 256): a graph captured for a few sweeps, or
    // extra streams over a few sweeps, do not predict the whole decode
    const int full = std::min<int>(iters, 256);
    if (rc == QM_OK) rc = trial(best, &best_ms, full);
    const int caps[3] = {0, 8, 12};
    for (int v = 0; v < 11 && rc == QM_OK; ++v) {
        qm_tuning t = best;
        if (v >= 8) {
            // codes on their own streams: other residency caps of the
            // shorter chains (the default is 10)
            if (ncodes < 2 || t.fuse_codes != 2 || t.resident_cap == caps[v - 8]) continue;
            t.resident_cap = caps[v - 8];
        }
        if (v == 7) {
            if (ncodes < 2 || !t.fuse_codes) continue;
            t.spread_codes = !t.spread_codes;
        }
        if (v == 5 || v == 6) {
            if (ncodes != 1) continue;  // fused mixed batches do not use tile groups
            t.tile_groups = v == 5 ? 2 : 4;
        }
        if (v == 4) {
            if (!lds_candidate || t.lds_resident == 1) continue;
            t.lds_resident = 1;
        }
        if (v == 3) t.stream_hint = !t.stream_hint;
        if (v == 0) t.merge = 0;
        if (v == 1) {
            if (ncodes < 2) continue;
            t.fuse_codes = t.fuse_codes == 2 ? 1 : 2;
        }
        if (v == 2) t.graph = 1;
        float ms = 0.0f;
        rc = trial(t, &ms, full);
        if (rc == QM_OK && ms < best_ms) {
            best_ms = ms;
            best = t;
        }
    }
    if (log) std::fclose(log);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    d->tun = best;
    drop_graph(*d);
    d->profiling = saved_prof;
    d->flags = saved_flags;
    return rc;
}

}  // extern "C"
