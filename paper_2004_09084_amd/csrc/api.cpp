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
        } else {
            d.col[d.d] = j;
            d.shift[d.d] = a;
            d.ent[d.d] = c.ent[i * c.nb + j];
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
    std::vector<RowDesc> hrows;  // schedule order
    std::vector<int32_t> gptr;
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
    struct Pending { size_t a, b; double bytes, checks; int kind; };  // kind 0: layer, 1: sweep
    std::vector<Pending> pending;
};

namespace {

int slot_ft(const qm_decoder &d, const Slot &s) {
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
    const size_t msg = (d.flags & QM_MSG_FP16) ? 2 : 4;
    for (Slot &s : d.slots) {
        const size_t fp = (size_t)s.Fpad;
        s.oA = off; off = align_up(off + fp * (size_t)s.n * 4);
        s.oR = off; off = align_up(off + fp * (size_t)s.code->nent1 * (size_t)s.code->Z * msg);
        s.oK = off; off = align_up(off + fp * (size_t)s.m * 4);
        s.oS = off; off = align_up(off + fp * (size_t)s.m);
        s.oFail = off; off = align_up(off + fp * 4);
        s.oRows = off; off = align_up(off + s.hrows.size() * sizeof(RowDesc));
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
void layer_work(const Slot &s, const RowDesc *hrows, int nrows, int msg16, double *bytes, double *checks) {
    const double per_edge = msg16 ? 12.0 : 16.0;
    double b = 0.0;
    for (int r = 0; r < nrows; ++r) b += per_edge * hrows[r].d + 4.0;
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

// The launch sequence of one decode (no host synchronisation: capturable).
int enqueue_decode(qm_decoder &d, const float *llr, const uint8_t *syn, int32_t iters, uint8_t *hard, float *app,
                   uint8_t *flags, hipStream_t st) {
    size_t on = 0, om = 0, of = 0;
    const int msg16 = (d.flags & QM_MSG_FP16) ? 1 : 0;
    for (Slot &s : d.slots) {
        if (s.F == 0) continue;
        const qm_code &c = *s.code;
        const TileGeom g = geom(d, s);
        float *A = reinterpret_cast<float *>(d.ws + s.oA);
        void *R = d.ws + s.oR;
        float *K = reinterpret_cast<float *>(d.ws + s.oK);
        uint8_t *S = reinterpret_cast<uint8_t *>(d.ws + s.oS);
        uint32_t *fl = reinterpret_cast<uint32_t *>(d.ws + s.oFail);
        const RowDesc *rows = reinterpret_cast<const RowDesc *>(d.ws + s.oRows);

        QM_HIP(qm_launch_to_tiles_f32(llr + on, A, s.F, s.n, g.ft_log2, g.ntiles, st));
        QM_HIP(qm_launch_to_tiles_u8(syn + om, S, s.F, s.m, g.ft_log2, g.ntiles, st));
        QM_HIP(qm_launch_kappa(A, S, K, rows, c.mb, g, st));
        const size_t rbytes = align_up((size_t)s.Fpad * c.nent1 * c.Z * (msg16 ? 2 : 4));
        QM_HIP(qm_launch_fill_u32(reinterpret_cast<uint32_t *>(R), 0u, rbytes / 4, st));
        QM_HIP(qm_launch_fill_u32(fl, 0u, (size_t)s.Fpad, st));

        LayerArgs la;
        la.A = A;
        la.R = R;
        la.K = K;
        la.Z = c.Z;
        la.ft_log2 = g.ft_log2;
        la.ntiles = g.ntiles;
        la.fpl = std::min(d.tun.frames_per_lane, 1 << g.ft_log2);
        const int lanes = (c.Z << g.ft_log2) / la.fpl;
        la.chunks = (lanes + d.tun.block - 1) / d.tun.block;
        la.strideA = (int64_t)s.n << g.ft_log2;
        la.strideR = ((int64_t)c.nent1 * c.Z) << g.ft_log2;
        la.strideK = (int64_t)s.m << g.ft_log2;
        const int G = (int)s.gptr.size() - 1;
        // the profiled sweep: the middle one, never the last (which also
        // forms the degree-1 APPs)
        const int tprof = (d.profiling && iters >= 2) ? (iters - 1) / 2 : -1;
        auto launch = [&](int p0, int nr, bool prof) -> int {
            la.rows = rows + p0;
            la.nrows = nr;
            if (!prof) {
                QM_HIP(qm_launch_layer(la, msg16, s.maxd_t, la.fpl, d.tun.block, st));
                return QM_OK;
            }
            hipEvent_t e0, e1;
            size_t i0, i1;
            int rc = take_event(d, &e0, &i0);
            if (rc == QM_OK) rc = take_event(d, &e1, &i1);
            if (rc != QM_OK) return rc;
            QM_HIP(hipEventRecord(e0, st));
            QM_HIP(qm_launch_layer(la, msg16, s.maxd_t, la.fpl, d.tun.block, st));
            QM_HIP(hipEventRecord(e1, st));
            qm_decoder::Pending pd{i0, i1, 0.0, 0.0, 0};
            layer_work(s, s.hrows.data() + p0, nr, msg16, &pd.bytes, &pd.checks);
            d.pending.push_back(pd);
            return QM_OK;
        };
        for (int t = 0; t < iters; ++t) {
            la.last = (t == iters - 1) ? 1 : 0;
            const bool prof = (t == tprof);
            size_t sw0 = 0, sw1 = 0;
            hipEvent_t es0 = nullptr, es1 = nullptr;
            if (prof) {
                const int rc = take_event(d, &es0, &sw0);
                if (rc != QM_OK) return rc;
                QM_HIP(hipEventRecord(es0, st));
            }
            for (int gi = 0; gi < G; ++gi) {
                if (d.tun.merge) {
                    const int rc = launch(s.gptr[gi], s.gptr[gi + 1] - s.gptr[gi], prof);
                    if (rc != QM_OK) return rc;
                } else {
                    for (int p = s.gptr[gi]; p < s.gptr[gi + 1]; ++p) {
                        const int rc = launch(p, 1, prof);
                        if (rc != QM_OK) return rc;
                    }
                }
            }
            if (prof) {
                const int rc = take_event(d, &es1, &sw1);
                if (rc != QM_OK) return rc;
                QM_HIP(hipEventRecord(es1, st));
                d.pending.push_back(qm_decoder::Pending{sw0, sw1, 0.0, 0.0, 1});
            }
        }
        QM_HIP(qm_launch_syndrome(A, S, rows, c.mb, fl, g, st));
        QM_HIP(qm_launch_finalize(A, fl, app ? app + on : nullptr, hard + on, flags + of, s.F, g, st));
        on += (size_t)s.F * s.n;
        om += (size_t)s.F * s.m;
        of += (size_t)s.F;
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
    if (flags & ~(QM_MSG_FP16 | QM_PERSISTENT | QM_VALIDATE | QM_GRAPH))
        return fail(QM_ERR_INVALID_ARG, "unknown flag bits");
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
        s.n = (int64_t)s.code->nb * s.code->Z;
        s.m = (int64_t)s.code->mb * s.code->Z;
        const int64_t widest = std::max<int64_t>(std::max<int64_t>(s.n, s.m), (int64_t)s.code->nent1 * s.code->Z);
        if (widest * 64 * 4 >= (int64_t)1 << 32) {
            delete d;
            return fail(QM_ERR_UNSUPPORTED, "code too wide for 32-bit in-tile byte offsets");
        }
        for (int i : s.code->rows) s.hrows.push_back(make_desc(*s.code, i));
        s.gptr = s.code->gptr;
        {
            const int md = s.code->max_d;
            s.maxd_t = md <= 2 ? 2 : md <= 6 ? md : md <= 8 ? 8 : 16;
        }
        d->slots.push_back(std::move(s));
    }
    d->tun.frames_per_tile = 16;
    d->tun.block = 256;
    d->tun.merge = 1;
    d->tun.persistent = (flags & QM_PERSISTENT) ? 1 : 0;
    d->tun.graph = (flags & QM_GRAPH) ? 1 : 0;
    d->tun.frames_per_lane = 2;
    layout(*d);
    *out = d;
    return QM_OK;
}

int qm_decoder_destroy(qm_decoder *d) {
    if (!d) return QM_OK;
    drop_graph(*d);
    if (d->cap) (void)hipStreamDestroy(d->cap);
    for (hipEvent_t e : d->ev_pool) (void)hipEventDestroy(e);
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
    for (Slot &s : d->slots)
        QM_HIP(hipMemcpy(d->ws + s.oRows, s.hrows.data(), s.hrows.size() * sizeof(RowDesc), hipMemcpyHostToDevice));
    d->bound = true;
    return QM_OK;
}

int qm_decoder_set_tuning(qm_decoder *d, const qm_tuning *t) {
    if (!d || !t) return fail(QM_ERR_INVALID_ARG, "NULL argument");
    qm_tuning n = *t;
    if (n.frames_per_tile == 0) n.frames_per_tile = 16;
    if (!is_pow2(n.frames_per_tile) || n.frames_per_tile > 64)
        return fail(QM_ERR_INVALID_ARG, "frames_per_tile must be a power of two <= 64");
    if (n.block == 0) n.block = 256;
    if (n.block < 64 || n.block > 256 || n.block % 64)
        return fail(QM_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 256]");
    if (n.persistent) return fail(QM_ERR_UNSUPPORTED, "persistent launch not available");
    if (n.frames_per_lane == 0) n.frames_per_lane = 2;
    if (n.frames_per_lane == 4)
        return fail(QM_ERR_UNSUPPORTED, "frames_per_lane 4 (128-bit buffer accesses) is switched off: it gave "
                                        "run-to-run varying results at Z = 20000 whose cause is not established");
    if (n.frames_per_lane != 1 && n.frames_per_lane != 2)
        return fail(QM_ERR_INVALID_ARG, "frames_per_lane must be 1 or 2");
    n.merge = n.merge ? 1 : 0;
    n.graph = n.graph ? 1 : 0;
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
    if (!llr || !syn || !hard || !flags) return fail(QM_ERR_INVALID_ARG, "NULL buffer");
    if (iters < 0) return fail(QM_ERR_INVALID_ARG, "iters must be >= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (d->flags & QM_VALIDATE) {
        size_t nl = 0, ns = 0;
        for (const Slot &s : d->slots) {
            nl += (size_t)s.F * s.n;
            ns += (size_t)s.F * s.m;
        }
        uint32_t *err = reinterpret_cast<uint32_t *>(d->ws + d->oErr);
        QM_HIP(qm_launch_fill_u32(err, 0u, 1, st));
        QM_HIP(qm_launch_validate(llr, nl, syn, ns, err, st));
        uint32_t h = 0;
        QM_HIP(hipMemcpyAsync(&h, err, 4, hipMemcpyDeviceToHost, st));
        QM_HIP(hipStreamSynchronize(st));
        if (h & 1u) return fail(QM_ERR_INPUT, "non-finite channel LLR");
        if (h & 2u) return fail(QM_ERR_INPUT, "syndrome value other than 0/1");
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
        if (p.kind == 0) {
            out->launches++;
            out->layer_ms += ms;
            out->layer_bytes += p.bytes;
            out->checks += p.checks;
        } else {
            out->sweeps++;
            out->sweep_ms += ms;
        }
    }
    if (reset) {
        d->pending.clear();
        d->ev_used = 0;
    }
    return QM_OK;
}

int qm_autotune(qm_decoder *d, const float *llr, const uint8_t *syn, int32_t iters, const char *cache_path,
                void *stream) {
    (void)d; (void)llr; (void)syn; (void)iters; (void)cache_path; (void)stream;
    return fail(QM_ERR_UNSUPPORTED, "autotune not available yet");
}

}  // extern "C"
