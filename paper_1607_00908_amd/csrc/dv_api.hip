// Host side of libdv: the C ABI declared in include/dv.h.
//
// A context owns every device buffer, sized once from the lattice, K_max and
// the batch size.  Pushes are queued on the host; when `batch` frames are
// queued, or at the next synchronising call, the queued frames go to the
// device together: each stage is one launch over all of them (frame =
// blockIdx.z, slot i holds the buffers of the batch's i-th frame), all on the
// context's stream, so no cross-stream ordering is needed and the host pays
// ten launches per batch.  The comparisons of a batch are independent: the
// device knows each frame's past from the frame headers.  Synchronising
// calls flush the queue, wait for the stream and copy the headers (and the
// requested arrays) back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <string>
#include <vector>

#include "dv.h"
#include "dv_internal.h"

// Completion event of one launch, shared by the contexts whose frames it
// carried (a group launch serves several).
struct LaunchEv {
    hipEvent_t e = nullptr;
    ~LaunchEv() {
        if (e) (void)hipEventDestroy(e);
    }
};
using EvRef = std::shared_ptr<LaunchEv>;

// Frames [.., end) of results page `page` are complete when `ev` is.
struct PageLaunch {
    EvRef ev;
    int page;
    int end;
};

struct dv_ctx {
    dv_config cfg;
    int device;
    hipStream_t stream;
    bool own_stream;
    int batch;               // frames per launch
    Bufs h_tab[DV_MAX_BATCH];  // host copy of the slot table
    Bufs *d_tab;             // device slot table
    Fields pending;          // queued field pointers
    int npending;
    int last;                // slot of the most recent frame sent to the device
    void *region;            // every device buffer of the context (one allocation)
    SeqState *h_state;       // pinned mirrors of the headers
    FrameState *h_frame;
    int32_t *d_edge_scratch; // [2 * K_max] for the couple-list getter
    int32_t *d_edge_ab;      // [K_max * max_degree] pairs
    int32_t *d_edge_total;
    uint8_t *d_obst;         // obstacle mask (DV_OBSTACLES), else null
    bool pushed;
    Prof prof;
    std::string err;
    // results pages: page p holds the records of up to pg_cap frames in
    // pinned host memory (written by the device) and their flips in device
    // memory.  Frames fill the current page in push order; when the next
    // launch does not fit, the other page is emptied and becomes current.
    bool keep_results;         // DV_KEEP_RESULTS: no frame is dropped unread
    int pg_cap;                // frames per page: max(batch, 8)
    FrameOut *h_pg[2];         // host view of the records
    int32_t *d_pgf[2];         // flips of each page
    int cur_pg;
    int pg_n[2];               // frames placed in each page
    int pg_rd[2];              // frames of each page returned by dv_get_results
    int last_pg, last_pos;     // record of the most recent frame
    std::deque<PageLaunch> inflight;  // launches with unread frames, oldest first
    // results moved to host memory before their page was reused, unread
    std::vector<dv_frame_info> sp_info;
    std::vector<dv_flip> sp_flips;
    size_t sp_head_info, sp_head_flips;
    hipStream_t copy_stream;   // device-to-host copies of completed results
};

namespace {

thread_local std::string g_create_error;

dv_status fail(dv_ctx *c, dv_status s, const std::string &msg) {
    if (c) c->err = msg;
    else g_create_error = msg;
    return s;
}

void place_comp(Carve &cv, CompBuf &C, size_t K, int maxdeg) {
    C.qx = cv.take<int32_t>(K);
    C.qy = cv.take<int32_t>(K);
    C.fx = cv.take<double>(K);
    C.fy = cv.take<double>(K);
    C.n = cv.take<int32_t>(K);
    C.root = cv.take<int32_t>(K);
    C.amb = cv.take<int32_t>(K);
    C.adj = cv.take<int32_t>(K * maxdeg);
}

void drop_events(dv_ctx *c) {
    if (c->prof.ev) {
        for (int i = 0; i < 2 * c->prof.cap; ++i) (void)hipEventDestroy(c->prof.ev[i]);
        delete[] c->prof.ev;
    }
    c->prof = Prof();
}

dv_status device_fail(dv_ctx *c, const char *what, hipError_t e) {
    return fail(c, DV_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

dv_frame_info to_info(const FrameOut &r) {
    dv_frame_info fi;
    std::memset(&fi, 0, sizeof(fi));
    fi.frame = r.frame;
    fi.status = r.status;
    fi.n_components = r.K;
    fi.n_edges = r.status == 0 ? r.E : 0;
    fi.n_flips = r.n_flips;
    fi.n_breaking = r.n_break;
    fi.n_excluded_past = r.excl_past;
    fi.n_excluded_now = r.excl_now;
    fi.n_ambiguous_centroids = r.amb;
    fi.global_trigger = (uint32_t)r.trigger;
    return fi;
}

// Records and flips of frames [a, b) of page p (their launches complete) into
// host memory; the page's flips of consecutive frames are contiguous.
dv_status read_frames(dv_ctx *c, int p, int a, int b, dv_frame_info *info, dv_flip *flips, int *nfl) {
    const FrameOut *R = c->h_pg[p];
    const int f0 = R[a].flip_off;
    int f = f0;
    for (int i = a; i < b; ++i) {
        if (R[i].flip_off != f || R[i].n_flips < 0)
            return fail(c, DV_ERR_INTERNAL, "results page records are inconsistent");
        f += R[i].n_flips;
        info[i - a] = to_info(R[i]);
    }
    *nfl = f - f0;
    if (f > f0) {
        hipError_t e = hipMemcpyAsync(flips, c->d_pgf[p] + (size_t)6 * f0, (size_t)(f - f0) * sizeof(dv_flip),
                                      hipMemcpyDeviceToHost, c->copy_stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->copy_stream);
        if (e != hipSuccess) return device_fail(c, "results copy failed", e);
    }
    return DV_OK;
}

// Move the unread frames of page p to host memory (waits for their launches).
dv_status spill(dv_ctx *c, int p) {
    for (auto it = c->inflight.rbegin(); it != c->inflight.rend(); ++it)
        if (it->page == p) {
            const hipError_t e = hipEventSynchronize(it->ev->e);
            if (e != hipSuccess) return device_fail(c, "results wait failed", e);
            break;   // stream order: the page's earlier launches are complete too
        }
    const int a = c->pg_rd[p], b = c->pg_n[p];
    if (b > a) {
        const FrameOut *R = c->h_pg[p];
        const int nf = R[b - 1].flip_off + R[b - 1].n_flips - R[a].flip_off;
        const size_t i0 = c->sp_info.size(), f0 = c->sp_flips.size();
        c->sp_info.resize(i0 + (b - a));
        c->sp_flips.resize(f0 + (size_t)std::max(nf, 0));
        int got = 0;
        dv_status s = read_frames(c, p, a, b, c->sp_info.data() + i0, c->sp_flips.data() + f0, &got);
        if (s != DV_OK) return s;
    }
    c->pg_rd[p] = b;
    return DV_OK;
}

// Page position of the next k frames of c (k <= pg_cap): the current page, or
// the other one emptied when they do not fit.  Returns the position word of
// the first frame (DV_PG_*); the others follow it.
dv_status take_page(dv_ctx *c, int k, uint32_t *ps0) {
    int p = c->cur_pg;
    bool fresh = c->pg_n[p] == 0;
    if (c->pg_n[p] + k > c->pg_cap) {
        const int o = 1 - p;
        if (c->keep_results && c->pg_rd[o] < c->pg_n[o]) {
            dv_status s = spill(c, o);
            if (s != DV_OK) return s;
        }
        for (auto it = c->inflight.begin(); it != c->inflight.end();)
            it = it->page == o ? c->inflight.erase(it) : it + 1;
        p = o;
        c->cur_pg = o;
        c->pg_n[o] = 0;
        c->pg_rd[o] = 0;
        fresh = true;
    }
    *ps0 = (uint32_t)c->pg_n[p] | ((uint32_t)p << 6) | (fresh ? 128u : 0u);
    return DV_OK;
}

// After a launch that placed k frames of c in its current page.
void note_launch(dv_ctx *c, int k, const EvRef &ev) {
    const int p = c->cur_pg;
    c->last_pg = p;
    c->last_pos = c->pg_n[p] + k - 1;
    c->pg_n[p] += k;
    if (c->keep_results) c->inflight.push_back(PageLaunch{ev, p, c->pg_n[p]});
}

// Completion event of a launch just enqueued on stream s.
dv_status record_launch(dv_ctx *c, hipStream_t s, EvRef *out) {
    auto ev = std::make_shared<LaunchEv>();
    hipError_t e = hipEventCreateWithFlags(&ev->e, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev->e, s);
    if (e != hipSuccess) return device_fail(c, "event record failed", e);
    *out = ev;
    return DV_OK;
}

// send the queued frames to the device
dv_status flush(dv_ctx *c) {
    const int n = c->npending;
    if (n == 0) return DV_OK;
    const Bufs &H = c->h_tab[0];
    Batch G;
    std::memset(&G, 0, sizeof(G));
    G.D = c->d_tab;
    G.n = n;
    uint32_t ps0 = 0;
    dv_status ts = take_page(c, n, &ps0);
    if (ts != DV_OK) return ts;
    for (int i = 0; i < n; ++i) G.idx[i] = i;
    for (int i = 0; i < n; ++i) G.pslot[i] = ps0 + (uint32_t)i;
    for (int i = 0; i <= n; ++i) {
        G.tbase[i] = i * H.ncells;
        G.bbase[i] = i * H.nty;
    }
    G.tiles = n * H.ncells;
    G.bands = n * H.nty;
    G.tpe = H.ncells;
    G.bpe = H.nty;
    G.kmax = H.kmax;
    G.nty = H.nty;
    G.classify = H.classify;
    G.geom = (H.open_x | H.open_y | (H.obst != nullptr)) ? 1 : 0;
    G.weighted = H.weighted;
    launch_label(G, c->pending, c->stream, c->prof);
    launch_voronoi(G, c->stream, c->prof);
    launch_compare(G, c->stream, c->prof);
    c->npending = 0;
    c->last = n - 1;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, DV_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    EvRef ev;
    if (c->keep_results) {
        dv_status rs = record_launch(c, c->stream, &ev);
        if (rs != DV_OK) return rs;
    }
    note_launch(c, n, ev);
    return DV_OK;
}

dv_status drain(dv_ctx *c) {
    dv_status s = flush(c);
    if (s != DV_OK) return s;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, DV_ERR_DEVICE, "stream error");
    return DV_OK;
}

void release(dv_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_events(c);
    if (c->region) (void)hipFree(c->region);
    c->region = nullptr;
    if (c->h_state) (void)hipHostFree(c->h_state);
    if (c->h_frame) (void)hipHostFree(c->h_frame);
    c->h_state = nullptr;
    c->h_frame = nullptr;
    c->inflight.clear();
    for (int p = 0; p < 2; ++p) {
        if (c->h_pg[p]) (void)hipHostFree(c->h_pg[p]);
        c->h_pg[p] = nullptr;
    }
    if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
    c->copy_stream = nullptr;
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    c->stream = nullptr;
}

dv_status check_cfg(const dv_config *cfg) {
    if (!cfg) return fail(nullptr, DV_ERR_ARG, "config is NULL");
    if (cfg->size != sizeof(dv_config)) return fail(nullptr, DV_ERR_ARG, "config size mismatch");
    if (cfg->lx < 3 || cfg->ly < 3 || cfg->lx > 65536 || cfg->ly > 65536)
        return fail(nullptr, DV_ERR_ARG, "lattice sides must be in [3, 65536]");
    if ((long long)cfg->lx * cfg->ly >= (1LL << 31))
        return fail(nullptr, DV_ERR_ARG, "lattice has 2^31 sites or more");
    if (cfg->phase != DV_PHASE_ABOVE && cfg->phase != DV_PHASE_BELOW)
        return fail(nullptr, DV_ERR_ARG, "phase must be DV_PHASE_ABOVE or DV_PHASE_BELOW");
    if (cfg->connectivity != 4 && cfg->connectivity != 8)
        return fail(nullptr, DV_ERR_ARG, "connectivity must be 4 or 8");
    if (cfg->max_components < 1 || cfg->max_components > (1 << 24))
        return fail(nullptr, DV_ERR_ARG, "max_components must be in [1, 2^24]");
    if (cfg->max_degree != 0 && (cfg->max_degree < 4 || cfg->max_degree > 64))
        return fail(nullptr, DV_ERR_ARG, "max_degree must be 0 or in [4, 64]");
    if (cfg->threshold != cfg->threshold) return fail(nullptr, DV_ERR_ARG, "threshold is NaN");
    if (cfg->flags & ~(DV_KEEP_MAPS | DV_CLASSIFY | DV_OBSTACLES | DV_OPEN_X | DV_OPEN_Y | DV_KEEP_RESULTS |
                       DV_WEIGHTED))
        return fail(nullptr, DV_ERR_ARG, "unknown flag bits");
    if (cfg->max_batch < 0 || cfg->max_batch > DV_MAX_BATCH)
        return fail(nullptr, DV_ERR_ARG, "max_batch must be 0 or in [1, 64]");
    return DV_OK;
}

dv_status sync_state(dv_ctx *c) {
    dv_status s = flush(c);
    if (s != DV_OK) return s;
    if (hipMemcpyAsync(c->h_state, c->h_tab[0].st, sizeof(SeqState), hipMemcpyDeviceToHost,
                       c->stream) != hipSuccess ||
        hipMemcpyAsync(c->h_frame, c->h_tab[c->last].fs, sizeof(FrameState),
                       hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(c, DV_ERR_DEVICE, std::string("device error: ") + hipGetErrorString(hipGetLastError()));
    return DV_OK;
}

// synchronise and require an accepted most recent push
dv_status ready(dv_ctx *c) {
    if (!c) return DV_ERR_ARG;
    if (!c->pushed) return fail(c, DV_ERR_STATE, "no frame has been pushed");
    (void)hipSetDevice(c->device);
    dv_status s = sync_state(c);
    if (s != DV_OK) return s;
    if (c->h_frame->status != 0) return fail(c, (dv_status)c->h_frame->status, "most recent frame was rejected (capacity)");
    return DV_OK;
}

}  // namespace

dv_status check_config(const dv_config *cfg) { return check_cfg(cfg); }

dv_status fail_global(dv_status s, const char *msg) { return fail(nullptr, s, msg); }

Bufs table_base(const dv_config &cfg) {
    Bufs B;
    std::memset(&B, 0, sizeof(B));
    B.lx = cfg.lx;
    B.ly = cfg.ly;
    B.ntx = (B.lx + DV_TILE - 1) / DV_TILE;
    B.nty = (B.ly + DV_TILE - 1) / DV_TILE;
    B.thr = cfg.threshold;
    B.phase = cfg.phase;
    B.conn = cfg.connectivity;
    B.kmax = cfg.max_components;
    B.maxdeg = cfg.max_degree;
    B.ncells = B.ntx * B.nty;
    B.keep_maps = (cfg.flags & DV_KEEP_MAPS) ? 1 : 0;
    B.classify = (cfg.flags & DV_CLASSIFY) ? 1 : 0;
    B.open_x = (cfg.flags & DV_OPEN_X) ? 1 : 0;
    B.open_y = (cfg.flags & DV_OPEN_Y) ? 1 : 0;
    B.weighted = (cfg.flags & DV_WEIGHTED) ? 1 : 0;
    return B;
}

void place_slot(Carve &cv, Bufs &b) {
    const size_t N = (size_t)b.lx * b.ly, tiles = (size_t)b.ncells, K = (size_t)b.kmax;
    const size_t segs = (size_t)b.ly * b.ntx;
    b.parent = cv.take<int32_t>(N);
    b.bpc = cv.take<uint16_t>(tiles * DV_BORDER);
    b.lab16 = cv.take<uint16_t>(tiles * DV_TILE_SITES);
    b.pieces = cv.take<uint16_t>(tiles * DV_TILE_SITES);
    b.prec = cv.take<int2>(tiles * (DV_TILE_SITES / 2));
    b.npieces = cv.take<int32_t>(tiles);
    b.seg_mask = cv.take<uint32_t>(segs);
    b.seg_prefix = cv.take<int32_t>(segs);
    b.band_sum = cv.take<int32_t>(b.nty);
    b.band_pre = cv.take<int32_t>(b.nty);
    b.acc_x = cv.take<long long>(K);
    b.acc_y = cv.take<long long>(K);
    b.acc_w = cv.take<long long>(K);
    b.acc_n = cv.take<int32_t>(K);
    b.acc_amb = cv.take<int32_t>(K);
    b.acc_root = cv.take<int32_t>(K);
    b.cell_count = cv.take<int32_t>(tiles);
    b.cell_start = cv.take<int32_t>(tiles + 1);
    b.cell_items = cv.take<int32_t>(K);
    b.cell_q = cv.take<int2>(K);
    b.comp_cell = cv.take<int32_t>(K);
    b.comp_slot = cv.take<int32_t>(K);
    b.tpairs = cv.take<int2>(tiles * DV_TILE_PAIRS);
    b.tpair_n = cv.take<int32_t>(tiles);
    b.cnt = cv.take<int32_t>(K);
    b.inv = cv.take<int32_t>(K);
    b.fs = cv.take<FrameState>(1);
    place_comp(cv, b.cur, K, b.maxdeg);
    b.phi = cv.take<int32_t>(K);
    b.trigger = cv.take<int32_t>(K);
    b.nb = cv.take<int32_t>(K);
    b.na = cv.take<int32_t>(K);
    b.ob = cv.take<int32_t>(K);
    b.oa = cv.take<int32_t>(K);
    b.act = cv.take<int32_t>(K);
    b.ecnt = cv.take<int32_t>(K);
    b.ebnd = cv.take<int32_t>(K);
    b.stage = cv.take<int32_t>(K * b.maxdeg * 12);
    b.labels = b.keep_maps ? cv.take<int32_t>(N) : nullptr;
    b.owner = b.keep_maps ? cv.take<int32_t>(N) : nullptr;
}

void place_shared(Carve &cv, Bufs &B, int page_frames) {
    const size_t K = (size_t)B.kmax;
    B.st = cv.take<SeqState>(1);
    place_comp(cv, B.past[0], K, B.maxdeg);
    place_comp(cv, B.past[1], K, B.maxdeg);
    // a frame has at most K_max * max_degree flips (breaking ones are couples of
    // the past rows, arising ones of the now rows, each row holding max_degree)
    for (int p = 0; p < 2; ++p) B.pg_flips[p] = cv.take<int32_t>((size_t)page_frames * K * B.maxdeg * 6);
}

extern "C" {

// The configuration with its defaults filled in (row length a multiple of
// four: row slots are read four at a time).
static dv_config normalised(const dv_config &in) {
    dv_config cfg = in;
    if (cfg.max_degree == 0) cfg.max_degree = 48;
    cfg.max_degree = (cfg.max_degree + 3) & ~3;
    if (cfg.max_batch == 0) cfg.max_batch = DV_DEFAULT_BATCH;
    return cfg;
}

// Every device buffer of a context in one region: measured (a Carve with no
// base), then placed.  c->cfg, c->batch and c->pg_cap are set; B is the
// shared part of the slot table.
static void layout_ctx(Carve &cv, dv_ctx *c, Bufs &B) {
    const size_t N = (size_t)B.lx * B.ly, K = (size_t)B.kmax;
    place_shared(cv, B, c->pg_cap);
    c->d_tab = cv.take<Bufs>(DV_MAX_BATCH);
    c->d_edge_scratch = cv.take<int32_t>(2 * K);
    c->d_edge_ab = cv.take<int32_t>(K * B.maxdeg);
    c->d_edge_total = cv.take<int32_t>(1);
    // one obstacle mask for every slot (no obstacle until set)
    uint8_t *obst = (c->cfg.flags & DV_OBSTACLES) ? cv.take<uint8_t>(N) : nullptr;
    B.obst = obst;
    c->d_obst = obst;
    for (int k = 0; k < c->batch; ++k) {
        c->h_tab[k] = B;
        place_slot(cv, c->h_tab[k]);
    }
}

dv_status dv_device_bytes(const dv_config *cfg_in, uint64_t *bytes) {
    if (!bytes) return fail(nullptr, DV_ERR_ARG, "bytes is NULL");
    *bytes = 0;
    dv_status s = check_cfg(cfg_in);
    if (s != DV_OK) return s;
    std::unique_ptr<dv_ctx> c(new dv_ctx());
    c->cfg = normalised(*cfg_in);
    c->batch = c->cfg.max_batch;
    c->pg_cap = std::max(c->batch, 8);
    Bufs B = table_base(c->cfg);
    Carve measure;
    layout_ctx(measure, c.get(), B);
    *bytes = (uint64_t)measure.off;
    return DV_OK;
}

dv_status dv_create(const dv_config *cfg_in, void *hip_stream, dv_ctx **out) {
    if (!out) return fail(nullptr, DV_ERR_ARG, "out is NULL");
    *out = nullptr;
    dv_status s = check_cfg(cfg_in);
    if (s != DV_OK) return s;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
        return fail(nullptr, DV_ERR_DEVICE, "no HIP device");
    if (cfg_in->device < 0 || cfg_in->device >= ndev)
        return fail(nullptr, DV_ERR_ARG, "device ordinal out of range");

    dv_ctx *c = new dv_ctx();
    c->cfg = normalised(*cfg_in);
    c->batch = c->cfg.max_batch;
    c->device = c->cfg.device;
    c->npending = 0;
    c->last = 0;
    c->h_state = nullptr;
    c->h_frame = nullptr;
    c->d_tab = nullptr;
    c->d_obst = nullptr;
    c->region = nullptr;
    c->keep_results = (c->cfg.flags & DV_KEEP_RESULTS) != 0;
    c->pg_cap = std::max(c->batch, 8);
    c->h_pg[0] = c->h_pg[1] = nullptr;
    c->d_pgf[0] = c->d_pgf[1] = nullptr;
    c->cur_pg = 0;
    c->pg_n[0] = c->pg_n[1] = c->pg_rd[0] = c->pg_rd[1] = 0;
    c->last_pg = c->last_pos = 0;
    c->sp_head_info = c->sp_head_flips = 0;
    c->copy_stream = nullptr;
    if (hipSetDevice(c->device) != hipSuccess) {
        delete c;
        return fail(nullptr, DV_ERR_DEVICE, "hipSetDevice failed");
    }
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
        c->own_stream = false;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return fail(nullptr, DV_ERR_DEVICE, "stream creation failed");
        }
        c->own_stream = true;
    }

    // shared part of the slot table
    Bufs B = table_base(c->cfg);
    const size_t N = (size_t)B.lx * B.ly, K = (size_t)B.kmax;
    Carve measure;
    {
        Bufs Bm = B;
        layout_ctx(measure, c, Bm);
    }
    bool ok = hipMalloc(&c->region, measure.off) == hipSuccess;
    if (ok) {
        Carve cv;
        cv.base = static_cast<char *>(c->region);
        layout_ctx(cv, c, B);
    }
    uint8_t *obst = c->d_obst;
    // results-page records: pinned host memory that the device writes
    for (int p = 0; ok && p < 2; ++p) {
        ok = hipHostMalloc((void **)&c->h_pg[p], sizeof(FrameOut) * DV_MAX_BATCH,
                           hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
             hipHostGetDevicePointer((void **)&B.pg_info[p], c->h_pg[p], 0) == hipSuccess;
        if (ok) {
            std::memset(c->h_pg[p], 0, sizeof(FrameOut) * DV_MAX_BATCH);
            c->d_pgf[p] = B.pg_flips[p];
        }
    }
    for (int k = 0; ok && k < c->batch; ++k) {
        c->h_tab[k].pg_info[0] = B.pg_info[0];
        c->h_tab[k].pg_info[1] = B.pg_info[1];
    }
    if (ok) ok = hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking) == hipSuccess;
    if (ok && (hipHostMalloc((void **)&c->h_state, sizeof(SeqState)) != hipSuccess ||
               hipHostMalloc((void **)&c->h_frame, sizeof(FrameState)) != hipSuccess))
        ok = false;
    if (!ok) {
        release(c);
        delete c;
        return fail(nullptr, DV_ERR_NOMEM, "device allocation failed");
    }
    // initial contents: slot table, zero accumulators and headers, empty rows
    hipStream_t s0 = c->stream;
    bool z = hipMemcpyAsync(c->d_tab, c->h_tab, sizeof(Bufs) * c->batch, hipMemcpyHostToDevice, s0) ==
                 hipSuccess &&
             hipMemsetAsync(B.st, 0, sizeof(SeqState), s0) == hipSuccess &&
             (!obst || hipMemsetAsync(obst, 0, N, s0) == hipSuccess);
    for (int b = 0; z && b < 2; ++b)
        z = hipMemsetD32Async((hipDeviceptr_t)B.past[b].adj, DV_EMPTY, K * B.maxdeg, s0) == hipSuccess;
    for (int k = 0; z && k < c->batch; ++k) {
        const Bufs &b = c->h_tab[k];
        z = hipMemsetAsync(b.acc_x, 0, K * sizeof(long long), s0) == hipSuccess &&
            hipMemsetAsync(b.acc_y, 0, K * sizeof(long long), s0) == hipSuccess &&
            hipMemsetAsync(b.acc_w, 0, K * sizeof(long long), s0) == hipSuccess &&
            hipMemsetAsync(b.acc_n, 0, K * sizeof(int), s0) == hipSuccess &&
            hipMemsetAsync(b.acc_amb, 0, K * sizeof(int), s0) == hipSuccess &&
            hipMemsetAsync(b.fs, 0, sizeof(FrameState), s0) == hipSuccess &&
            hipMemsetD32Async((hipDeviceptr_t)b.cur.adj, DV_EMPTY, K * B.maxdeg, s0) == hipSuccess;
    }
    if (!z || hipStreamSynchronize(s0) != hipSuccess) {
        release(c);
        delete c;
        return fail(nullptr, DV_ERR_DEVICE, "device initialisation failed");
    }
    c->pushed = false;
    *out = c;
    return DV_OK;
}

dv_status dv_push_frame(dv_ctx *c, const float *field_device) {
    if (!c) return DV_ERR_ARG;
    if (!field_device) return fail(c, DV_ERR_ARG, "field is NULL");
    (void)hipSetDevice(c->device);
    c->pending.p[c->npending++] = field_device;
    c->pushed = true;
    if (c->npending == c->batch) return flush(c);
    return DV_OK;
}

dv_status dv_sync(dv_ctx *c) {
    if (!c) return DV_ERR_ARG;
    (void)hipSetDevice(c->device);
    return drain(c);
}

dv_status dv_set_obstacles(dv_ctx *c, const uint8_t *mask, int32_t mask_on_device) {
    if (!c) return DV_ERR_ARG;
    if (!c->d_obst) return fail(c, DV_ERR_STATE, "context made without DV_OBSTACLES");
    (void)hipSetDevice(c->device);
    // frames pushed before this call keep the mask they were pushed with
    dv_status s = flush(c);
    if (s != DV_OK) return s;
    const size_t N = (size_t)c->cfg.lx * c->cfg.ly;
    hipError_t e;
    if (!mask) e = hipMemsetAsync(c->d_obst, 0, N, c->stream);
    else
        e = hipMemcpyAsync(c->d_obst, mask, N, mask_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           c->stream);
    if (e != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(c, DV_ERR_DEVICE, std::string("mask copy failed: ") + hipGetErrorString(e));
    return DV_OK;
}

dv_status dv_get_info(dv_ctx *c, dv_frame_info *info) {
    if (!c || !info) return DV_ERR_ARG;
    if (!c->pushed) return fail(c, DV_ERR_STATE, "no frame has been pushed");
    (void)hipSetDevice(c->device);
    dv_status s = sync_state(c);
    if (s != DV_OK) return s;
    const SeqState &h = *c->h_state;
    const FrameState &f = *c->h_frame;
    dv_frame_info fi;
    std::memset(&fi, 0, sizeof(fi));
    fi.frame = h.frame;
    fi.status = f.status;
    fi.n_components = f.K_now;
    fi.n_edges = f.status == 0 ? f.E_now : 0;
    fi.n_flips = f.n_flips;
    fi.n_breaking = f.n_break;
    fi.n_excluded_past = f.n_excl_past;
    fi.n_excluded_now = f.n_excl_now;
    fi.n_ambiguous_centroids = f.n_amb;
    fi.global_trigger = (uint32_t)f.global_trigger;
    *info = fi;
    return (dv_status)f.status;
}

dv_status dv_get_flips(dv_ctx *c, dv_flip *host_out, int32_t capacity, int32_t *n_out) {
    if (!c || !n_out || capacity < 0) return DV_ERR_ARG;
    dv_status s = ready(c);
    if (s != DV_OK) return s;
    const FrameOut &r = c->h_pg[c->last_pg][c->last_pos];
    const int n = r.n_flips;
    *n_out = n;
    if (n > capacity) return fail(c, DV_ERR_CAPACITY, "flip buffer too small");
    if (n > 0) {
        if (!host_out) return fail(c, DV_ERR_ARG, "host_out is NULL");
        if (hipMemcpy(host_out, c->d_pgf[c->last_pg] + (size_t)6 * r.flip_off, (size_t)n * sizeof(dv_flip),
                      hipMemcpyDeviceToHost) != hipSuccess)
            return fail(c, DV_ERR_DEVICE, "copy failed");
    }
    return DV_OK;
}

}  // extern "C"

namespace {

// Unread frames whose launches are complete (all of them after a drain):
// the spilled ones, then those of the older page, then the current page's.
struct Avail {
    int spill;           // frames in the spill store
    int pages[2];        // page order: older first
    int end[2];          // readable end of each page (frames [pg_rd, end))
};

Avail available(dv_ctx *c, bool all_done) {
    Avail a;
    a.spill = (int)(c->sp_info.size() - c->sp_head_info);
    a.pages[0] = 1 - c->cur_pg;
    a.pages[1] = c->cur_pg;
    a.end[0] = a.end[1] = 0;
    int done[2] = {c->pg_rd[0], c->pg_rd[1]};
    if (all_done) {
        done[0] = c->pg_n[0];
        done[1] = c->pg_n[1];
    } else {
        for (const PageLaunch &L : c->inflight) {
            if (hipEventQuery(L.ev->e) != hipSuccess) break;   // later launches are later on the stream
            done[L.page] = std::max(done[L.page], L.end);
        }
    }
    for (int k = 0; k < 2; ++k) a.end[k] = std::max(done[a.pages[k]], c->pg_rd[a.pages[k]]);
    return a;
}

dv_status results_prologue(dv_ctx *c, int32_t wait) {
    if (!c->keep_results) return fail(c, DV_ERR_STATE, "context made without DV_KEEP_RESULTS");
    (void)hipSetDevice(c->device);
    if (wait) return drain(c);
    return DV_OK;
}

}  // namespace

extern "C" {

dv_status dv_results_ready(dv_ctx *c, int32_t wait, int32_t *n_frames, int32_t *n_flips) {
    if (!c || !n_frames || !n_flips) return DV_ERR_ARG;
    dv_status s = results_prologue(c, wait);
    if (s != DV_OK) return s;
    const Avail a = available(c, wait != 0);
    long long nf = a.spill, nfl = (long long)(c->sp_flips.size() - c->sp_head_flips);
    for (int k = 0; k < 2; ++k) {
        const int p = a.pages[k];
        for (int i = c->pg_rd[p]; i < a.end[k]; ++i) nfl += c->h_pg[p][i].n_flips;
        nf += a.end[k] - c->pg_rd[p];
    }
    if (nfl > INT32_MAX) return fail(c, DV_ERR_CAPACITY, "more than 2^31 flips unread");
    *n_frames = (int32_t)nf;
    *n_flips = (int32_t)nfl;
    return DV_OK;
}

dv_status dv_get_results(dv_ctx *c, int32_t wait, dv_frame_info *infos, int32_t cap_frames,
                         int32_t *n_frames, dv_flip *flips, int32_t cap_flips, int32_t *n_flips) {
    if (!c || !n_frames || !n_flips || cap_frames < 0 || cap_flips < 0) return DV_ERR_ARG;
    if ((cap_frames > 0 && !infos) || (cap_flips > 0 && !flips)) return DV_ERR_ARG;
    *n_frames = 0;
    *n_flips = 0;
    dv_status s = results_prologue(c, wait);
    if (s != DV_OK) return s;
    const Avail a = available(c, wait != 0);
    int nf = 0, nfl = 0;
    bool all = true;
    // spilled frames first (oldest)
    while (c->sp_head_info < c->sp_info.size()) {
        const dv_frame_info &fi = c->sp_info[c->sp_head_info];
        if (nf + 1 > cap_frames || (long long)nfl + fi.n_flips > cap_flips) {
            all = false;
            break;
        }
        infos[nf++] = fi;
        if (fi.n_flips > 0)
            std::memcpy(flips + nfl, c->sp_flips.data() + c->sp_head_flips, (size_t)fi.n_flips * sizeof(dv_flip));
        nfl += fi.n_flips;
        c->sp_head_flips += fi.n_flips;
        ++c->sp_head_info;
    }
    if (c->sp_head_info == c->sp_info.size()) {
        c->sp_info.clear();
        c->sp_flips.clear();
        c->sp_head_info = c->sp_head_flips = 0;
    }
    for (int k = 0; all && k < 2; ++k) {
        const int p = a.pages[k];
        const int a0 = c->pg_rd[p];
        int b = a0, add = 0;
        while (b < a.end[k]) {
            const int f = c->h_pg[p][b].n_flips;
            if (nf + (b - a0) + 1 > cap_frames || (long long)nfl + add + f > cap_flips) {
                all = false;
                break;
            }
            add += f;
            ++b;
        }
        if (b > a0) {
            int got = 0;
            s = read_frames(c, p, a0, b, infos + nf, flips + nfl, &got);
            if (s != DV_OK) return s;
            nf += b - a0;
            nfl += got;
            c->pg_rd[p] = b;
        }
    }
    // launches whose frames have all been read
    while (!c->inflight.empty() && c->inflight.front().end <= c->pg_rd[c->inflight.front().page])
        c->inflight.pop_front();
    *n_frames = nf;
    *n_flips = nfl;
    if (!all) return fail(c, DV_ERR_CAPACITY, "result buffers too small for every ready frame");
    return DV_OK;
}

dv_status dv_get_labels(dv_ctx *c, int32_t *host_out) {
    if (!c || !host_out) return DV_ERR_ARG;
    if (!(c->cfg.flags & DV_KEEP_MAPS)) return fail(c, DV_ERR_STATE, "maps not kept (DV_KEEP_MAPS)");
    dv_status s = ready(c);
    if (s != DV_OK) return s;
    const Bufs &B = c->h_tab[c->last];
    const size_t N = (size_t)B.lx * B.ly;
    if (hipMemcpy(host_out, B.labels, N * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, DV_ERR_DEVICE, "copy failed");
    return DV_OK;
}

dv_status dv_get_owner(dv_ctx *c, int32_t *host_out) {
    if (!c || !host_out) return DV_ERR_ARG;
    if (!(c->cfg.flags & DV_KEEP_MAPS)) return fail(c, DV_ERR_STATE, "maps not kept (DV_KEEP_MAPS)");
    dv_status s = ready(c);
    if (s != DV_OK) return s;
    const Bufs &B = c->h_tab[c->last];
    const size_t N = (size_t)B.lx * B.ly;
    if (hipMemcpy(host_out, B.owner, N * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, DV_ERR_DEVICE, "copy failed");
    return DV_OK;
}

dv_status dv_get_components(dv_ctx *c, int32_t *q8_xy, double *xy, int32_t *size, int32_t capacity,
                            int32_t *n_out) {
    if (!c || !n_out || capacity < 0) return DV_ERR_ARG;
    dv_status s = ready(c);
    if (s != DV_OK) return s;
    const SeqState &h = *c->h_state;
    const int K = h.K[h.sel];
    *n_out = K;
    if (K > capacity) return fail(c, DV_ERR_CAPACITY, "component buffer too small");
    if (K == 0) return DV_OK;
    const CompBuf &C = c->h_tab[0].past[h.sel];
    std::vector<int32_t> qx(K), qy(K);
    std::vector<double> fx(K), fy(K);
    bool ok = hipMemcpy(qx.data(), C.qx, K * 4, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(qy.data(), C.qy, K * 4, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(fx.data(), C.fx, K * 8, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(fy.data(), C.fy, K * 8, hipMemcpyDeviceToHost) == hipSuccess;
    if (ok && size) ok = hipMemcpy(size, C.n, K * 4, hipMemcpyDeviceToHost) == hipSuccess;
    if (!ok) return fail(c, DV_ERR_DEVICE, "copy failed");
    for (int k = 0; k < K; ++k) {
        if (q8_xy) { q8_xy[2 * k] = qx[k]; q8_xy[2 * k + 1] = qy[k]; }
        if (xy) { xy[2 * k] = fx[k]; xy[2 * k + 1] = fy[k]; }
    }
    return DV_OK;
}

dv_status dv_get_edges(dv_ctx *c, int32_t *ab, int32_t capacity, int32_t *n_out) {
    if (!c || !n_out || capacity < 0) return DV_ERR_ARG;
    dv_status s = ready(c);
    if (s != DV_OK) return s;
    launch_edge_list(c->h_tab[0], c->d_tab, c->d_edge_ab, c->d_edge_total, c->d_edge_scratch, c->stream);
    int32_t E = 0;
    if (hipMemcpyAsync(&E, c->d_edge_total, 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(c, DV_ERR_DEVICE, "edge list failed");
    *n_out = E;
    if (E > capacity) return fail(c, DV_ERR_CAPACITY, "edge buffer too small");
    if (E > 0) {
        if (!ab) return fail(c, DV_ERR_ARG, "ab is NULL");
        if (hipMemcpy(ab, c->d_edge_ab, (size_t)E * 8, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(c, DV_ERR_DEVICE, "copy failed");
    }
    return DV_OK;
}

dv_status dv_get_matching(dv_ctx *c, int32_t *phi, int32_t capacity, int32_t *n_out) {
    if (!c || !n_out || capacity < 0) return DV_ERR_ARG;
    dv_status s = ready(c);
    if (s != DV_OK) return s;
    const int KP = c->h_frame->K_past;
    *n_out = KP;
    if (KP > capacity) return fail(c, DV_ERR_CAPACITY, "matching buffer too small");
    if (KP == 0) return DV_OK;
    if (!phi) return fail(c, DV_ERR_ARG, "phi is NULL");
    // Phi with dropped past points as -1, written to scratch on the device
    launch_phi_out(c->h_tab[0], c->d_tab, c->last, c->d_edge_ab, c->stream);
    if (hipMemcpyAsync(phi, c->d_edge_ab, (size_t)KP * 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(c, DV_ERR_DEVICE, "copy failed");
    return DV_OK;
}

void dv_destroy(dv_ctx *c) {
    if (!c) return;
    release(c);
    delete c;
}

static const char *const STAGE_NAMES[ST_COUNT] = {
    "tile_ccl", "merge", "resolve", "relabel", "finalize", "owner_edges", "rows", "match", "diff",
    "events", "place"};

const char *dv_stage_name(int32_t stage) {
    return (stage >= 0 && stage < ST_COUNT) ? STAGE_NAMES[stage] : nullptr;
}

dv_status dv_set_profile(dv_ctx *c, int32_t stage, int32_t capacity) {
    if (!c) return DV_ERR_ARG;
    if (stage < -1 || stage >= ST_COUNT || (stage >= 0 && (capacity < 1 || capacity > (1 << 20))))
        return fail(c, DV_ERR_ARG, "bad stage or capacity");
    (void)hipSetDevice(c->device);
    dv_status ds = drain(c);
    if (ds != DV_OK) return ds;
    drop_events(c);
    if (stage < 0) return DV_OK;
    c->prof.ev = new hipEvent_t[2 * (size_t)capacity];
    for (int i = 0; i < 2 * capacity; ++i) {
        if (hipEventCreate(&c->prof.ev[i]) != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(c->prof.ev[j]);
            delete[] c->prof.ev;
            c->prof = Prof();
            return fail(c, DV_ERR_DEVICE, "event creation failed");
        }
    }
    c->prof.cap = capacity;
    c->prof.stage = stage;
    return DV_OK;
}

dv_status dv_get_profile(dv_ctx *c, double *total_ms, int32_t *launches) {
    if (!c || !total_ms || !launches) return DV_ERR_ARG;
    (void)hipSetDevice(c->device);
    dv_status ds = drain(c);
    if (ds != DV_OK) return ds;
    double tot = 0.0;
    for (int i = 0; i < c->prof.used; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->prof.ev[2 * i], c->prof.ev[2 * i + 1]) != hipSuccess)
            return fail(c, DV_ERR_DEVICE, "event query failed");
        tot += ms;
    }
    *total_ms = tot;
    *launches = c->prof.used;
    c->prof.used = 0;
    return DV_OK;
}

// ---- groups -----------------------------------------------------------------

struct dv_group {
    int n;
    int device;
    hipStream_t stream;
    dv_ctx *m[DV_MAX_ENTRIES];
    Bufs h_tab[DV_MAX_ENTRIES];  // members' slot 0, sequence i for member i
    Bufs *d_tab;
    Prof prof;                   // never enabled
};

dv_status dv_group_create(dv_ctx *const *members, int32_t n, dv_group **out) {
    if (!out) return fail(nullptr, DV_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!members || n < 1 || n > DV_MAX_ENTRIES)
        return fail(nullptr, DV_ERR_ARG, "a group has 1 .. 64 members");
    for (int i = 0; i < n; ++i) {
        if (!members[i]) return fail(nullptr, DV_ERR_ARG, "member is NULL");
        if (members[i]->device != members[0]->device || members[i]->stream != members[0]->stream)
            return fail(nullptr, DV_ERR_ARG, "members must share the device and the stream");
    }
    dv_group *g = new dv_group();
    g->n = n;
    g->device = members[0]->device;
    g->stream = members[0]->stream;
    g->d_tab = nullptr;
    (void)hipSetDevice(g->device);
    for (int i = 0; i < n; ++i) {
        g->m[i] = members[i];
        g->h_tab[i] = members[i]->h_tab[0];
        g->h_tab[i].seq = i;
    }
    const bool ok = hipMalloc(&g->d_tab, sizeof(Bufs) * n) == hipSuccess &&
                    hipMemcpyAsync(g->d_tab, g->h_tab, sizeof(Bufs) * n, hipMemcpyHostToDevice,
                                   g->stream) == hipSuccess &&
                    hipStreamSynchronize(g->stream) == hipSuccess;
    if (!ok) {
        dv_group_destroy(g);
        return fail(nullptr, DV_ERR_NOMEM, "group allocation failed");
    }
    *out = g;
    return DV_OK;
}

dv_status dv_group_push_some(dv_group *g, const int32_t *members, const float *const *fields,
                             int32_t n) {
    if (!g || !members || !fields || n < 1 || n > g->n) return DV_ERR_ARG;
    bool seen[DV_MAX_ENTRIES] = {false};
    for (int i = 0; i < n; ++i) {
        const int k = members[i];
        if (k < 0 || k >= g->n || seen[k]) return DV_ERR_ARG;
        seen[k] = true;
        if (!fields[i]) return fail(g->m[k], DV_ERR_ARG, "field is NULL");
    }
    (void)hipSetDevice(g->device);
    Fields F;
    std::memset(&F, 0, sizeof(F));
    Batch G;
    std::memset(&G, 0, sizeof(G));
    G.D = g->d_tab;
    G.n = n;
    bool alike = true;
    bool keep = false;
    for (int i = 0; i < n; ++i) {
        const int k = members[i];
        dv_status s = flush(g->m[k]);
        if (s == DV_OK) s = take_page(g->m[k], 1, &G.pslot[i]);
        if (s != DV_OK) return s;
        keep = keep || g->m[k]->keep_results;
        const Bufs &b = g->h_tab[k];
        F.p[i] = fields[i];
        G.idx[i] = k;
        G.tbase[i + 1] = G.tbase[i] + b.ncells;
        G.bbase[i + 1] = G.bbase[i] + b.nty;
        G.kmax = std::max(G.kmax, b.kmax);
        G.nty = std::max(G.nty, b.nty);
        G.classify |= b.classify;
        G.geom |= (b.open_x | b.open_y | (b.obst != nullptr)) ? 1 : 0;
        G.weighted |= b.weighted;
        alike = alike && b.ncells == g->h_tab[members[0]].ncells && b.nty == g->h_tab[members[0]].nty;
    }
    G.tiles = G.tbase[n];
    G.bands = G.bbase[n];
    G.tpe = alike ? g->h_tab[members[0]].ncells : 0;
    G.bpe = alike ? g->h_tab[members[0]].nty : 0;
    launch_label(G, F, g->stream, g->prof);
    launch_voronoi(G, g->stream, g->prof);
    launch_compare(G, g->stream, g->prof);
    const hipError_t e = hipGetLastError();
    EvRef ev;
    dv_status rs = DV_OK;
    if (e == hipSuccess && keep) rs = record_launch(g->m[members[0]], g->stream, &ev);
    for (int i = 0; i < n; ++i) {
        dv_ctx *c = g->m[members[i]];
        c->last = 0;
        c->pushed = true;
        if (e != hipSuccess) fail(c, DV_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
        else note_launch(c, 1, ev);
    }
    if (e != hipSuccess) return DV_ERR_DEVICE;
    return rs;
}

dv_status dv_group_push(dv_group *g, const float *const *fields) {
    if (!g || !fields) return DV_ERR_ARG;
    int32_t all[DV_MAX_ENTRIES];
    for (int i = 0; i < g->n; ++i) all[i] = i;
    return dv_group_push_some(g, all, fields, g->n);
}

void dv_group_destroy(dv_group *g) {
    if (!g) return;
    (void)hipSetDevice(g->device);
    (void)hipStreamSynchronize(g->stream);
    if (g->d_tab) (void)hipFree(g->d_tab);
    delete g;
}

const char *dv_status_str(dv_status s) {
    switch (s) {
        case DV_OK: return "ok";
        case DV_ERR_ARG: return "invalid argument";
        case DV_ERR_CAPACITY: return "capacity exceeded";
        case DV_ERR_NOMEM: return "out of memory";
        case DV_ERR_DEVICE: return "device error";
        case DV_ERR_STATE: return "invalid state";
        case DV_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

const char *dv_last_error(const dv_ctx *c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
