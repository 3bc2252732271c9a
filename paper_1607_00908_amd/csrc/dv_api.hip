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
#include <string>
#include <vector>

#include "dv.h"
#include "dv_internal.h"

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
    std::vector<void *> allocs;
    SeqState *h_state;       // pinned mirrors of the headers
    FrameState *h_frame;
    int32_t *d_edge_scratch; // [2 * K_max] for the couple-list getter
    int32_t *d_edge_ab;      // [K_max * max_degree] pairs
    int32_t *d_edge_total;
    uint8_t *d_obst;         // obstacle mask (DV_OBSTACLES), else null
    bool pushed;
    Prof prof;
    std::string err;
};

namespace {

thread_local std::string g_create_error;

dv_status fail(dv_ctx *c, dv_status s, const std::string &msg) {
    if (c) c->err = msg;
    else g_create_error = msg;
    return s;
}

template <class T>
bool dalloc(dv_ctx *c, T **p, size_t count) {
    void *q = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) return false;
    c->allocs.push_back(q);
    *p = static_cast<T *>(q);
    return true;
}

void drop_events(dv_ctx *c) {
    if (c->prof.ev) {
        for (int i = 0; i < 2 * c->prof.cap; ++i) (void)hipEventDestroy(c->prof.ev[i]);
        delete[] c->prof.ev;
    }
    c->prof = Prof();
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
    for (int i = 0; i < n; ++i) G.idx[i] = i;
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
    launch_label(G, c->pending, c->stream, c->prof);
    launch_voronoi(G, c->stream, c->prof);
    launch_compare(G, c->stream, c->prof);
    c->npending = 0;
    c->last = n - 1;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, DV_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
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
    for (void *p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    if (c->h_state) (void)hipHostFree(c->h_state);
    if (c->h_frame) (void)hipHostFree(c->h_frame);
    c->h_state = nullptr;
    c->h_frame = nullptr;
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
    if (cfg->flags & ~(DV_KEEP_MAPS | DV_CLASSIFY | DV_OBSTACLES | DV_OPEN_X | DV_OPEN_Y))
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

extern "C" {

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
    c->cfg = *cfg_in;
    if (c->cfg.max_degree == 0) c->cfg.max_degree = 48;
    // row slots are read four at a time
    c->cfg.max_degree = (c->cfg.max_degree + 3) & ~3;
    if (c->cfg.max_batch == 0) c->cfg.max_batch = DV_DEFAULT_BATCH;
    c->batch = c->cfg.max_batch;
    c->device = c->cfg.device;
    c->npending = 0;
    c->last = 0;
    c->h_state = nullptr;
    c->h_frame = nullptr;
    c->d_tab = nullptr;
    c->d_obst = nullptr;
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
    Bufs B;
    std::memset(&B, 0, sizeof(B));
    B.lx = c->cfg.lx;
    B.ly = c->cfg.ly;
    B.ntx = (B.lx + DV_TILE - 1) / DV_TILE;
    B.nty = (B.ly + DV_TILE - 1) / DV_TILE;
    B.thr = c->cfg.threshold;
    B.phase = c->cfg.phase;
    B.conn = c->cfg.connectivity;
    B.kmax = c->cfg.max_components;
    B.maxdeg = c->cfg.max_degree;
    B.ncells = B.ntx * B.nty;
    B.keep_maps = (c->cfg.flags & DV_KEEP_MAPS) ? 1 : 0;
    B.classify = (c->cfg.flags & DV_CLASSIFY) ? 1 : 0;
    B.open_x = (c->cfg.flags & DV_OPEN_X) ? 1 : 0;
    B.open_y = (c->cfg.flags & DV_OPEN_Y) ? 1 : 0;
    const size_t N = (size_t)B.lx * B.ly, tiles = (size_t)B.ncells, K = (size_t)B.kmax;
    const size_t segs = (size_t)B.ly * B.ntx;
    auto comp_alloc = [&](CompBuf &C) {
        return dalloc(c, &C.qx, K) && dalloc(c, &C.qy, K) && dalloc(c, &C.fx, K) &&
               dalloc(c, &C.fy, K) && dalloc(c, &C.n, K) && dalloc(c, &C.root, K) &&
               dalloc(c, &C.amb, K) && dalloc(c, &C.adj, K * B.maxdeg);
    };
    bool ok = dalloc(c, &B.st, 1) && comp_alloc(B.past[0]) && comp_alloc(B.past[1]) &&
              dalloc(c, &c->d_tab, DV_MAX_BATCH) && dalloc(c, &c->d_edge_scratch, 2 * K) &&
              dalloc(c, &c->d_edge_ab, K * B.maxdeg) && dalloc(c, &c->d_edge_total, 1);
    uint8_t *obst = nullptr;   // one mask for every slot (no obstacle until set)
    if (ok && (c->cfg.flags & DV_OBSTACLES)) {
        ok = dalloc(c, &obst, N);
        B.obst = obst;
        c->d_obst = obst;
    }
    // per-slot buffers
    for (int k = 0; ok && k < c->batch; ++k) {
        Bufs &b = c->h_tab[k];
        b = B;
        ok = dalloc(c, &b.parent, N) && dalloc(c, &b.lab16, tiles * DV_TILE_SITES) &&
             dalloc(c, &b.pieces, tiles * DV_TILE_SITES) && dalloc(c, &b.npieces, tiles) &&
             dalloc(c, &b.seg_mask, segs) && dalloc(c, &b.seg_prefix, segs) &&
             dalloc(c, &b.band_sum, (size_t)B.nty) && dalloc(c, &b.acc_x, K) &&
             dalloc(c, &b.acc_y, K) && dalloc(c, &b.acc_n, K) && dalloc(c, &b.acc_amb, K) &&
             dalloc(c, &b.acc_root, K) && dalloc(c, &b.cell_count, tiles) &&
             dalloc(c, &b.cell_start, tiles + 1) && dalloc(c, &b.cell_items, K) &&
             dalloc(c, &b.cell_q, K) && dalloc(c, &b.comp_cell, K) && dalloc(c, &b.comp_slot, K) &&
             dalloc(c, &b.tpairs, tiles * DV_TILE_PAIRS) && dalloc(c, &b.tpair_n, tiles) &&
             dalloc(c, &b.cnt, K) && dalloc(c, &b.inv, K) && dalloc(c, &b.fs, 1) &&
             comp_alloc(b.cur) && dalloc(c, &b.phi, K) && dalloc(c, &b.trigger, K) &&
             dalloc(c, &b.nb, K) && dalloc(c, &b.na, K) && dalloc(c, &b.ob, K) &&
             dalloc(c, &b.oa, K) && dalloc(c, &b.flips, K * B.maxdeg * 6) &&
             dalloc(c, &b.act, K) && dalloc(c, &b.ecnt, K) && dalloc(c, &b.ebnd, K) &&
             dalloc(c, &b.stage, K * B.maxdeg * 12);
        if (ok && B.keep_maps) ok = dalloc(c, &b.labels, N) && dalloc(c, &b.owner, N);
    }
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
    const int n = c->h_frame->n_flips;
    *n_out = n;
    if (n > capacity) return fail(c, DV_ERR_CAPACITY, "flip buffer too small");
    if (n > 0) {
        if (!host_out) return fail(c, DV_ERR_ARG, "host_out is NULL");
        if (hipMemcpy(host_out, c->h_tab[c->last].flips, (size_t)n * sizeof(dv_flip), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(c, DV_ERR_DEVICE, "copy failed");
    }
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
    for (int i = 0; i < n; ++i) {
        const int k = members[i];
        dv_status s = flush(g->m[k]);
        if (s != DV_OK) return s;
        const Bufs &b = g->h_tab[k];
        F.p[i] = fields[i];
        G.idx[i] = k;
        G.tbase[i + 1] = G.tbase[i] + b.ncells;
        G.bbase[i + 1] = G.bbase[i] + b.nty;
        G.kmax = std::max(G.kmax, b.kmax);
        G.nty = std::max(G.nty, b.nty);
        G.classify |= b.classify;
        G.geom |= (b.open_x | b.open_y | (b.obst != nullptr)) ? 1 : 0;
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
    for (int i = 0; i < n; ++i) {
        dv_ctx *c = g->m[members[i]];
        c->last = 0;
        c->pushed = true;
        if (e != hipSuccess) fail(c, DV_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    }
    return e == hipSuccess ? DV_OK : DV_ERR_DEVICE;
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
