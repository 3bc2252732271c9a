// Host side of libdv: the C ABI declared in include/dv.h.
//
// A context owns every device buffer, sized once from the lattice and K_max.
// Frames go through a pipeline of `depth` slots: frame f uses slot f % depth
// for everything up to its Delaunay couples (labelling, centres, colouring),
// enqueued on that slot's stream, so consecutive frames overlap on the
// device.  Its comparison with the last accepted frame (matching, diff,
// commit) runs on one chain stream in frame order.  Events order the work:
//   slot stream  waits for the caller's stream at the push (the field is
//                ready) and for the chain of the slot's previous frame (its
//                buffers are free again);
//   chain        waits for the slot's stage of the frame.
// No host synchronisation happens in a push.  Synchronising calls wait for the
// chain and copy the sequence header (and the requested arrays) back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "dv.h"
#include "dv_internal.h"

#define DV_MAX_DEPTH 4

struct Slot {
    Bufs B;                  // slot buffers + the shared chain buffers
    hipStream_t stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_s1 = nullptr, ev_done = nullptr;
};

struct dv_ctx {
    dv_config cfg;
    int device;
    hipStream_t stream;      // the caller's (or owned) stream: input ordering
    bool own_stream;
    hipStream_t chain;       // comparison chain
    int depth;
    Slot slot[DV_MAX_DEPTH];
    int64_t pushes;          // frames pushed so far
    int last;                // slot of the most recent push
    std::vector<void *> allocs;
    SeqState *h_state;       // pinned mirror of the sequence header
    int32_t *d_edge_scratch; // [2 * K_max] for the couple-list getter
    int32_t *d_edge_ab;      // [K_max * max_degree] pairs
    int32_t *d_edge_total;
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

// wait for every stream of the context
bool drain(dv_ctx *c) {
    bool ok = true;
    for (int k = 0; k < c->depth; ++k)
        if (c->slot[k].stream) ok = hipStreamSynchronize(c->slot[k].stream) == hipSuccess && ok;
    if (c->chain) ok = hipStreamSynchronize(c->chain) == hipSuccess && ok;
    if (c->stream) ok = hipStreamSynchronize(c->stream) == hipSuccess && ok;
    return ok;
}

void release(dv_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)drain(c);
    drop_events(c);
    for (int k = 0; k < DV_MAX_DEPTH; ++k) {
        Slot &S = c->slot[k];
        if (S.ev_in) (void)hipEventDestroy(S.ev_in);
        if (S.ev_s1) (void)hipEventDestroy(S.ev_s1);
        if (S.ev_done) (void)hipEventDestroy(S.ev_done);
        if (S.stream) (void)hipStreamDestroy(S.stream);
        S = Slot();
    }
    if (c->chain) (void)hipStreamDestroy(c->chain);
    c->chain = nullptr;
    for (void *p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    if (c->h_state) (void)hipHostFree(c->h_state);
    c->h_state = nullptr;
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
    if (cfg->flags & ~DV_KEEP_MAPS) return fail(nullptr, DV_ERR_ARG, "unknown flag bits");
    if (cfg->pipeline_depth < 0 || cfg->pipeline_depth > DV_MAX_DEPTH)
        return fail(nullptr, DV_ERR_ARG, "pipeline_depth must be 0 or in [1, 4]");
    return DV_OK;
}

dv_status sync_state(dv_ctx *c) {
    if (!drain(c) ||
        hipMemcpyAsync(c->h_state, c->slot[0].B.st, sizeof(SeqState), hipMemcpyDeviceToHost,
                       c->chain) != hipSuccess ||
        hipStreamSynchronize(c->chain) != hipSuccess)
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
    if (c->h_state->status != 0) return fail(c, (dv_status)c->h_state->status, "most recent frame was rejected (capacity)");
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
    if (c->cfg.pipeline_depth == 0) c->cfg.pipeline_depth = 3;
    c->depth = c->cfg.pipeline_depth;
    c->device = c->cfg.device;
    c->chain = nullptr;
    c->pushes = 0;
    c->last = 0;
    c->h_state = nullptr;
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
    bool ok = hipStreamCreateWithFlags(&c->chain, hipStreamNonBlocking) == hipSuccess;
    for (int k = 0; ok && k < c->depth; ++k) {
        Slot &S = c->slot[k];
        ok = hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&S.ev_in, hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&S.ev_s1, hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&S.ev_done, hipEventDisableTiming) == hipSuccess;
    }
    if (!ok) {
        release(c);
        delete c;
        return fail(nullptr, DV_ERR_DEVICE, "stream or event creation failed");
    }

    // shared part of the buffer table
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
    const size_t N = (size_t)B.lx * B.ly, tiles = (size_t)B.ncells, K = (size_t)B.kmax;
    const size_t segs = (size_t)B.ly * B.ntx;
    auto comp_alloc = [&](CompBuf &C) {
        return dalloc(c, &C.qx, K) && dalloc(c, &C.qy, K) && dalloc(c, &C.fx, K) &&
               dalloc(c, &C.fy, K) && dalloc(c, &C.n, K) && dalloc(c, &C.root, K) &&
               dalloc(c, &C.amb, K) && dalloc(c, &C.adj, K * B.maxdeg);
    };
    ok = dalloc(c, &B.phi, K) && dalloc(c, &B.trigger, K) && dalloc(c, &B.nb, K) &&
         dalloc(c, &B.na, K) && dalloc(c, &B.ob, K) && dalloc(c, &B.oa, K) &&
         dalloc(c, &B.flips, K * B.maxdeg * 6) && dalloc(c, &B.stage, K * B.maxdeg * 12) &&
         dalloc(c, &B.st, 1) && comp_alloc(B.past[0]) && comp_alloc(B.past[1]) &&
         dalloc(c, &c->d_edge_scratch, 2 * K) && dalloc(c, &c->d_edge_ab, K * B.maxdeg) &&
         dalloc(c, &c->d_edge_total, 1);
    // per-slot buffers
    for (int k = 0; ok && k < c->depth; ++k) {
        Bufs &b = c->slot[k].B;
        b = B;
        ok = dalloc(c, &b.parent, N) && dalloc(c, &b.lab16, N) &&
             dalloc(c, &b.pieces, tiles * DV_TILE_SITES) && dalloc(c, &b.npieces, tiles) &&
             dalloc(c, &b.seg_mask, segs) && dalloc(c, &b.seg_prefix, segs) &&
             dalloc(c, &b.band_sum, (size_t)B.nty) && dalloc(c, &b.acc_x, K) &&
             dalloc(c, &b.acc_y, K) && dalloc(c, &b.acc_n, K) && dalloc(c, &b.acc_amb, K) &&
             dalloc(c, &b.acc_root, K) && dalloc(c, &b.cell_count, tiles) &&
             dalloc(c, &b.cell_start, tiles + 1) && dalloc(c, &b.cell_items, K) &&
             dalloc(c, &b.cell_q, K) && dalloc(c, &b.comp_cell, K) && dalloc(c, &b.comp_slot, K) &&
             dalloc(c, &b.cnt, K) && dalloc(c, &b.inv, K) && dalloc(c, &b.fs, 1) &&
             comp_alloc(b.cur);
        if (ok && B.keep_maps) ok = dalloc(c, &b.labels, N) && dalloc(c, &b.owner, N);
    }
    if (ok && hipHostMalloc((void **)&c->h_state, sizeof(SeqState)) != hipSuccess) ok = false;
    if (!ok) {
        release(c);
        delete c;
        return fail(nullptr, DV_ERR_NOMEM, "device allocation failed");
    }
    // initial contents: zero accumulators and headers, empty rows
    hipStream_t s0 = c->chain;
    bool z = hipMemsetAsync(B.st, 0, sizeof(SeqState), s0) == hipSuccess;
    for (int b = 0; z && b < 2; ++b)
        z = hipMemsetD32Async((hipDeviceptr_t)B.past[b].adj, DV_EMPTY, K * B.maxdeg, s0) == hipSuccess;
    for (int k = 0; z && k < c->depth; ++k) {
        const Bufs &b = c->slot[k].B;
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
    const int k = (int)(c->pushes % c->depth);
    Slot &S = c->slot[k];
    S.B.field = field_device;
    bool ok = hipEventRecord(S.ev_in, c->stream) == hipSuccess &&
              hipStreamWaitEvent(S.stream, S.ev_in, 0) == hipSuccess;
    // the slot's previous frame must have left the chain (no-op before its first use)
    if (ok && c->pushes >= c->depth) ok = hipStreamWaitEvent(S.stream, S.ev_done, 0) == hipSuccess;
    if (!ok) return fail(c, DV_ERR_DEVICE, "event ordering failed");
    launch_label(S.B, S.stream, c->prof);
    launch_voronoi(S.B, S.stream, c->prof);
    ok = hipEventRecord(S.ev_s1, S.stream) == hipSuccess &&
         hipStreamWaitEvent(c->chain, S.ev_s1, 0) == hipSuccess;
    if (!ok) return fail(c, DV_ERR_DEVICE, "event ordering failed");
    launch_chain(S.B, c->chain, c->prof);
    if (hipEventRecord(S.ev_done, c->chain) != hipSuccess) return fail(c, DV_ERR_DEVICE, "event record failed");
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, DV_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    c->last = k;
    c->pushes += 1;
    c->pushed = true;
    return DV_OK;
}

dv_status dv_sync(dv_ctx *c) {
    if (!c) return DV_ERR_ARG;
    (void)hipSetDevice(c->device);
    if (!drain(c)) return fail(c, DV_ERR_DEVICE, "stream error");
    return DV_OK;
}

dv_status dv_get_info(dv_ctx *c, dv_frame_info *info) {
    if (!c || !info) return DV_ERR_ARG;
    if (!c->pushed) return fail(c, DV_ERR_STATE, "no frame has been pushed");
    (void)hipSetDevice(c->device);
    dv_status s = sync_state(c);
    if (s != DV_OK) return s;
    const SeqState &h = *c->h_state;
    dv_frame_info fi;
    std::memset(&fi, 0, sizeof(fi));
    fi.frame = h.frame;
    fi.status = h.status;
    fi.n_components = h.K_now;
    fi.n_edges = h.status == 0 ? h.E[h.sel] : 0;
    fi.n_flips = h.n_flips;
    fi.n_breaking = h.n_break;
    fi.n_excluded_past = h.n_excl_past;
    fi.n_excluded_now = h.n_excl_now;
    fi.n_ambiguous_centroids = h.n_amb;
    fi.global_trigger = (uint32_t)h.global_trigger;
    *info = fi;
    return (dv_status)h.status;
}

dv_status dv_get_flips(dv_ctx *c, dv_flip *host_out, int32_t capacity, int32_t *n_out) {
    if (!c || !n_out || capacity < 0) return DV_ERR_ARG;
    dv_status s = ready(c);
    if (s != DV_OK) return s;
    const int n = c->h_state->n_flips;
    *n_out = n;
    if (n > capacity) return fail(c, DV_ERR_CAPACITY, "flip buffer too small");
    if (n > 0) {
        if (!host_out) return fail(c, DV_ERR_ARG, "host_out is NULL");
        if (hipMemcpy(host_out, c->slot[0].B.flips, (size_t)n * sizeof(dv_flip), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(c, DV_ERR_DEVICE, "copy failed");
    }
    return DV_OK;
}

dv_status dv_get_labels(dv_ctx *c, int32_t *host_out) {
    if (!c || !host_out) return DV_ERR_ARG;
    if (!(c->cfg.flags & DV_KEEP_MAPS)) return fail(c, DV_ERR_STATE, "maps not kept (DV_KEEP_MAPS)");
    dv_status s = ready(c);
    if (s != DV_OK) return s;
    const Bufs &B = c->slot[c->last].B;
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
    const Bufs &B = c->slot[c->last].B;
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
    const CompBuf &C = c->slot[0].B.past[h.sel];
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
    launch_edge_list(c->slot[c->last].B, c->d_edge_ab, c->d_edge_total, c->d_edge_scratch, c->chain);
    int32_t E = 0;
    if (hipMemcpyAsync(&E, c->d_edge_total, 4, hipMemcpyDeviceToHost, c->chain) != hipSuccess ||
        hipStreamSynchronize(c->chain) != hipSuccess)
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
    const int KP = c->h_state->K_past_cmp;
    *n_out = KP;
    if (KP > capacity) return fail(c, DV_ERR_CAPACITY, "matching buffer too small");
    if (KP == 0) return DV_OK;
    if (!phi) return fail(c, DV_ERR_ARG, "phi is NULL");
    // Phi with dropped past points as -1, written to scratch on the device
    launch_phi_out(c->slot[c->last].B, c->d_edge_ab, c->chain);
    if (hipMemcpyAsync(phi, c->d_edge_ab, (size_t)KP * 4, hipMemcpyDeviceToHost, c->chain) != hipSuccess ||
        hipStreamSynchronize(c->chain) != hipSuccess)
        return fail(c, DV_ERR_DEVICE, "copy failed");
    return DV_OK;
}

void dv_destroy(dv_ctx *c) {
    if (!c) return;
    release(c);
    delete c;
}

static const char *const STAGE_NAMES[ST_COUNT] = {
    "tile_ccl", "merge", "resolve", "relabel", "finalize", "owner_edges", "match", "diff", "place"};

const char *dv_stage_name(int32_t stage) {
    return (stage >= 0 && stage < ST_COUNT) ? STAGE_NAMES[stage] : nullptr;
}

dv_status dv_set_profile(dv_ctx *c, int32_t stage, int32_t capacity) {
    if (!c) return DV_ERR_ARG;
    if (stage < -1 || stage >= ST_COUNT || (stage >= 0 && (capacity < 1 || capacity > (1 << 20))))
        return fail(c, DV_ERR_ARG, "bad stage or capacity");
    (void)hipSetDevice(c->device);
    if (!drain(c)) return fail(c, DV_ERR_DEVICE, "stream error");
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
    if (!drain(c)) return fail(c, DV_ERR_DEVICE, "stream error");
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
