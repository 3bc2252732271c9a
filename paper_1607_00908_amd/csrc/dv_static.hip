// dv_compare_static: the comparison of two frames (the procedure of Sec.
// 3.1-3.2.4 on a past and a now field) with every device buffer in one
// file-scope device array, for callers that cannot allocate.  It runs the
// kernels of the context path, as a launch of two frames of one sequence:
// the now frame's past is the past frame of the same launch.
//
// The array is `scratch` below.  Its address on a device comes from
// hipGetSymbolAddress, taken once per device with that device current and
// kept; host code uses only that address.  Every call on a device shares the
// array and leaves its contents: a call clears what must start empty before
// its kernels, and calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "dv.h"
#include "dv_internal.h"

#define DV_STATIC_BYTES (48u << 20)   // the scratch array (bytes)
#define DV_STATIC_DEVICES 64

static __device__ __align__(256) unsigned char scratch[DV_STATIC_BYTES];

namespace {

std::mutex g_mu;
void *g_scratch[DV_STATIC_DEVICES];   // address of scratch on each device (null: not looked up)

// Address of the scratch array on `device` (current).
dv_status scratch_on(int device, char **out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail_global(DV_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed");
        g_scratch[device] = p;
    }
    *out = static_cast<char *>(g_scratch[device]);
    return DV_OK;
}

// Words to fill at the start of a call: ranges of 32-bit words.
#define DV_FILLS 18
struct Fills {
    int *p[DV_FILLS];
    long long n[DV_FILLS];
    int v[DV_FILLS];
    int count;
};

__global__ __launch_bounds__(256) void k_fill(Fills f) {
    for (int r = 0; r < f.count; ++r) {
        int *p = f.p[r];
        const long long n = f.n[r];
        const int v = f.v[r];
        for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
             i += (long long)gridDim.x * blockDim.x)
            p[i] = v;
    }
}

// The two slot-table entries, passed by value and written in place.
__global__ void k_put_table(Bufs *dst, Bufs a, Bufs b) {
    if (threadIdx.x == 0) {
        dst[0] = a;
        dst[1] = b;
    }
}

// The now frame's record into the caller's dv_frame_info, and its first
// `cap` flips into the caller's array.
__global__ __launch_bounds__(256) void k_out(const FrameOut *rec, const int *flips, dv_flip *out, int cap,
                                             dv_frame_info *info) {
    const FrameOut r = *rec;
    const int n = min(r.n_flips, cap);
    const int *src = flips + (size_t)6 * r.flip_off;
    for (int i = threadIdx.x; i < 6 * n; i += blockDim.x) (&out[0].a)[i] = src[i];
    if (threadIdx.x == 0) {
        dv_frame_info fi;
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
        *info = fi;
    }
}

}  // namespace

extern "C" dv_status dv_compare_static(const dv_config *cfg_in, void *hip_stream, const float *past_field,
                                       const float *now_field, dv_flip *flips_device, int32_t capacity,
                                       dv_frame_info *info_device) {
    dv_status s = check_config(cfg_in);
    if (s != DV_OK) return s;
    if (!past_field || !now_field || !info_device || capacity < 0 || (capacity > 0 && !flips_device))
        return fail_global(DV_ERR_ARG, "null field or output, or negative capacity");
    if (cfg_in->flags & DV_OBSTACLES)
        return fail_global(DV_ERR_ARG, "dv_compare_static takes no obstacle mask");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail_global(DV_ERR_DEVICE, "no HIP device");
    if (cfg_in->device < 0 || cfg_in->device >= ndev || cfg_in->device >= DV_STATIC_DEVICES)
        return fail_global(DV_ERR_ARG, "device ordinal out of range");
    dv_config cfg = *cfg_in;
    if (cfg.max_degree == 0) cfg.max_degree = 48;
    cfg.max_degree = (cfg.max_degree + 3) & ~3;
    cfg.flags &= ~(DV_KEEP_MAPS | DV_KEEP_RESULTS);   // no getters: no maps are written
    if (hipSetDevice(cfg.device) != hipSuccess) return fail_global(DV_ERR_DEVICE, "hipSetDevice failed");
    const hipStream_t st = (hipStream_t)hip_stream;

    // the buffers of a two-frame launch: shared part, one results page of
    // two frames and its records, the slot table, two slots
    Bufs B = table_base(cfg);
    Bufs tab[2];
    FrameOut *rec = nullptr;
    Bufs *d_tab = nullptr;
    auto layout = [&](Carve &cv) {
        place_shared(cv, B, 2);
        rec = cv.take<FrameOut>(2);
        B.pg_info[0] = B.pg_info[1] = rec;
        d_tab = cv.take<Bufs>(2);
        for (int k = 0; k < 2; ++k) {
            tab[k] = B;
            place_slot(cv, tab[k]);
        }
    };
    Carve measure;
    layout(measure);
    if (measure.off > DV_STATIC_BYTES)
        return fail_global(DV_ERR_CAPACITY, "configuration needs more than the 48 MiB static scratch "
                                            "(lattice, max_components and max_degree too large)");
    char *base = nullptr;
    s = scratch_on(cfg.device, &base);
    if (s != DV_OK) return s;
    Carve cv;
    cv.base = base;
    layout(cv);

    // what must start empty: sequence header, past rows, the slots' sums,
    // frame headers and rows (the same state a new context starts from)
    const long long K = B.kmax, KD = (long long)B.kmax * B.maxdeg;
    Fills f;
    std::memset(&f, 0, sizeof(f));
    bool fits = true;
    auto add = [&](void *p, long long words, int v) {
        if (f.count == DV_FILLS) {
            fits = false;
            return;
        }
        f.p[f.count] = static_cast<int *>(p);
        f.n[f.count] = words;
        f.v[f.count] = v;
        ++f.count;
    };
    add(B.st, sizeof(SeqState) / 4, 0);
    add(B.past[0].adj, KD, DV_EMPTY);
    add(B.past[1].adj, KD, DV_EMPTY);
    for (int k = 0; k < 2; ++k) {
        add(tab[k].acc_x, 2 * K, 0);
        add(tab[k].acc_y, 2 * K, 0);
        add(tab[k].acc_w, 2 * K, 0);
        add(tab[k].acc_n, K, 0);
        add(tab[k].acc_amb, K, 0);
        add(tab[k].fs, sizeof(FrameState) / 4, 0);
    }
    add(tab[0].cur.adj, KD, DV_EMPTY);
    add(tab[1].cur.adj, KD, DV_EMPTY);
    if (!fits) return fail_global(DV_ERR_INTERNAL, "fill list too short");
    const int fgrid = (int)std::min<long long>((KD + 255) / 256, 1024);
    hipLaunchKernelGGL(k_fill, dim3(fgrid), dim3(256), 0, st, f);
    hipLaunchKernelGGL(k_put_table, dim3(1), dim3(64), 0, st, d_tab, tab[0], tab[1]);

    // one launch per stage over the two frames; the now frame's past is the
    // past frame (same sequence, earlier entry)
    Batch G;
    std::memset(&G, 0, sizeof(G));
    G.D = d_tab;
    G.n = 2;
    G.idx[0] = 0;
    G.idx[1] = 1;
    G.pslot[0] = 0u | 128u;   // page 0, record 0, page starts empty
    G.pslot[1] = 1u | 128u;
    G.tbase[1] = B.ncells;
    G.tbase[2] = 2 * B.ncells;
    G.bbase[1] = B.nty;
    G.bbase[2] = 2 * B.nty;
    G.tiles = 2 * B.ncells;
    G.bands = 2 * B.nty;
    G.tpe = B.ncells;
    G.bpe = B.nty;
    G.kmax = B.kmax;
    G.nty = B.nty;
    G.classify = B.classify;
    G.geom = (B.open_x | B.open_y) ? 1 : 0;
    G.weighted = B.weighted;
    Fields F;
    std::memset(&F, 0, sizeof(F));
    F.p[0] = past_field;
    F.p[1] = now_field;
    Prof P;
    launch_label(G, F, st, P);
    launch_voronoi(G, st, P);
    launch_compare(G, st, P);
    hipLaunchKernelGGL(k_out, dim3(1), dim3(256), 0, st, rec + 1, (const int *)B.pg_flips[0], flips_device,
                       (int)capacity, info_device);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail_global(DV_ERR_DEVICE, hipGetErrorString(e));
    return DV_OK;
}
