// Internal definitions shared by the HIP sources of libdv (device state,
// buffer table, kernel launchers).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dv.h"

#define DV_TILE 32                 // tile edge in sites (labelling, colouring)
#define DV_TILE_SITES (DV_TILE * DV_TILE)
#define DV_BORDER (4 * DV_TILE)    // border entries of a tile: top row, bottom row, left, right column
#define DV_BLOCK 256               // threads per tile workgroup
#define DV_EMPTY 0x77777777        // MAXLINK: empty row slot / no colour
#define DV_CAND_CAP 128            // candidate centre images held in LDS per chunk
#define DV_TILE_PAIRS 128          // couples a colouring tile lists for the row build

// error bits raised on the device during a frame
#define DV_E_KMAX 1u               // more components than K_max
#define DV_E_DEGREE 2u             // a Delaunay row overflowed max_degree

#define DV_MAX_BATCH 64            // frames of one sequence processed by one launch
#define DV_MAX_ENTRIES 64          // frames (of one or several sequences) in one launch
#define DV_DEFAULT_BATCH 32        // what max_batch = 0 selects

// Per-frame header, one per batch slot (device memory).
struct FrameState {
    int32_t K_now;         // components found in the frame (raw, may exceed K_max)
    uint32_t err;          // DV_E_* bits of the frame
    int32_t rows_dirty;    // rows of the slot's adjacency that may hold entries
    int32_t n_amb;         // components crossing their own antipodal line
    int32_t E2_acc;        // sum of now row lengths (2E)
    int32_t excl_acc;      // now points dropped by the isomorphism
    // outputs of the comparison with the past
    int32_t status;        // 0 accepted, else DV_ERR_CAPACITY
    int32_t n_flips;
    int32_t n_break;
    int32_t n_excl_past;
    int32_t n_excl_now;
    int32_t global_trigger;
    int32_t K_past;        // K of the past frame it was compared with (0: none)
    int32_t E_now;         // undirected couples of the frame
    int32_t nb_acc;        // breaking couples found by the row comparison
    int32_t na_acc;        // arising couples found by the row comparison
    int32_t pad[2];
};

// Result record of one frame in a results page: written by the device into
// pinned host memory, read by the host once the launch has completed.
struct FrameOut {
    long long frame;       // accepted frames of the sequence up to and including this one
    int32_t status;        // 0 accepted, else DV_ERR_CAPACITY
    int32_t K, E;          // components (raw when rejected), undirected couples
    int32_t n_flips, n_break;
    int32_t excl_past, excl_now;
    int32_t amb;           // components crossing their own antipodal line
    int32_t trigger;       // global trigger
    int32_t flip_off;      // first flip of the frame in the page's flip array
    int32_t pad[3];
};

// Sequence header (device memory).  Two past buffers alternate: buffer `sel`
// holds the last accepted frame before the batch in flight; the batch's last
// accepted frame is copied into buffer 1 - sel, and the commit flips `sel`.
struct SeqState {
    int32_t sel;
    int32_t past_valid;
    int32_t K[2];          // components held by each past buffer
    int32_t E[2];          // undirected couples held by each past buffer
    int32_t pad0;
    int32_t pg_fill[2];    // flips held by each results page
    int32_t pad;
    int64_t frame;         // accepted frames
};

// Component arrays of one buffer.
struct CompBuf {
    int32_t *qx, *qy;      // Q.8 centre
    double *fx, *fy;       // float64 centre
    int32_t *n;            // member count
    int32_t *root;         // smallest linear index of the component
    int32_t *amb;          // 1 when the component crosses its antipodal line
    int32_t *adj;          // rows [K_max][max_degree]: unordered sets, DV_EMPTY padded
};

// Everything a kernel may touch: the buffers of one batch slot (one frame)
// and the past buffers shared by all slots.  The table of all slots lives in
// device memory; a kernel takes its frame's entry (blockIdx.z) and, for the
// comparison, the entry of the frame before it.
struct Bufs {
    int32_t seq;           // sequence of the entry within a launch (past and commit)
    int32_t lx, ly, ntx, nty;
    float thr;
    int32_t phase, conn;
    int32_t kmax, maxdeg;
    int32_t ncells;        // bucket grid = tile grid
    int32_t keep_maps;     // write the label / owner maps
    int32_t classify;      // fill the flips' event flags
    int32_t open_x, open_y;  // 1: walls across that axis instead of wrapping
    int32_t weighted;      // centres weighted by the quantised field (DV_WEIGHTED)
    const uint8_t *obst;   // [N] obstacle sites (nonzero), or null: none
    int32_t *parent;       // [N] union-find over piece roots (linear site indices)
    uint16_t *bpc;         // [tiles][DV_BORDER] tile-local piece root of every tile-border
                           // site (0xffff outside): top row, bottom row, left column,
                           // right column, 32 entries each
    int32_t *labels;       // [N] output label map
    int32_t *owner;        // [N] output colour map
    uint16_t *lab16;       // [tiles][32][32] piece slot of every site (its index in the
                           // tile's piece list), 0xffff outside
                           // (tile-major: a tile's 2 KB are contiguous)
    uint16_t *pieces;      // [tiles][DV_TILE_SITES] tile-local root site of each piece slot
    int2 *prec;            // [tiles][DV_TILE_SITES / 2] per piece slot: canonical rank of
                           // its component, component root (x | y << 16)
    int32_t *npieces;      // [tiles]
    uint32_t *seg_mask;    // [ly][ntx] component-root bits per (row, tile column)
    int32_t *seg_prefix;   // [ly][ntx] roots before each segment within its band
    int32_t *band_sum;     // [nty] roots per band of 32 rows
    int32_t *band_pre;     // [nty] roots in the bands before each band
    // component accumulation (self-cleaning: finalize zeroes what it reads)
    long long *acc_x, *acc_y;   // sums of offsets from the root (weighted: of w * offset)
    long long *acc_w;           // [K_max] sums of the site weights (weighted centres only)
    int32_t *acc_n, *acc_amb, *acc_root;
    // bucket grid of the frame's centres
    int32_t *cell_count;   // [ncells]
    int32_t *cell_start;   // [ncells + 1]
    int32_t *cell_items;   // [K_max] labels ordered by cell
    int2 *cell_q;          // [K_max] their Q.8 centres
    int32_t *comp_cell, *comp_slot;  // [K_max]
    int2 *tpairs;          // [tiles][DV_TILE_PAIRS] distinct couples found by each tile
    int32_t *tpair_n;      // [tiles]
    int32_t *cnt;          // [K_max] preimages of each now label
    int32_t *inv;          // [K_max] now -> past (valid when cnt == 1)
    CompBuf cur;           // components and rows of the frame
    FrameState *fs;
    // comparison with the past
    int32_t *phi;          // [K_max] past -> now
    int32_t *trigger;      // [K_max] local trigger per kept past label
    int32_t *nb, *na;      // [K_max] breaking / arising count per now row
    int32_t *ob, *oa;      // [K_max] their exclusive prefixes
    int32_t *stage;        // [K_max][2 * max_degree][6] flips of each row, row order
    // event classification (when classify): per now label
    int32_t *act;          // [K_max] the row changed (an end of a flip)
    int32_t *ecnt;         // [K_max] active points connected in either graph
    int32_t *ebnd;         // [K_max] bit 0: boundary point of the now graph, bit 1: of the past
    CompBuf past[2];       // shared by the slots
    SeqState *st;          // shared by the slots
    // results pages (shared by the slots): every frame's record and flips,
    // kept until the host has read them
    FrameOut *pg_info[2];  // [page frames] records, pinned host memory (device view)
    int32_t *pg_flips[2];  // [page frames * K_max * max_degree][6] flips, device memory
};

// Results-page position of a launch entry: bits 0-5 the frame's record, bit 6
// the page, bit 7 set when the page starts empty with this launch.
#define DV_PG_POS(v) ((int)((v) & 63u))
#define DV_PG_PAGE(v) ((int)(((v) >> 6) & 1u))
#define DV_PG_FRESH(v) ((int)(((v) >> 7) & 1u))

// Field pointers of the frames of one launch.
struct Fields {
    const float *p[DV_MAX_ENTRIES];
};

// One launch's work: entries 0 .. n-1 of the device slot table D (frames of
// one or several sequences, each with its own lattice), and the prefix sums
// of their tile and band counts, so that a flat block index finds its entry.
// Entry e of a launch is row idx[e] of a device slot table, which is a
// separate kernel argument (const, restrict: slot fields are loaded once,
// not after every store).  Everything else travels in the kernel arguments,
// so a launch over any subset of a table needs no upload.
struct Batch {
    const Bufs *D;         // the table (host side only; kernels take it separately)
    int n;
    int tiles, bands;      // totals over the entries
    int tpe, bpe;          // tiles / bands of every entry when all are alike, else 0
    int kmax, nty;         // largest K_max and band count (launch shapes)
    int classify;          // some entry classifies events
    int geom;              // some entry has walls or obstacles (general kernels)
    int weighted;          // some entry has weighted centres
    int idx[DV_MAX_ENTRIES];        // table row of each entry
    uint32_t pslot[DV_MAX_ENTRIES]; // results-page position of each entry (DV_PG_*)
    int tbase[DV_MAX_ENTRIES + 1];  // first flat tile of each entry
    int bbase[DV_MAX_ENTRIES + 1];  // first flat band (32 rows) of each entry
};

// Entry holding flat index idx (base: prefix sums, n + 1 values; per: the
// common count when every entry has the same, else 0).
__device__ __forceinline__ int entry_of(const int *base, int per, int n, int idx) {
    if (per > 0) return idx / per;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= idx) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Entries of the launch that belong to sequence `seq` and passed their stage
// checks, as a bit mask over entry indices: lane j of the calling wave loads
// entry j, so every lane of the wave must make the call.
__device__ __forceinline__ unsigned long long accepted_entries(const Bufs *D, const Batch &G, int seq) {
    const int lane = threadIdx.x & 63;
    bool m = false;
    if (lane < G.n) {
        const Bufs &Bj = D[G.idx[lane]];
        m = Bj.seq == seq && Bj.fs->err == 0;
    }
    return __ballot(m);
}

// Past of entry i of a launch, given the mask of accepted entries of its
// sequence: the last earlier one, else -1 for the sequence's past buffer.
__device__ __forceinline__ int past_slot(unsigned long long accepted, int i) {
    const unsigned long long m = accepted & ((1ull << i) - 1ull);
    return m ? 63 - __clzll(m) : -1;
}

// The same by a walk over the earlier entries with uniform (scalar) loads:
// cheaper where many waves each need it, since the entries' headers stay in
// the scalar cache.
__device__ __forceinline__ int past_slot_walk(const Bufs *D, const Batch &G, int i) {
    const int q = D[G.idx[i]].seq;
    for (int j = i - 1; j >= 0; --j)
        if (D[G.idx[j]].seq == q && D[G.idx[j]].fs->err == 0) return j;
    return -1;
}

// Stage ids, in launch order (names in dv_api.hip).
enum {
    ST_TILE_CCL, ST_MERGE, ST_RESOLVE, ST_RELABEL, ST_FINALIZE, ST_OWNER_EDGES, ST_ROWS,
    ST_MATCH, ST_DIFF, ST_EVENTS, ST_PLACE, ST_COUNT
};

// Optional event bracketing of one stage (measurement only).
struct Prof {
    int stage = -1;          // stage to time, -1 none
    int cap = 0, used = 0;   // recorded launches
    hipEvent_t *ev = nullptr;  // [2 * cap]
    void begin(int id, hipStream_t s) {
        if (id == stage && used < cap) (void)hipEventRecord(ev[2 * used], s);
    }
    void end(int id, hipStream_t s) {
        if (id == stage && used < cap) {
            (void)hipEventRecord(ev[2 * used + 1], s);
            ++used;
        }
    }
};

// Bump placement of device buffers in one region, each piece 256-byte
// aligned; with a null base it only measures the region.
struct Carve {
    char *base = nullptr;
    size_t off = 0;
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += (count ? count : 1) * sizeof(T);
        return p;
    }
};
// Buffers of one batch slot (one frame), and those shared by the slots of a
// sequence (past components, sequence header, results-page flips of
// page_frames frames each; the page records are placed by the caller).  B
// must hold the lattice, K_max, max_degree, the tile counts and keep_maps.
// (dv_api.hip)
void place_slot(Carve &cv, Bufs &b);
void place_shared(Carve &cv, Bufs &B, int page_frames);
// Checks of a configuration done before any device work, and the error text
// returned by dv_last_error(NULL) (dv_api.hip).
dv_status check_config(const dv_config *cfg);
dv_status fail_global(dv_status s, const char *msg);
// Slot-table fields of a configuration (lattice, tiles, threshold, flags):
// every pointer null (dv_api.hip).
Bufs table_base(const dv_config &cfg);

// Launchers (all on stream s).
// k_label.hip
void launch_label(const Batch &G, const Fields &F, hipStream_t s, Prof &P);
// k_voronoi.hip
void launch_voronoi(const Batch &G, hipStream_t s, Prof &P);
// k_diff.hip: comparison of every entry with its past, commit per sequence
void launch_compare(const Batch &G, hipStream_t s, Prof &P);
// inspection helpers (k_diff.hip); slot: the most recent frame
void launch_phi_out(const Bufs &H, const Bufs *D, int slot, int32_t *d_out, hipStream_t s);
void launch_edge_list(const Bufs &H, const Bufs *D, int32_t *d_out_ab, int32_t *d_count,
                      int32_t *d_scratch, hipStream_t s);
