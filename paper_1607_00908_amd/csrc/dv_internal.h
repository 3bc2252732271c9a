// Internal definitions shared by the HIP sources of libdv (device state,
// buffer table, kernel launchers).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define DV_TILE 32                 // tile edge in sites (labelling, colouring)
#define DV_TILE_SITES (DV_TILE * DV_TILE)
#define DV_BLOCK 256               // threads per tile workgroup
#define DV_EMPTY 0x77777777        // MAXLINK: empty row slot / no colour
#define DV_CAND_CAP 512            // candidate centre images held in LDS per chunk

// error bits raised on the device during a frame
#define DV_E_KMAX 1u               // more components than K_max
#define DV_E_DEGREE 2u             // a Delaunay row overflowed max_degree

// Frame header kept in device memory.  Two component / adjacency buffers
// alternate: buffer `sel` holds the last accepted frame (the past), buffer
// 1 - sel receives the frame being processed.
struct DevState {
    int32_t sel;
    int32_t past_valid;
    int32_t K[2];          // components held by each buffer
    int32_t E[2];          // undirected couples held by each buffer
    int32_t rows_dirty[2]; // rows of each buffer that may hold entries
    int32_t K_now;         // components found in the current frame (raw)
    uint32_t err;          // DV_E_* bits of the current frame
    int32_t E2_now;        // sum of row lengths of the current frame (2E)
    int32_t n_flips;
    int32_t n_break;
    int32_t n_excl_past;
    int32_t n_excl_now;
    int32_t n_amb;
    int32_t global_trigger;
    int32_t status;        // 0 accepted, else DV_ERR_CAPACITY of the last push
    int32_t K_past_cmp;    // K of the past frame used by the current comparison
    int32_t done_fin;      // blocks of k_finalize that have finished (last one resets)
    int32_t done_spare;
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

// Everything a kernel may touch.  Passed by value.
struct Bufs {
    int32_t lx, ly, ntx, nty;
    float thr;
    int32_t phase, conn;
    int32_t kmax, maxdeg;
    int32_t ncells;        // bucket grid = tile grid
    int32_t keep_maps;     // write the label / owner maps
    const float *field;
    int32_t *parent;       // [N] union-find over tile-border sites and piece roots
    int32_t *labels;       // [N] output label map
    int32_t *owner;        // [N] output colour map
    uint16_t *lab16;       // [N] tile-local root of every site, 0xffff outside
    uint16_t *pieces;      // [tiles][DV_TILE_SITES] local roots of each tile
    int32_t *npieces;      // [tiles]
    uint32_t *seg_mask;    // [ly][ntx] component-root bits per (row, tile column)
    int32_t *seg_prefix;   // [ly][ntx] roots before each segment within its band
    int32_t *band_sum;     // [nty] roots per band of 32 rows
    // component accumulation (self-cleaning: finalize zeroes what it reads)
    long long *acc_x, *acc_y;
    int32_t *acc_n, *acc_amb, *acc_root;
    // bucket grid of the now centres
    int32_t *cell_count;   // [ncells]
    int32_t *cell_start;   // [ncells + 1]
    int32_t *cell_items;   // [K_max] labels ordered by cell
    int2 *cell_q;          // [K_max] their Q.8 centres
    int32_t *comp_cell, *comp_slot;  // [K_max]
    // matching / diff
    int32_t *phi;          // [K_max] past -> now
    int32_t *cnt;          // [K_max] preimages of each now label
    int32_t *inv;          // [K_max] now -> past (valid when cnt == 1)
    int32_t *trigger;      // [K_max] local trigger per kept past label
    int32_t *nb, *na;      // [K_max] breaking / arising count per now row
    int32_t *ob, *oa;      // [K_max] their exclusive prefixes
    int32_t *stage;        // [K_max][2 * max_degree][6] flips of each row, row order
    int32_t *flips;        // [K_max * max_degree][6]
    CompBuf comp[2];
    DevState *st;
};

// Stage ids, in launch order (names in dv_api.hip).
enum {
    ST_TILE_CCL, ST_MERGE, ST_RESOLVE, ST_RELABEL, ST_FINALIZE, ST_OWNER_EDGES, ST_DIFF,
    ST_PLACE, ST_COUNT
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

// launchers (k_label.hip)
void launch_label(const Bufs &B, hipStream_t s, Prof &P);
// launchers (k_voronoi.hip)
void launch_voronoi(const Bufs &B, hipStream_t s, Prof &P);
// launchers (k_diff.hip)
void launch_diff(const Bufs &B, hipStream_t s, Prof &P);
// inspection helpers (k_diff.hip)
void launch_phi_out(const Bufs &B, int32_t *d_out, hipStream_t s);
void launch_edge_list(const Bufs &B, int32_t *d_out_ab, int32_t *d_count, int32_t *d_scratch,
                      hipStream_t s);
