/*
 * dv.h -- C ABI of the GPU detector of topological changes in dynamic lattice
 * Voronoi diagrams (Bernaschi, Lulli, Sbragaglia, "GPU Based Detection of
 * Topological Changes in Voronoi Diagrams", arXiv:1607.00908).
 *
 * One context follows one sequence of lattice fields (one simulation stream).
 * Each pushed field goes through the paper's procedure on the GPU:
 *   Sec. 3.1    threshold, cluster labelling, sizes and centres of mass
 *   Sec. 3.2.1  digital Voronoi colouring of the lattice by the centres
 *   Sec. 3.2.2  Voronoi-vertex sites (frame gaps) and the neighbour rules that
 *               give the Delaunay couples, compressed into sorted rows
 *   Sec. 3.2.3  kinematic isomorphism Phi_{P->N} between the previous ("past")
 *               and the current ("now") centres, translation of the past rows,
 *               row compare (local / global trigger), exclusion of bubbles that
 *               appear or disappear
 *   Sec. 3.2.4  breaking and arising couples (edge flips)
 *
 * Conventions fixed by this library where the paper leaves them open:
 *   - lattice: lx * ly sites, site (x, y) at linear index y*lx + x, periodic
 *     in both axes unless DV_OPEN_X / DV_OPEN_Y put walls across an axis;
 *     connectivity 8 (the D2Q9 directions) or 4;
 *   - walls (Sec. 3.2.2, frame on the domain boundary): on a walled axis
 *     components do not connect across the edge, offsets and distances are
 *     plain differences, and frame points beyond the edge count as MAXLINK
 *     (no gap, never a neighbour);
 *   - obstacles (Sec. 3.2.1, supplementary binary field; DV_OBSTACLES): an
 *     obstacle site is never inside a component and its colour is MAXLINK;
 *     the other sites are coloured by straight-line distance as before, and
 *     cells that meet only across an obstacle are not neighbours;
 *   - inside: rho > threshold (phase DV_PHASE_ABOVE, droplets) or
 *     rho < threshold (DV_PHASE_BELOW, bubbles); equality and NaN are outside;
 *   - labels 0..K-1 in increasing order of each component's smallest linear
 *     index, DV_NO_LABEL (-1) outside;
 *   - centres: unweighted mean of the member sites, offsets taken from the
 *     smallest-index member with the signed minimum image in
 *     [-floor(L/2), L-1-floor(L/2)]; Q.8 value (units of 1/256 site) =
 *     256*r + floor((512*S + n) / (2n)) mod 256L (exact integers);
 *   - colouring: squared periodic distance between Q.8 points in exact
 *     integers, ties to the lowest label;
 *   - inner-frame points of the second-neighbour rule: the four half-integer
 *     points (x +/- 1/2, y +/- 1/2);
 *   - matching: nearest now centre of each past centre (exact, ties to the
 *     lowest label); a past point is kept when its image has exactly one
 *     preimage, a now point when it has exactly one preimage; couples that
 *     touch a dropped point are ignored on both sides.
 *
 * Threading: a context is used by one host thread at a time.  Distinct
 * contexts are independent, also on one device.
 * Errors: every call returns a dv_status; no call writes partial results to
 * caller memory.  Argument errors are found on the host before any device work.
 */
#ifndef DV_H
#define DV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Colour of "no cell" and row padding value (Sec. 3.2.1, footnote on MAXLINK). */
#define DV_MAXLINK 0x77777777
#define DV_NO_LABEL (-1)

/* flags */
#define DV_KEEP_MAPS 1u  /* label / owner maps stay readable after each push */
#define DV_CLASSIFY 2u   /* fill dv_flip.flags with the event classification */
#define DV_OBSTACLES 4u  /* the context holds an obstacle mask (dv_set_obstacles) */
#define DV_OPEN_X 8u     /* walls across x instead of the periodic wrap          */
#define DV_OPEN_Y 16u    /* walls across y instead of the periodic wrap          */
#define DV_KEEP_RESULTS 32u /* keep every frame's record and flips until
                                dv_get_results returns them (Sec. 3.2.4, Sec. 4) */
#define DV_WEIGHTED 64u  /* centres are the centroids of Sec. 2 with the field as
                            density instead of the unit-weight centres of mass of
                            Sec. 3.1: site weight floor(256 rho + 1/2) clamped to
                            [1, 65535], exact integer sums, Q.8 rounded half up;
                            sizes stay member counts */

/* dv_flip.flags bits (with DV_CLASSIFY; Sec. 3.2.4, extraction of events).
 * Active points are the ends of the flips.  BULK: both ends are connected to
 * at least three active points (counted over the past graph translated by Phi
 * and the now graph).  BOUNDARY: both ends are boundary points of the graph
 * holding the couple (past graph for breaking, now graph for arising), a
 * boundary point having a couple whose ends share fewer than two neighbours.
 * A flip with neither bit is not part of a bulk or boundary event. */
#define DV_FLIP_BULK 1u
#define DV_FLIP_BOUNDARY 2u

typedef enum {
    DV_OK = 0,
    DV_ERR_ARG = 1,       /* invalid argument or configuration               */
    DV_ERR_CAPACITY = 2,  /* a configured capacity was exceeded (see below)   */
    DV_ERR_NOMEM = 3,     /* device or host allocation failed                 */
    DV_ERR_DEVICE = 4,    /* a HIP call failed                                */
    DV_ERR_STATE = 5,     /* call not valid in the current state              */
    DV_ERR_INTERNAL = 6
} dv_status;

typedef enum { DV_PHASE_ABOVE = 0, DV_PHASE_BELOW = 1 } dv_phase;

typedef struct dv_ctx dv_ctx;

typedef struct {
    uint32_t size;           /* = sizeof(dv_config); guards the ABI                */
    int32_t lx, ly;          /* lattice, each >= 3, lx*ly < 2^31, each <= 65536     */
    float threshold;         /* inside / outside threshold on the field            */
    int32_t phase;           /* dv_phase                                           */
    int32_t connectivity;    /* 8 (default) or 4                                   */
    int32_t max_components;  /* K_max, 1 .. 2^24; device memory is sized from it   */
    int32_t max_degree;      /* row capacity of the adjacency (Delaunay degree),
                                4 .. 64; 0 selects 48                              */
    int32_t device;          /* HIP device ordinal                                 */
    uint32_t flags;          /* DV_KEEP_MAPS | DV_CLASSIFY | DV_OBSTACLES |
                                DV_OPEN_X | DV_OPEN_Y | DV_KEEP_RESULTS            */
    int32_t max_batch;       /* frames sent to the device together, 1 .. 64; 0
                                selects 32.  Each holds its own per-site buffers. */
} dv_config;

/* One edge flip (Sec. 3.2.4).  a < b are now labels; pa, pb the past labels
 * with Phi(pa) = a and Phi(pb) = b.  kind = -1 breaking (couple only in the
 * past triangulation), +1 arising (only in the now triangulation).  flags:
 * DV_FLIP_* bits when the context has DV_CLASSIFY, else 0.  Flips are ordered
 * breaking first, then arising, each by (a, b) ascending. */
typedef struct {
    int32_t a, b;
    int32_t pa, pb;
    int32_t kind;
    uint32_t flags;
} dv_flip;

/* Summary of one frame (Sec. 3.1 counts, Sec. 3.2.3 exclusions and trigger,
 * Sec. 3.2.4 flips): of the most recent push (dv_get_info), or of every frame
 * in push order (dv_get_results). */
typedef struct {
    int64_t frame;                  /* frames accepted up to and including this one    */
    int32_t status;                 /* DV_OK, or DV_ERR_CAPACITY when rejected          */
    int32_t n_components;           /* K of the most recent push (may exceed K_max
                                       when status is DV_ERR_CAPACITY)                  */
    int32_t n_edges;                /* E: undirected Delaunay couples                   */
    int32_t n_flips;
    int32_t n_breaking;
    int32_t n_excluded_past;        /* past points dropped by the isomorphism          */
    int32_t n_excluded_now;         /* now points with no or several preimages          */
    int32_t n_ambiguous_centroids;  /* components crossing their own antipodal line    */
    uint32_t global_trigger;        /* 1 when any row changed (Sec. 3.2.3)             */
} dv_frame_info;

/* Create a context on cfg->device (state of one sequence of configurations
 * compared frame by frame, Sec. 3.2.3).  hip_stream is a hipStream_t on that
 * device, or NULL for a stream the context creates (and destroys).  All
 * device work of the context is ordered on that stream.  Pushed frames are
 * queued on the host and sent to the device together, max_batch at a time
 * (or fewer, at the next synchronising call): every stage then runs as one
 * launch over all of them.  On success *out owns every device buffer; on
 * failure *out is NULL. */
dv_status dv_create(const dv_config *cfg, void *hip_stream, dv_ctx **out);

/* Device memory, in bytes, that dv_create takes for cfg: the one region of
 * every per-slot and shared buffer of the procedure of Sec. 3.1-3.2.4 (the
 * results-page records and the sequence header are pinned host memory, not
 * counted).  Touches no device; DV_ERR_ARG for an invalid cfg or a NULL
 * bytes. */
dv_status dv_device_bytes(const dv_config *cfg, uint64_t *bytes);

/* Enqueue one frame: the whole procedure of Sec. 3.1-3.2.4 runs on it.
 * field_device: lx*ly float32 values in device memory,
 * row-major (x fastest), complete in the order of the context's stream at
 * the time of this call.  The field is read asynchronously on that stream,
 * at the latest when the next synchronising call (dv_get_flips, dv_get_info,
 * any getter, dv_sync) sends the queue: the caller keeps it alive and
 * unmodified until that call returns.  The call never waits for the device;
 * every max_batch-th push enqueues the launches of the queued frames.
 * The first accepted frame has no past and yields no flips.  A frame whose
 * component count exceeds K_max, or whose Delaunay degree exceeds the row
 * capacity, is rejected and the past state stays that of the last accepted
 * frame.  The rejection is reported in that frame's record (dv_get_results)
 * and, while it is the most recent push, by dv_get_info, dv_get_flips and the
 * other getters (DV_ERR_CAPACITY). */
dv_status dv_push_frame(dv_ctx *ctx, const float *field_device);

/* Set the obstacle mask (Sec. 3.2.1): lx*ly bytes, row-major, nonzero = obstacle;
 * in device memory when mask_on_device is nonzero, else host memory; NULL
 * clears every obstacle.  The context keeps its own copy: frames pushed
 * before the call keep the previous mask, later ones use this one.  Queued
 * frames are sent first and the call returns when the copy is complete.
 * Needs DV_OBSTACLES at creation (else DV_ERR_STATE); the mask starts empty. */
dv_status dv_set_obstacles(dv_ctx *ctx, const uint8_t *mask, int32_t mask_on_device);

/* Breaking and arising couples of the most recent push (Sec. 3.2.4), in the
 * order given at dv_flip.  Waits for the device.  When capacity is smaller
 * than the count, *n_out receives the count, nothing is written and
 * DV_ERR_CAPACITY is returned.  With batched pushes only the last frame of
 * the batch is the most recent push: dv_get_results returns every frame's. */
dv_status dv_get_flips(dv_ctx *ctx, dv_flip *host_out, int32_t capacity, int32_t *n_out);

/* Wait for the device; fill *info for the most recent push (counts of
 * Sec. 3.1-3.2.4).  Returns the status of that push (DV_OK or
 * DV_ERR_CAPACITY); *info is filled either way. */
dv_status dv_get_info(dv_ctx *ctx, dv_frame_info *info);

/* ---- every frame's results (Sec. 3.2.4: the flips of each comparison; Sec.
 * 4: detection at every interval of the run).  Needs DV_KEEP_RESULTS, else
 * DV_ERR_STATE.  The library keeps, for every frame sent to the device, its
 * dv_frame_info and its flips until dv_get_results has returned them: frames
 * of a batch are never overwritten unread (when a results page has to be
 * reused first, its unread frames are moved to host memory).
 *
 * wait != 0: queued frames are sent and every pushed frame is waited for.
 * wait == 0: nothing is sent or waited for; only frames whose launch has
 *            completed count (possibly none).
 *
 * dv_results_ready: *n_frames unread frames and *n_flips flips in them. */
dv_status dv_results_ready(dv_ctx *ctx, int32_t wait, int32_t *n_frames, int32_t *n_flips);

/* Return unread frames oldest first (push order, rejected frames included,
 * with status DV_ERR_CAPACITY and no flips): infos[i] for the i-th, and their
 * flips concatenated in the same order (infos[i].n_flips each, dv_flip order
 * within a frame).  Whole frames are returned while both capacities allow;
 * *n_frames and *n_flips receive what was written.  Returns DV_OK when every
 * ready frame was returned, DV_ERR_CAPACITY when some remain unread (they are
 * returned by the next call).  Host outputs; NULL is accepted for an output
 * whose capacity is 0. */
dv_status dv_get_results(dv_ctx *ctx, int32_t wait, dv_frame_info *infos, int32_t cap_frames,
                         int32_t *n_frames, dv_flip *flips, int32_t cap_flips, int32_t *n_flips);

/* Send any queued frames and wait until every pushed frame has gone through
 * the procedure of Sec. 3.1-3.2.4. */
dv_status dv_sync(dv_ctx *ctx);

/* Release everything the context owns (the sequence state of Sec. 3.2.3:
 * past centres and rows).  NULL is accepted. */
void dv_destroy(dv_ctx *ctx);

/* ---- inspection (all synchronise; host outputs; state of the most recent
 * push, which must have been accepted, else its error is returned) ---- */

/* Label map of the cluster labelling (Sec. 3.1), lx*ly int32 row-major,
 * DV_NO_LABEL outside.  Needs DV_KEEP_MAPS (else DV_ERR_STATE). */
dv_status dv_get_labels(dv_ctx *ctx, int32_t *host_out);
/* Colour map of the digital Voronoi tessellation (Sec. 3.2.1): nearest centre
 * of every site, DV_MAXLINK on obstacles and when there is no centre; lx*ly
 * int32 row-major.  Needs DV_KEEP_MAPS. */
dv_status dv_get_owner(dv_ctx *ctx, int32_t *host_out);
/* Centres of mass and sizes of the components (Sec. 3.1, last step; centroid
 * equation of Sec. 2 with unit weights): q8_xy[2k], [2k+1] Q.8 centre;
 * xy[2k], [2k+1] float64 centre; size[k] member count; any output pointer may
 * be NULL.  capacity and *n_out count components (DV_ERR_CAPACITY with the
 * count when too small). */
dv_status dv_get_components(dv_ctx *ctx, int32_t *q8_xy, double *xy, int32_t *size,
                            int32_t capacity, int32_t *n_out);
/* Delaunay couples given by the neighbour rules (Sec. 3.2.2, compressed
 * adjacency of Sec. 3.2.2-3.2.3): undirected, ab[2e] < ab[2e+1], sorted by
 * (a, b); capacity and *n_out count couples. */
dv_status dv_get_edges(dv_ctx *ctx, int32_t *ab, int32_t capacity, int32_t *n_out);
/* Kinematic isomorphism Phi_{P->N} of the most recent comparison (Sec.
 * 3.2.3) indexed by past label; -1 for past points dropped as appearing /
 * vanishing bubbles; *n_out = K of the past frame (0 for the first frame). */
dv_status dv_get_matching(dv_ctx *ctx, int32_t *phi, int32_t capacity, int32_t *n_out);

/* ---- groups: many independent fields in one launch per stage ---- */

/* (The paper runs one sequence at a time, Sec. 4; a group runs the same
 * per-frame procedure of Sec. 3.1-3.2.4 on the frames of several sequences.)
 * A group sends one frame of each of its members to the device together:
 * every stage is one launch over all members' frames, whatever their lattice
 * sizes (a flat work list of tiles).  Members are contexts made by dv_create
 * with the same device and the same hip_stream; each keeps its own past,
 * outputs and getters, which see the group's frames like pushed ones.
 * 1 <= n <= 64.  The group borrows the members: they must outlive it.  On
 * failure *out is NULL and nothing is allocated. */
typedef struct dv_group dv_group;
dv_status dv_group_create(dv_ctx *const *members, int32_t n, dv_group **out);

/* Push fields_device[i] (lx*ly float32 of member i, device memory) into member
 * i for every member, and send them to the device at once (frames a member
 * had queued go first).  Asynchronous like dv_push_frame; the fields follow
 * the same lifetime rule (until the next synchronising call on the member). */
dv_status dv_group_push(dv_group *g, const float *const *fields_device);

/* Push fields_device[i] into member members[i] for i < n (distinct members,
 * 1 <= n <= group size, any order) and send them at once: a launch over the
 * members that have a frame, the others untouched (continuous batching of
 * streams whose frames arrive at different times). */
dv_status dv_group_push_some(dv_group *g, const int32_t *members, const float *const *fields_device,
                             int32_t n);

/* Release the group (not its members, whose state of Sec. 3.2.3 stays).
 * NULL is accepted. */
void dv_group_destroy(dv_group *g);

/* ---- no allocation ---- */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the result
 * of
 *     dv_create(cfg) ; dv_push_frame(past_field) ; dv_push_frame(now_field) ;
 *     dv_get_info -> *info_device ; dv_get_flips -> flips_device ; dv_destroy
 * computed with no allocation and no synchronisation.  Every buffer is carved
 * from one static device array of 48 MiB per device (held from the first call
 * on that device until the process ends); a configuration whose buffers do not
 * fit returns DV_ERR_CAPACITY before any device work (512 x 512 sites with
 * max_components 2048 and max_degree 48 fit; 1024 x 1024 sites with
 * max_components 4096 do not).
 * cfg: as for dv_create; DV_OBSTACLES is refused (DV_ERR_ARG), DV_KEEP_MAPS,
 * DV_KEEP_RESULTS and max_batch are ignored.  hip_stream: the stream the
 * work is ordered on (NULL: the null stream); the fields are read and the
 * outputs written in that stream's order.  Outputs in device memory:
 * *info_device receives the now frame's dv_frame_info (status DV_ERR_CAPACITY
 * when it was rejected; n_flips may exceed capacity), flips_device the first
 * min(n_flips, capacity) flips in dv_flip order.  Calls on one device share
 * the array: calls whose work overlaps on the device (other streams, other
 * threads) race and must be ordered by the caller.  Errors (DV_ERR_ARG,
 * DV_ERR_CAPACITY, DV_ERR_DEVICE) are returned before or at the launch; the
 * text is dv_last_error(NULL). */
dv_status dv_compare_static(const dv_config *cfg, void *hip_stream, const float *past_field_device,
                            const float *now_field_device, dv_flip *flips_device, int32_t capacity,
                            dv_frame_info *info_device);

/* ---- measurement ---- */

/* Stages of the per-frame procedure, in launch order: threshold and cluster
 * labelling (Sec. 3.1) in tile_ccl, merge, resolve, relabel; centres and the
 * centre grid (Sec. 3.1) in finalize; colouring and neighbour rules (Sec.
 * 3.2.1-3.2.2) in owner_edges; compressed rows (Sec. 3.2.2) in rows;
 * isomorphism (Sec. 3.2.3) in match; row comparison and flips (Sec.
 * 3.2.3-3.2.4) in diff and place; event classification (Sec. 3.2.4) in
 * events. */
#define DV_N_STAGES 11
/* Bracket every launch of one stage with HIP events on the context's stream
 * (one launch covers every frame of a batch).
 * stage: 0 .. DV_N_STAGES-1, or -1 to stop.  capacity: launches that can be
 * recorded before the next dv_get_profile (further launches are not timed).
 * Creates the events; returns DV_ERR_ARG for a bad stage or capacity. */
dv_status dv_set_profile(dv_ctx *ctx, int32_t stage, int32_t capacity);
/* Wait for the device; *total_ms = summed event time of the recorded
 * launches, *launches = their number; clears the record. */
dv_status dv_get_profile(dv_ctx *ctx, double *total_ms, int32_t *launches);
/* Name of a stage of the list above ("tile_ccl", "owner_edges", ...); NULL
 * when out of range. */
const char *dv_stage_name(int32_t stage);

/* Text of a status code (errors of the calls above). */
const char *dv_status_str(dv_status s);
/* Text of the last error on this context ("" when none).  NULL ctx: text of
 * the last dv_create or dv_compare_static failure of the calling thread. */
const char *dv_last_error(const dv_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* DV_H */
