// Cluster labelling and centre-of-mass sums (Sec. 3.1 of the paper).
//
// The lattice is cut into 32x32 tiles.  Per frame:
//   k_tile_ccl   threshold + union-find of each tile in LDS; every tile-local
//                root ("piece") gets an entry in the global parent array
//                (global linear site indices) and a slot in the tile's piece
//                list; every inside site's slot goes to a 16-bit map, and the
//                piece root of every tile-border site to the tile's 128-entry
//                border array (whole lines, read by k_merge);
//   k_merge      unions of pieces across tile borders and the periodic seams
//                (none across a wall);
//   k_resolve    per band of 32 rows: each piece finds its global root;
//                component roots (the smallest linear index of each component)
//                are marked in a bitmap of (row, tile column) segments, which
//                is scanned in raster order within the band;
//   k_rank       per piece: the canonical rank of its component (roots before
//                it in raster order) and the component root's coordinates;
//   k_relabel    reads the piece slots written by k_tile_ccl, writes
//                canonical labels and accumulates exact integer offsets from
//                each component's root (signed minimum image) per piece, then
//                per component.
// Union-find always links the larger index under the smaller one, so the root
// of every tree is its smallest index.
#include "dv_device.h"

#define RES_TILES 1024   // tiles of a band handled per pass of k_resolve

namespace {

// ---- union-find in LDS over tile-local indices -----------------------------
// Every parent is a smaller index than its child, so walks end at a root.
// Finds shorten the path they walk with plain stores (path splitting: a node
// gets its grandparent).  Such a store can replace a hook that another thread
// has just made on the same node; but that node had already stopped being a
// root, so the hooking thread's atomicMin returned its earlier parent and
// the thread retries with it: no union is lost.
__device__ __forceinline__ int lfind(int *L, int a) {
    int p = L[a];
    if (p == a) return a;
    int prev = a;
    for (;;) {
        const int next = L[p];
        if (next == p) return p;
        L[prev] = next;
        prev = p;
        p = next;
    }
}

__device__ void lunite(int *L, int a, int b) {
    bool done;
    do {
        a = lfind(L, a);
        b = lfind(L, b);
        if (a < b) {
            const int old = atomicMin(&L[b], a);
            done = (old == b);
            b = old;
        } else if (b < a) {
            const int old = atomicMin(&L[a], b);
            done = (old == a);
            a = old;
        } else {
            done = true;
        }
    } while (!done);
}

// ---- union-find in global memory over linear site indices -------------------
// gfind2 shortens paths as lfind does.  gfind_ro walks without writing: it is
// the find of a pass that also stores final roots, which a concurrent
// shortening store could otherwise replace with an intermediate ancestor.
__device__ __forceinline__ int gfind_ro(const gint *P, int a) {
    int p = P[a];
    while (p != a) {
        a = p;
        p = P[a];
    }
    return a;
}

// Finds of two nodes at once: the walks advance together, so the loads of a
// step are in flight together (a root's parent is itself, so both loads are
// always valid); each walk shortens its path (a node gets its grandparent, as
// in lfind), and each step moves to a smaller index, so both end.
__device__ __forceinline__ void gfind2(gint *P, int &a, int &b) {
    int pa = P[a], pb = P[b];
    int preva = a, prevb = b;
    bool da = pa == a, db = pb == b;
    while (!(da && db)) {
        const int na = P[pa], nb = P[pb];
        if (!da) {
            if (na == pa) {
                da = true;
            } else {
                P[preva] = na;
                preva = pa;
                pa = na;
            }
        }
        if (!db) {
            if (nb == pb) {
                db = true;
            } else {
                P[prevb] = nb;
                prevb = pb;
                pb = nb;
            }
        }
    }
    a = pa;
    b = pb;
}

__device__ void gunite(gint *P, int a, int b) {
    bool done;
    do {
        gfind2(P, a, b);
        if (a < b) {
            const int old = __hip_atomic_fetch_min(P + b, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            done = (old == b);
            b = old;
        } else if (b < a) {
            const int old = __hip_atomic_fetch_min(P + a, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            done = (old == a);
            a = old;
        } else {
            done = true;
        }
    } while (!done);
}

// Thread t of a 256-thread block owns column t & 31 and rows (t >> 5) + 8i,
// i = 0..3: every wave-wide load touches two full 128-byte rows, and a wave
// ballot gives the inside masks of those two rows.
//
// Start of the horizontal run of inside sites that contains column x, in a
// row whose inside mask is m (bit x set).
__device__ __forceinline__ int run_start(uint32_t m, int x) {
    const uint32_t below = x == 31 ? 0xffffffffu : ((2u << x) - 1u);
    const uint32_t out = ~m & below;
    return out ? 32 - __clz(out) : 0;
}

// One wave per tile, four tiles per block (GEOM: some entry of the launch has
// walls or obstacles; the periodic, unobstructed instance carries none of
// their tests).  Lane l takes column l & 31 and the rows (l >> 5) + 2k,
// k = 0..15, so that every wave load covers two whole rows.  A wave works on
// its own tile from start to end: it waits for nothing but its own LDS
// accesses, so the four tiles of a block overlap their latencies.
template <bool GEOM>
__global__ __launch_bounds__(256, 8) void k_tile_ccl(const Bufs *__restrict__ D, Batch G, Fields F) {
    // (the same for every lane of the wave: read once, so that the slot's
    // fields are loaded into scalar registers)
    const int gt = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (gt >= G.tiles) return;   // a whole wave; there is no block barrier below
    const int e = entry_of(G.tbase, G.tpe, G.n, gt);
    const Bufs B = D[G.idx[e]];   // (a copy: the loads are not repeated after stores)
    // per wave: tile-local union-find (after the slots are assigned, a piece
    // root's entry also holds its slot in bits 16..), row masks
    __shared__ int Ls[4][DV_TILE_SITES];
    __shared__ uint32_t rowms[4][DV_TILE];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int *L = Ls[w];
    uint32_t *rowm = rowms[w];
    const int tile = gt - G.tbase[e];
    const int tx = tile % B.ntx, ty = tile / B.ntx;
    const int x0 = tx * DV_TILE, y0 = ty * DV_TILE;
    const int tw = min(DV_TILE, B.lx - x0), th = min(DV_TILE, B.ly - y0);
    FrameState *fs = B.fs;
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    };

    // per-frame resets spread over the grid
    if (tile == 0 && lane == 0) {
        fs->K_now = 0;
        fs->err = 0;
        fs->n_amb = 0;
        fs->E2_acc = 0;
        fs->excl_acc = 0;
        fs->nb_acc = 0;
        fs->na_acc = 0;
    }
    if (lane == 0) B.cell_count[tile] = 0;
    if (lane < th) gmem(B.seg_mask)[(size_t)(y0 + lane) * B.ntx + tx] = 0u;
    {   // empty the rows this frame will fill
        const size_t total = (size_t)fs->rows_dirty * B.maxdeg;
        const size_t stride = (size_t)B.ncells * 64;
        auto adj = gmem(B.cur.adj);
        for (size_t i = (size_t)tile * 64 + lane; i < total; i += stride) adj[i] = DV_EMPTY;
    }

    const int cx = lane & 31, h = lane >> 5;
    // the field (and obstacle) values of the lane's sites, loads issued
    // together; beyond a ragged tile's edge a lane reads the nearest site of
    // the tile and ignores it
    const float *field = F.p[e];
    const size_t tbase = (size_t)y0 * B.lx + x0;
    const int xc = min(cx, tw - 1);
    // inside masks of the rows, each site pointing to its run's first site;
    // in two halves of eight sites (fewer values live at once)
    unsigned starts = 0;   // bit k: the lane's site k starts a run
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        float v[8];
        uint8_t ob[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * half + j;
            const size_t g = tbase + (size_t)(min(h + 2 * k, th - 1) * B.lx + xc);
            v[j] = field[g];
            ob[j] = (GEOM && B.obst) ? gmem(B.obst)[g] : (uint8_t)0;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * half + j, y = h + 2 * k;
            const bool in = cx < tw && y < th && !ob[j] && (B.phase == 0 ? (v[j] > B.thr) : (v[j] < B.thr));
            const unsigned long long bal = __ballot(in);
            const uint32_t m = (uint32_t)(h == 0 ? bal : (bal >> 32));
            if (cx == 0) rowm[y] = m;
            const int rs = in ? run_start(m, cx) : -1;
            L[y * 32 + cx] = in ? y * 32 + rs : -1;
            starts |= (rs == cx) ? 1u << k : 0u;
        }
    }
    wave_sync();
    // Unions of each run [a, b] with the runs of the row above that touch
    // it: columns a - 1 .. b + 1 (8-connectivity) or a .. b (4): the run
    // holding the lowest touching site of the row above, and every other
    // run of that row starting inside the span.  Lane y takes row y.
    if (lane >= 1 && lane < 32 && lane < th) {
        const int y = lane;
        const uint32_t m = rowm[y], up = rowm[y - 1];
        if (m && up) {
            const uint32_t st_up = up & ~(up << 1);
            uint32_t rst = m & ~(m << 1);
            while (rst) {
                const int a = __ffs(rst) - 1;
                rst &= rst - 1;
                const uint32_t rest = ~(m >> a);            // bit k clear: a + k inside
                const int b = rest ? a + __ffs(rest) - 2 : 31;
                const int lo = (B.conn == 8 && a > 0) ? a - 1 : a;
                const int hi = (B.conn == 8 && b < 31) ? b + 1 : b;
                const uint32_t span = (hi == 31 ? 0xffffffffu : ((2u << hi) - 1u)) & ~((1u << lo) - 1u);
                const uint32_t hit = up & span;
                if (!hit) continue;
                const int me = y * 32 + a;
                const int p0 = __ffs(hit) - 1;
                lunite(L, me, (y - 1) * 32 + run_start(up, p0));
                uint32_t more = st_up & hit & ~(1u << p0);
                while (more) {
                    const int q = __ffs(more) - 1;
                    more &= more - 1;
                    lunite(L, me, (y - 1) * 32 + q);
                }
            }
        }
    }
    wave_sync();
    // roots of the run starts, stored once every find has ended (a find that
    // is still shortening its path could otherwise replace a stored root with
    // an intermediate ancestor); other inside sites keep pointing at their
    // run start
    unsigned rootp[8];   // roots of sites 2j and 2j + 1 in the low / high half (0xffff: none)
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int s = (h + 2 * k) * 32 + cx;
        const unsigned r = ((starts >> k) & 1u) && L[s] < s ? (unsigned)lfind(L, s) : 0xffffu;
        rootp[k >> 1] = (k & 1) ? (rootp[k >> 1] | (r << 16)) : r;
    }
    wave_sync();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const unsigned r = (rootp[k >> 1] >> (16 * (k & 1))) & 0xffffu;
        if (r != 0xffffu) L[(h + 2 * k) * 32 + cx] = (int)r;
    }
    wave_sync();
    // piece roots (L[s] == s) take consecutive slots in the tile's piece list
    // (a wave prefix); the slot goes into bits 16.. of the root's entry
    int npc = 0;
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int y = h + 2 * k, s = y * 32 + cx;
        const bool pr = L[s] == s;
        const unsigned long long bal = __ballot(pr);
        if (pr) {
            const int slot = npc + __popcll(bal & below);
            L[s] = s | (slot << 16);
            gmem(B.pieces)[(size_t)tile * DV_TILE_SITES + slot] = (uint16_t)s;
            const int g = (y0 + y) * B.lx + x0 + cx;
            gmem(B.parent)[g] = g;
        }
        npc += __popcll(bal);
    }
    wave_sync();
    // the 16-bit map holds each inside site's piece slot, the border array
    // each border site's piece root (an outside site is marked, so that
    // merging needs no field)
    auto bp = gmem(B.bpc) + (size_t)tile * DV_BORDER;
    auto lab = gmem(B.lab16) + (size_t)tile * DV_TILE_SITES;
    // site -> its run start -> the start's root -> the root's slot, without
    // branches (an outside site follows itself), so that the reads of the
    // sixteen sites are in flight together
    unsigned rootq[8];   // piece roots of sites 2j and 2j + 1 in the low / high half (0xffff: outside)
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int y = h + 2 * k, s = y * 32 + cx;
        const int v0 = L[s];
        const bool in = v0 >= 0;
        const int i1 = in ? (v0 & 0xffff) : s;
        const int i2 = in ? (L[i1] & 0xffff) : s;
        const int v2 = L[i2];
        const unsigned r = in ? (unsigned)i2 : 0xffffu;
        rootq[k >> 1] = (k & 1) ? (rootq[k >> 1] | (r << 16)) : r;
        if (cx < tw && y < th) lab[y * 32 + cx] = in ? (uint16_t)((unsigned)v2 >> 16) : (uint16_t)0xffff;
    }
    wave_sync();
    // every site's piece root into the table (0xffff outside, also beyond a
    // ragged tile's edge), then the border array as two whole lines per
    // lane: top and bottom row, left and right column
#pragma unroll
    for (int k = 0; k < 16; ++k)
        L[(h + 2 * k) * 32 + cx] = (int)((rootq[k >> 1] >> (16 * (k & 1))) & 0xffffu);
    wave_sync();
    {
        const int c = lane & 31;
        const int a = h == 0 ? L[c] : L[(th - 1) * 32 + c];
        const int b = h == 0 ? L[c * 32] : L[c * 32 + tw - 1];
        bp[lane] = (uint16_t)a;
        bp[2 * DV_TILE + lane] = (uint16_t)b;
    }
    if (lane == 0) B.npieces[tile] = npc;
}

// Unions between inside sites of neighbouring tiles (the border arrays hold
// the piece root of every tile-border site, or 0xffff when outside).  One
// wave per tile: lane j < 32 takes row j of the tile's last column against
// the next column (periodic); lane 32 + j takes column j of the last row
// against the next row.  Together they cover every adjacent pair that
// crosses a tile border, including the diagonal pairs at tile corners and
// the periodic seams; a pair across a wall is not formed.  Uniting two sites
// is uniting their pieces, so the pairs of piece roots are united, and a
// pair equal to one the previous thread of the same line unites is skipped
// (two pieces usually touch along many sites).
__device__ __forceinline__ void merge_line(gint *P, int ps, const int pu[3], bool conn8, bool active,
                                           int lane) {
    // pairs of this thread: up to three (ps, pu[k])
    int a[3], b[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const bool use = active && ps >= 0 && pu[k] >= 0 && (conn8 || k == 1);
        a[k] = use ? ps : -1;
        b[k] = use ? pu[k] : -1;
    }
    // the previous thread's pairs (lanes 0 and 32 start a line: what they
    // receive is not used)
    int pa[3], pb[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        pa[k] = wave_prev(a[k], -1);
        pb[k] = wave_prev(b[k], -1);
    }
    const bool first = (lane & 31) == 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (a[k] < 0) continue;
        bool dup = false;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            dup = dup || (!first && pa[q] == a[k] && pb[q] == b[k]);
            if (q < k) dup = dup || (a[q] == a[k] && b[q] == b[k]);
        }
        if (!dup) gunite(P, a[k], b[k]);
    }
}

// The border pairs of tile gt (flat over the launch) that lane `lane` unites:
// the piece root of its site and of up to three neighbours (-1 when outside
// or not formed).
template <bool GEOM>
__device__ __forceinline__ void border_pairs(const Bufs &B, int tile, int lane, int &ps, int pu[3],
                                             bool &active) {
    const int tx = tile % B.ntx, ty = tile / B.ntx;
    const int x0 = tx * DV_TILE, y0 = ty * DV_TILE;
    const int tw = min(DV_TILE, B.lx - x0), th = min(DV_TILE, B.ly - y0);
    const int lx = B.lx, ly = B.ly;
    const int j = lane & 31;
    const auto bp = gmem(B.bpc);
    const int ntx = B.ntx;
    // piece root (linear index) of the site (x, y) from entry `at` of its
    // tile's border array, -1 outside
    auto piece = [&](int x, int y, int at) -> int {
        const int xt = x & ~(DV_TILE - 1), yt = y & ~(DV_TILE - 1);
        const int v = bp[(size_t)((yt >> 5) * ntx + (xt >> 5)) * DV_BORDER + at];
        return v == 0xffff ? -1 : (yt + (v >> 5)) * lx + xt + (v & 31);
    };
    ps = -1;
    pu[0] = pu[1] = pu[2] = -1;
    if (lane < 32) {
        // row j of the last column against the next column (the first
        // column of its tile: left-column entries)
        const int x = x0 + tw - 1, y = y0 + j;
        active = j < th && !(GEOM && B.open_x && x + 1 == lx);
        if (active) {
            const int xn = (x + 1 == lx) ? 0 : x + 1;
            ps = piece(x, y, 3 * DV_TILE + j);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                int yn = y + k - 1;
                const bool cut = GEOM && B.open_y && (yn < 0 || yn >= ly);
                yn = yn < 0 ? yn + ly : (yn >= ly ? yn - ly : yn);
                pu[k] = cut ? -1 : piece(xn, yn, 2 * DV_TILE + (yn & (DV_TILE - 1)));
            }
        }
    } else {
        // column j of the last row against the next row (the first row of
        // its tile: top-row entries)
        const int x = x0 + j, y = y0 + th - 1;
        active = j < tw && !(GEOM && B.open_y && y + 1 == ly);
        if (active) {
            const int yn = (y + 1 == ly) ? 0 : y + 1;
            ps = piece(x, y, DV_TILE + j);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                int xn = x + k - 1;
                const bool cut = GEOM && B.open_x && (xn < 0 || xn >= lx);
                xn = xn < 0 ? xn + lx : (xn >= lx ? xn - lx : xn);
                pu[k] = cut ? -1 : piece(xn, yn, xn & (DV_TILE - 1));
            }
        }
    }
}

// MERGE_TILES tiles per wave, four waves per block: the border loads of all
// of a wave's tiles are in flight together before their unions.
#define MERGE_TILES 2
template <bool GEOM>
__global__ __launch_bounds__(256) void k_merge(const Bufs *__restrict__ D, Batch G) {
    const int gt0 = __builtin_amdgcn_readfirstlane((blockIdx.x * 4 + (threadIdx.x >> 6)) * MERGE_TILES);
    if (gt0 >= G.tiles) return;
    const int lane = threadIdx.x & 63;
    int ps[MERGE_TILES], pu[MERGE_TILES][3];
    bool active[MERGE_TILES];
    const Bufs *Bt[MERGE_TILES];
#pragma unroll
    for (int m = 0; m < MERGE_TILES; ++m) {
        const int gt = min(gt0 + m, G.tiles - 1);
        const int e = entry_of(G.tbase, G.tpe, G.n, gt);
        Bt[m] = &D[G.idx[e]];
        border_pairs<GEOM>(*Bt[m], gt - G.tbase[e], lane, ps[m], pu[m], active[m]);
        active[m] = active[m] && gt0 + m < G.tiles;
    }
#pragma unroll
    for (int m = 0; m < MERGE_TILES; ++m)
        merge_line(gmem(Bt[m]->parent), ps[m], pu[m], Bt[m]->conn == 8, active[m], lane);
}

// One block per band of 32 rows: every piece of the band's tiles finds its
// component root (the smallest linear index of the component); component
// roots set their bit in the band's (row, tile column) segment words, which
// are then scanned in raster order.  seg_prefix holds the number of roots
// before each segment within the band, band_sum the band's total; k_bandpre
// then writes band_pre (roots in the bands before each band), K and the
// capacity check.
// Segment (y, tile column c) covers sites y*lx + 32c .. 32c+31, so raster
// order of segments is the row-major order of the [ly][ntx] arrays.
__global__ __launch_bounds__(1024) void k_resolve(const Bufs *__restrict__ D, Batch G) {
    const int e = entry_of(G.bbase, G.bpe, G.n, blockIdx.x);
    const Bufs B = D[G.idx[e]];
    __shared__ int pre[RES_TILES + 1];
    __shared__ int wsum[16];
    const int ty = blockIdx.x - G.bbase[e], t = threadIdx.x;
    const int y0 = ty * DV_TILE, th = min(DV_TILE, B.ly - y0);
    const int ntx = B.ntx;
    for (int c0 = 0; c0 < ntx; c0 += RES_TILES) {
        const int nt = min(RES_TILES, ntx - c0);
        const int tile0 = ty * ntx + c0;
        // pieces of tiles c0 .. c0 + nt - 1, numbered through a block scan
        const int total = block_exclusive_scan(B.npieces + tile0, pre, nt, wsum);
        __syncthreads();
        for (int f = t; f < total; f += blockDim.x) {
            int lo = 0, hi = nt - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (pre[mid] <= f) lo = mid; else hi = mid - 1;
            }
            const int tx = c0 + lo;
            const int r = B.pieces[(size_t)(tile0 + lo) * DV_TILE_SITES + (f - pre[lo])];
            const int g = (y0 + (r >> 5)) * B.lx + tx * DV_TILE + (r & 31);
            const int root = gfind_ro(gmem(B.parent), g);
            if (root != g) gmem(B.parent)[g] = root;
            else atomicOr(&B.seg_mask[(size_t)(y0 + (r >> 5)) * ntx + tx], 1u << (r & 31));
        }
        __syncthreads();
    }
    // raster-order prefix of the root bits within the band
    const int n = th * ntx;
    const size_t base = (size_t)y0 * ntx;
    const int lane = t & 63, wid = t >> 6, nw = blockDim.x >> 6;
    int carry = 0;
    for (int c0 = 0; c0 < n; c0 += blockDim.x) {
        const int i = c0 + t;
        const int v = i < n ? __popc(B.seg_mask[base + i]) : 0;
        const int x = wave_incl_sum(v);
        __syncthreads();
        if (lane == 63) wsum[wid] = x;
        __syncthreads();
        int before = carry;
        for (int w = 0; w < wid; ++w) before += wsum[w];
        if (i < n) B.seg_prefix[base + i] = before + x - v;
        int tot = 0;
        for (int w = 0; w < nw; ++w) tot += wsum[w];
        carry += tot;
    }
    if (t == 0) B.band_sum[ty] = carry;
}

// One block per frame: the band totals become prefixes (roots in the bands
// before each band), and K and the capacity check are published.  (A kernel
// of its own: a last-block ticket in k_resolve would need a device-wide
// release in every band's block.)
__global__ __launch_bounds__(1024) void k_bandpre(const Bufs *__restrict__ D, Batch G) {
    const Bufs B = D[G.idx[blockIdx.z]];
    __shared__ int wsum[16];
    const int K = block_exclusive_scan(B.band_sum, B.band_pre, B.nty, wsum);
    if (threadIdx.x == 0) {
        FrameState *fs = B.fs;
        fs->K_now = K;
        if (K > B.kmax) atomicOr(&fs->err, DV_E_KMAX);
        fs->rows_dirty = min(K, B.kmax);
    }
}

// RANK_LANES lanes per tile (a tile has few pieces in the usual case): every
// piece's canonical rank (the component roots before its root in raster
// order) and its component root, by piece slot, so that k_relabel reads them
// with its first loads.  The component root's piece records the root for the
// centre.
#define RANK_LANES 8
__global__ __launch_bounds__(256) void k_rank(const Bufs *__restrict__ D, Batch G) {
    const int gt = blockIdx.x * (256 / RANK_LANES) + threadIdx.x / RANK_LANES;
    if (gt >= G.tiles) return;
    const int e = entry_of(G.tbase, G.tpe, G.n, gt);
    const Bufs B = D[G.idx[e]];
    const int tile = gt - G.tbase[e];
    const int x0 = (tile % B.ntx) * DV_TILE, y0 = (tile / B.ntx) * DV_TILE;
    const int lx = B.lx, j = threadIdx.x % RANK_LANES;
    const int np = gmem(B.npieces)[tile];
    for (int k = j; k < np; k += RANK_LANES) {
        const int r = gmem(B.pieces)[(size_t)tile * DV_TILE_SITES + k];
        const int g = (y0 + (r >> 5)) * lx + x0 + (r & 31);
        const int Gr = gmem(B.parent)[g];    // component root (compressed)
        const int gx = Gr % lx, gy = Gr / lx;
        const size_t seg = (size_t)gy * B.ntx + (gx >> 5);
        const uint32_t below = (1u << (gx & 31)) - 1u;
        const int rank = gmem(B.band_pre)[gy / DV_TILE] + gmem(B.seg_prefix)[seg] +
                         __popc(gmem(B.seg_mask)[seg] & below);
        st_int2(B.prec, (size_t)tile * (DV_TILE_SITES / 2) + k, rank, gx | (gy << 16));
        if (Gr == g && rank < B.kmax) gmem(B.acc_root)[rank] = Gr;
    }
}

__device__ __forceinline__ int wrap_off(int v, int L) {
    // v in (-L, L) -> signed minimum image in [-floor(L/2), L-1-floor(L/2)]
    const int h = L >> 1;
    if (v > L - 1 - h) v -= L;
    else if (v < -h) v += L;
    return v;
}

// Site weight of the density-weighted centres (centroid equation of Sec. 2):
// the field value quantised to 1/256, clamped to [1, 65535] (float64, exact).
__device__ __forceinline__ int site_weight(float rho) {
    const double v = floor(256.0 * (double)rho + 0.5);
    return !(v >= 1.0) ? 1 : (v > 65535.0 ? 65535 : (int)v);
}

// WT: some entry of the launch has weighted centres (its runs read the field
// again for the site weights; the other entries' sums are the unit-weight ones).
template <bool GEOM, bool WT>
__global__ __launch_bounds__(DV_BLOCK) void k_relabel(const Bufs *__restrict__ D, Batch G, Fields F) {
    const int e = entry_of(G.tbase, G.tpe, G.n, blockIdx.x);
    const Bufs B = D[G.idx[e]];   // (a copy: the loads are not repeated after stores)
    // piece slot of every site (0xffff outside), as written by k_tile_ccl
    __shared__ uint16_t L[DV_TILE_SITES];
    // per piece (indexed by its slot; a tile has at most 512 pieces): rank,
    // component root (x | y << 16), integer sums
    __shared__ int prank[DV_TILE_SITES / 2];
    __shared__ uint32_t pxy[DV_TILE_SITES / 2];
    __shared__ int psx[DV_TILE_SITES / 2], psy[DV_TILE_SITES / 2], pn[DV_TILE_SITES / 2];
    // weighted sums per piece: w * dx, w * dy, w (64-bit)
    __shared__ long long wsx[WT ? DV_TILE_SITES / 2 : 1], wsy[WT ? DV_TILE_SITES / 2 : 1],
        wsw[WT ? DV_TILE_SITES / 2 : 1];
    const bool wt = WT && B.weighted;
    __shared__ uint32_t rowm[DV_TILE];
    __shared__ uint16_t runs[DV_TILE_SITES / 2];   // (row << 5) | first column of each run
    __shared__ int nruns;
    const int tile = blockIdx.x - G.tbase[e];
    const int tx = tile % B.ntx, ty = tile / B.ntx;
    const int x0 = tx * DV_TILE, y0 = ty * DV_TILE;
    const int tw = min(DV_TILE, B.lx - x0), th = min(DV_TILE, B.ly - y0);
    const int t = threadIdx.x, lx = B.lx, ly = B.ly;

    // piece slots of the tile's sites and its piece count, as written by k_tile_ccl
    const int cx = t & 31, ry = t >> 5;
    uint16_t u[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = ry + 8 * i;
        const bool ok = cx < tw && y < th;
        u[i] = gmem(B.lab16)[(size_t)tile * DV_TILE_SITES + (ok ? y * 32 + cx : 0)];
    }
    const int np = gmem(B.npieces)[tile];
    // the first wave reads the ranks of slots 0..63 at once, in use or not (a
    // tile usually has a few pieces; the slots are allocated): 512 bytes per
    // tile, and no load that waits for the piece count
    int2 pr0 = make_int2(0, 0);
    if (t < 64) pr0 = ld_int2(B.prec, (size_t)tile * (DV_TILE_SITES / 2) + t);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = ry + 8 * i;
        L[y * 32 + cx] = (cx < tw && y < th) ? u[i] : (uint16_t)0xffff;
    }
    // each piece (thread t takes slot t; at most 512): rank and component
    // root as k_rank found them
    for (int k = t; k < np; k += DV_BLOCK) {
        const int2 pr = (k == t && t < 64) ? pr0 : ld_int2(B.prec, (size_t)tile * (DV_TILE_SITES / 2) + k);
        prank[k] = pr.x;
        pxy[k] = (uint32_t)pr.y;
        psx[k] = 0;
        psy[k] = 0;
        pn[k] = 0;
        if (WT) wsx[k] = wsy[k] = wsw[k] = 0;
    }
    __syncthreads();

    // offsets from the root: minimum image on a periodic axis; on a walled axis
    // plain differences (wrap_off over twice the length changes nothing), and
    // no antipodal line to cross
    const bool ox = GEOM && B.open_x, oy = GEOM && B.open_y;
    const int wlx = ox ? 2 * lx : lx, wly = oy ? 2 * ly : ly;
    const int hix = ox ? INT_MAX : lx - 1 - (lx >> 1);
    const int hiy = oy ? INT_MAX : ly - 1 - (ly >> 1);
    const int lane = t & 63;
    // label map and row masks
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = ry + 8 * i, s = y * 32 + cx;
        const int r = L[s];
        const bool inside = r != 0xffff;
        const unsigned long long bal = __ballot(inside);
        if (cx == 0) rowm[y] = (uint32_t)(lane < 32 ? bal : (bal >> 32));
        if (B.keep_maps && cx < tw && y < th)
            gmem(B.labels)[(size_t)(y0 + y) * lx + x0 + cx] = inside ? prank[r] : -1;
    }
    __syncthreads();
    // list of the horizontal runs: lane y of the first wave writes those of row y
    if (t < 64) {
        const uint32_t m = t < 32 ? rowm[t] : 0u;
        uint32_t st = m & ~(m << 1);
        const int c = __popc(st);
        const int x = wave_incl_sum(c);
        for (int k = x - c; st; ++k) {
            runs[k] = (uint16_t)((t << 5) | (__ffs(st) - 1));
            st &= st - 1;
        }
        if (t == 63) nruns = x;
    }
    __syncthreads();
    // one thread per run: its closed-form sums go to its piece; a run that
    // meets the root's antipodal line checks its sites (an adjacent inside
    // site is a member; crossing the line makes the unwrapped coordinates
    // jump by L - 1; such sites are rare, their neighbours are read from the
    // global map)
    const int nr = nruns;
    for (int k = t; k < nr; k += DV_BLOCK) {
        const int y = runs[k] >> 5, a = runs[k] & 31;
        const int r = L[y * 32 + a];
        const uint32_t m = rowm[y];
        const int len = __builtin_ctzll(~(unsigned long long)(m >> a));   // a full row is 32
        const int prx = (int)(pxy[r] & 0xffffu), pry = (int)(pxy[r] >> 16);
        const int dx = wrap_off(x0 + a - prx, wlx);
        const int dy = wrap_off(y0 + y - pry, wly);
        const int dx_end = wrap_off(x0 + a + len - 1 - prx, wlx);
        const bool straight = dx_end - dx == len - 1;
        int sxr;
        if (straight) {
            sxr = (dx + dx_end) * len / 2;
        } else {
            sxr = 0;
            for (int j = 0; j < len; ++j) sxr += wrap_off(x0 + a + j - prx, wlx);
        }
        atomicAdd(&pn[r], len);
        if (wt) {
            // the run's sites with their weights (the field row is read again)
            const float *frow = F.p[e] + (size_t)(y0 + y) * lx + x0 + a;
            long long swx = 0;
            int sw = 0;
            for (int j = 0; j < len; ++j) {
                const int w = site_weight(frow[j]);
                const int dxj = straight ? dx + j : wrap_off(x0 + a + j - prx, wlx);
                swx += (long long)w * dxj;
                sw += w;
            }
            atomicAdd((unsigned long long *)&wsx[r], (unsigned long long)swx);
            atomicAdd((unsigned long long *)&wsy[r], (unsigned long long)((long long)dy * sw));
            atomicAdd((unsigned long long *)&wsw[r], (unsigned long long)sw);
        } else {
            atomicAdd(&psx[r], sxr);
            atomicAdd(&psy[r], dy * len);
        }
        if (dy == hiy || !straight || (dx <= hix && hix <= dx_end)) {
            bool amb = false;
            const int gy = y0 + y;
            const int yp = gy + 1 == ly ? 0 : gy + 1, ym = gy == 0 ? ly - 1 : gy - 1;
            auto inside_at = [&](int xx, int yy) {
                const size_t tl = (size_t)(yy >> 5) * B.ntx + (xx >> 5);
                return gmem(B.lab16)[tl * DV_TILE_SITES + (yy & 31) * 32 + (xx & 31)] != 0xffff;
            };
            for (int j = 0; j < len; ++j) {
                const int gx = x0 + a + j;
                const int dxj = wrap_off(gx - prx, wlx);
                if (dxj != hix && dy != hiy) continue;
                const int xp = gx + 1 == lx ? 0 : gx + 1, xm = gx == 0 ? lx - 1 : gx - 1;
                if (dxj == hix) {
                    amb = amb || inside_at(xp, gy);
                    if (B.conn == 8) amb = amb || inside_at(xp, ym) || inside_at(xp, yp);
                }
                if (dy == hiy) {
                    amb = amb || inside_at(gx, yp);
                    if (B.conn == 8) amb = amb || inside_at(xm, yp) || inside_at(xp, yp);
                }
            }
            if (amb && prank[r] < B.kmax) atomicOr(&B.acc_amb[prank[r]], 1);
        }
    }
    __syncthreads();
    for (int k = t; k < np; k += DV_BLOCK) {
        const int rank = prank[k];
        if (rank >= B.kmax) continue;
        if (wt) {
            atomicAdd((unsigned long long *)&B.acc_x[rank], (unsigned long long)wsx[k]);
            atomicAdd((unsigned long long *)&B.acc_y[rank], (unsigned long long)wsy[k]);
            atomicAdd((unsigned long long *)&B.acc_w[rank], (unsigned long long)wsw[k]);
        } else {
            atomicAdd((unsigned long long *)&B.acc_x[rank], (unsigned long long)(long long)psx[k]);
            atomicAdd((unsigned long long *)&B.acc_y[rank], (unsigned long long)(long long)psy[k]);
        }
        atomicAdd(&B.acc_n[rank], pn[k]);
    }
}

}  // namespace

void launch_label(const Batch &G, const Fields &F, hipStream_t s, Prof &P) {
    P.begin(ST_TILE_CCL, s);
    if (G.geom) hipLaunchKernelGGL(k_tile_ccl<true>, dim3((G.tiles + 3) / 4), dim3(256), 0, s, G.D, G, F);
    else hipLaunchKernelGGL(k_tile_ccl<false>, dim3((G.tiles + 3) / 4), dim3(256), 0, s, G.D, G, F);
    P.end(ST_TILE_CCL, s);
    P.begin(ST_MERGE, s);
    const int merge_blocks = (G.tiles + 4 * MERGE_TILES - 1) / (4 * MERGE_TILES);
    if (G.geom) hipLaunchKernelGGL(k_merge<true>, dim3(merge_blocks), dim3(256), 0, s, G.D, G);
    else hipLaunchKernelGGL(k_merge<false>, dim3(merge_blocks), dim3(256), 0, s, G.D, G);
    P.end(ST_MERGE, s);
    P.begin(ST_RESOLVE, s);
    hipLaunchKernelGGL(k_resolve, dim3(G.bands), dim3(1024), 0, s, G.D, G);
    hipLaunchKernelGGL(k_bandpre, dim3(1, 1, G.n), dim3(1024), 0, s, G.D, G);
    hipLaunchKernelGGL(k_rank, dim3((G.tiles + 256 / RANK_LANES - 1) / (256 / RANK_LANES)), dim3(256), 0, s, G.D, G);
    P.end(ST_RESOLVE, s);
    P.begin(ST_RELABEL, s);
    if (G.weighted) {
        if (G.geom) hipLaunchKernelGGL((k_relabel<true, true>), dim3(G.tiles), dim3(DV_BLOCK), 0, s, G.D, G, F);
        else hipLaunchKernelGGL((k_relabel<false, true>), dim3(G.tiles), dim3(DV_BLOCK), 0, s, G.D, G, F);
    } else {
        if (G.geom) hipLaunchKernelGGL((k_relabel<true, false>), dim3(G.tiles), dim3(DV_BLOCK), 0, s, G.D, G, F);
        else hipLaunchKernelGGL((k_relabel<false, false>), dim3(G.tiles), dim3(DV_BLOCK), 0, s, G.D, G, F);
    }
    P.end(ST_RELABEL, s);
}
