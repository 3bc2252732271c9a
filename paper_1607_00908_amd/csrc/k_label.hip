// Cluster labelling and centre-of-mass sums (Sec. 3.1 of the paper).
//
// The lattice is cut into 32x32 tiles.  Per frame:
//   k_tile_ccl   threshold + union-find of each tile in LDS; every tile-border
//                site and every tile-local root ("piece") gets an entry in the
//                global parent array (global linear site indices);
//   k_merge      unions across tile borders and the periodic seams;
//   k_resolve    each piece finds its global root; component roots (which are
//                the smallest linear index of each component) are marked in a
//                bitmap of (row, tile column) segments;
//   k_rank_scan  per band of 32 rows: exclusive prefix of the root bits in
//                raster order -> canonical label of every root; K;
//   k_relabel    re-runs the tile union-find, writes canonical labels and
//                accumulates exact integer offsets from each component's root
//                (signed minimum image) per piece, then per component.
// Union-find always links the larger index under the smaller one, so the root
// of every tree is its smallest index.
#include "dv_internal.h"

namespace {

__device__ __forceinline__ bool is_in(float v, float thr, int phase) {
    return phase == 0 ? (v > thr) : (v < thr);
}

// ---- union-find in LDS over tile-local indices -----------------------------
__device__ __forceinline__ int lfind(const int *L, int a) {
    int p = L[a];
    while (p != a) { a = p; p = L[a]; }
    return a;
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
__device__ __forceinline__ int gfind(const int *P, int a) {
    int p = P[a];
    while (p != a) { a = p; p = P[a]; }
    return a;
}

__device__ void gunite(int *P, int a, int b) {
    bool done;
    do {
        a = gfind(P, a);
        b = gfind(P, b);
        if (a < b) {
            const int old = atomicMin(&P[b], a);
            done = (old == b);
            b = old;
        } else if (b < a) {
            const int old = atomicMin(&P[a], b);
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

// Labels the inside sites of one tile with tile-local union-find.  On return
// (after a barrier) L[s] is the smallest tile-local index of the piece of s,
// or -1 when s is outside or beyond the lattice.  rowm: LDS [32] row masks.
//
// Runs of a row are connected by construction (each site points to its run's
// first site).  Runs of consecutive rows are united once per touching pair:
// a site unites its run with the run above that starts to be adjacent at its
// responsibility column -- column x + 1 for every site, and additionally
// columns a - 1 and a for the first site a of a run (8-connectivity), or
// column x for every site (4-connectivity).
__device__ void tile_ccl(const Bufs &B, int x0, int y0, int tw, int th, int *L, uint32_t *rowm) {
    const int t = threadIdx.x, cx = t & 31, ry = t >> 5, lane = t & 63;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = ry + 8 * i;
        bool in = false;
        if (cx < tw && y < th)
            in = is_in(B.field[(size_t)(y0 + y) * B.lx + x0 + cx], B.thr, B.phase);
        const unsigned long long bal = __ballot(in);
        const uint32_t m = (uint32_t)(lane < 32 ? bal : (bal >> 32));
        if (cx == 0) rowm[y] = m;
        L[y * 32 + cx] = in ? y * 32 + run_start(m, cx) : -1;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = ry + 8 * i, s = y * 32 + cx;
        if (y == 0 || L[s] < 0) continue;
        const uint32_t m = rowm[y], up = rowm[y - 1];
        if (up == 0u) continue;
        const int a = run_start(m, cx);
        const int me = y * 32 + a;
        if (B.conn == 8) {
            const int lo = a > 0 ? a - 1 : 0;
            // candidate columns above: x + 1, plus a - 1 and a at the run start
            int cand[3] = {cx + 1, -1, -1};
            if (cx == a) { cand[1] = a - 1; cand[2] = a; }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int u = cand[k];
                if (u < lo || u > 31 || !((up >> u) & 1u)) continue;
                if (u > lo && ((up >> (u - 1)) & 1u)) continue;   // not the first of its run
                lunite(L, me, (y - 1) * 32 + run_start(up, u));
            }
        } else {
            const int u = cx;
            if ((up >> u) & 1u) {
                if (u == a || !((up >> (u - 1)) & 1u)) lunite(L, me, (y - 1) * 32 + run_start(up, u));
            }
        }
    }
    __syncthreads();
    // roots of the run starts, then every site takes its run start's root
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = ry + 8 * i, s = y * 32 + cx;
        if (L[s] == s || (L[s] >= 0 && L[s] < s && run_start(rowm[y], cx) == cx)) L[s] = lfind(L, s);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = ry + 8 * i, s = y * 32 + cx;
        if (L[s] >= 0) {
            const int st = y * 32 + run_start(rowm[y], cx);
            if (st != s) L[s] = L[st];
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(DV_BLOCK) void k_tile_ccl(Bufs B) {
    __shared__ int L[DV_TILE_SITES];
    __shared__ uint32_t rowm[DV_TILE];
    __shared__ int npc;
    const int tx = blockIdx.x, ty = blockIdx.y, tile = ty * B.ntx + tx;
    const int x0 = tx * DV_TILE, y0 = ty * DV_TILE;
    const int tw = min(DV_TILE, B.lx - x0), th = min(DV_TILE, B.ly - y0);
    const int t = threadIdx.x;
    DevState *st = B.st;
    const int now = 1 - st->sel;

    // per-frame resets spread over the grid
    if (tile == 0 && t == 0) {
        st->K_now = 0;
        st->err = 0;
        st->E2_now = 0;
        st->n_flips = 0;
        st->n_break = 0;
        st->n_excl_past = 0;
        st->n_excl_now = 0;
        st->n_amb = 0;
        st->global_trigger = 0;
    }
    if (t == 0) {
        B.cell_count[tile] = 0;
        if (tx == 0) B.band_sum[ty] = 0;
        npc = 0;
    }
    {   // empty the rows of the buffer this frame will fill
        const size_t total = (size_t)st->rows_dirty[now] * B.maxdeg;
        const size_t stride = (size_t)gridDim.x * gridDim.y * DV_BLOCK;
        int *adj = B.comp[now].adj;
        for (size_t i = (size_t)tile * DV_BLOCK + t; i < total; i += stride) adj[i] = DV_EMPTY;
    }

    tile_ccl(B, x0, y0, tw, th, L, rowm);

    const int cx = t & 31, ry = t >> 5;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = ry + 8 * i, s = y * 32 + cx;
        const int r = L[s];
        if (r < 0) continue;
        const int g = (y0 + y) * B.lx + x0 + cx;
        if (r == s) {
            const int slot = atomicAdd(&npc, 1);
            B.pieces[(size_t)tile * DV_TILE_SITES + slot] = (uint16_t)s;
            B.parent[g] = g;
        } else if (cx == 0 || y == 0 || cx == tw - 1 || y == th - 1) {
            B.parent[g] = (y0 + (r >> 5)) * B.lx + x0 + (r & 31);
        }
    }
    __syncthreads();
    if (t == 0) B.npieces[tile] = npc;
}

// Unions between inside sites of neighbouring tiles.  Thread j < 32 takes row
// j of the tile's last column against the next column (periodic); thread
// 32 + j takes column j of the last row against the next row.  Together they
// cover every adjacent pair that crosses a tile border, including the
// diagonal pairs at tile corners and the periodic seams.
__global__ __launch_bounds__(64) void k_merge(Bufs B) {
    const int tx = blockIdx.x, ty = blockIdx.y;
    const int x0 = tx * DV_TILE, y0 = ty * DV_TILE;
    const int tw = min(DV_TILE, B.lx - x0), th = min(DV_TILE, B.ly - y0);
    const int lx = B.lx, ly = B.ly;
    int j = threadIdx.x;
    if (j < 32) {
        if (j >= th) return;
        const int x = x0 + tw - 1, y = y0 + j;
        const int s = y * lx + x;
        if (!is_in(B.field[s], B.thr, B.phase)) return;
        const int xn = (x + 1 == lx) ? 0 : x + 1;
        for (int dy = -1; dy <= 1; ++dy) {
            if (B.conn == 4 && dy != 0) continue;
            int yn = y + dy;
            yn = yn < 0 ? yn + ly : (yn >= ly ? yn - ly : yn);
            const int u = yn * lx + xn;
            if (is_in(B.field[u], B.thr, B.phase)) gunite(B.parent, s, u);
        }
    } else {
        j -= 32;
        if (j >= tw) return;
        const int x = x0 + j, y = y0 + th - 1;
        const int s = y * lx + x;
        if (!is_in(B.field[s], B.thr, B.phase)) return;
        const int yn = (y + 1 == ly) ? 0 : y + 1;
        for (int dx = -1; dx <= 1; ++dx) {
            if (B.conn == 4 && dx != 0) continue;
            int xn = x + dx;
            xn = xn < 0 ? xn + lx : (xn >= lx ? xn - lx : xn);
            const int u = yn * lx + xn;
            if (is_in(B.field[u], B.thr, B.phase)) gunite(B.parent, s, u);
        }
    }
}

// Each piece finds its component root; roots are marked per segment.
__global__ __launch_bounds__(DV_BLOCK) void k_resolve(Bufs B) {
    __shared__ uint32_t mask[DV_TILE];
    __shared__ int nroot;
    const int tx = blockIdx.x, ty = blockIdx.y, tile = ty * B.ntx + tx;
    const int x0 = tx * DV_TILE, y0 = ty * DV_TILE;
    const int th = min(DV_TILE, B.ly - y0);
    const int t = threadIdx.x;
    if (t < DV_TILE) mask[t] = 0u;
    if (t == 0) nroot = 0;
    __syncthreads();
    const int np = B.npieces[tile];
    for (int i = t; i < np; i += DV_BLOCK) {
        const int r = B.pieces[(size_t)tile * DV_TILE_SITES + i];
        const int g = (y0 + (r >> 5)) * B.lx + x0 + (r & 31);
        const int root = gfind(B.parent, g);
        if (root != g) {
            B.parent[g] = root;
        } else {
            atomicOr(&mask[r >> 5], 1u << (r & 31));
            atomicAdd(&nroot, 1);
        }
    }
    __syncthreads();
    if (t < th) B.seg_mask[(size_t)(y0 + t) * B.ntx + tx] = mask[t];
    if (t == 0 && nroot) atomicAdd(&B.band_sum[ty], nroot);
}

// Exclusive prefix (raster order) of root bits, one block per band of rows.
// Segment (y, tile column c) covers sites y*lx + 32c .. 32c+31, so raster
// order of segments is the row-major order of the [ly][ntx] arrays.
__global__ __launch_bounds__(DV_BLOCK) void k_rank_scan(Bufs B) {
    __shared__ int wsum[DV_BLOCK / 64];
    __shared__ int s_off;
    const int ty = blockIdx.x, t = threadIdx.x;
    const int lane = t & 63, wid = t >> 6;
    const int y0 = ty * DV_TILE, th = min(DV_TILE, B.ly - y0);
    // offset of this band = roots in all earlier bands
    int part = 0;
    for (int b = t; b < ty; b += DV_BLOCK) part += B.band_sum[b];
    for (int o = 32; o > 0; o >>= 1) part += __shfl_down(part, o, 64);
    if (lane == 0) wsum[wid] = part;
    __syncthreads();
    if (t == 0) {
        int s = 0;
        for (int w = 0; w < DV_BLOCK / 64; ++w) s += wsum[w];
        s_off = s;
    }
    __syncthreads();
    int carry = s_off;
    const int n = th * B.ntx;
    const size_t base = (size_t)y0 * B.ntx;
    for (int c0 = 0; c0 < n; c0 += DV_BLOCK) {
        const int i = c0 + t;
        const int v = i < n ? __popc(B.seg_mask[base + i]) : 0;
        // inclusive scan within the wave
        int x = v;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        __syncthreads();
        if (lane == 63) wsum[wid] = x;
        __syncthreads();
        int before = carry;
        for (int w = 0; w < wid; ++w) before += wsum[w];
        if (i < n) B.seg_prefix[base + i] = before + x - v;
        int tot = 0;
        for (int w = 0; w < DV_BLOCK / 64; ++w) tot += wsum[w];
        carry += tot;
    }
    if (ty == B.nty - 1 && t == 0) {
        DevState *st = B.st;
        const int K = carry;
        st->K_now = K;
        if (K > B.kmax) st->err |= DV_E_KMAX;
        st->rows_dirty[1 - st->sel] = min(K, B.kmax);
    }
}

__device__ __forceinline__ int wrap_off(int v, int L) {
    // v in (-L, L) -> signed minimum image in [-floor(L/2), L-1-floor(L/2)]
    const int h = L >> 1;
    if (v > L - 1 - h) v -= L;
    else if (v < -h) v += L;
    return v;
}

__global__ __launch_bounds__(DV_BLOCK) void k_relabel(Bufs B) {
    __shared__ int L[DV_TILE_SITES];
    __shared__ int prank[DV_TILE_SITES];
    __shared__ int prx[DV_TILE_SITES], pry[DV_TILE_SITES];
    __shared__ int psx[DV_TILE_SITES], psy[DV_TILE_SITES], pn[DV_TILE_SITES];
    __shared__ uint8_t in34[34 * 34];
    __shared__ uint32_t rowm[DV_TILE];
    DevState *st = B.st;
    if (st->err) return;
    const int tx = blockIdx.x, ty = blockIdx.y, tile = ty * B.ntx + tx;
    const int x0 = tx * DV_TILE, y0 = ty * DV_TILE;
    const int tw = min(DV_TILE, B.lx - x0), th = min(DV_TILE, B.ly - y0);
    const int t = threadIdx.x, lx = B.lx, ly = B.ly;

    // inside flags of the tile and its one-site ring (periodic)
    for (int w = t; w < (tw + 2) * (th + 2); w += DV_BLOCK) {
        const int wx = w % (tw + 2) - 1, wy = w / (tw + 2) - 1;
        int gx = x0 + wx, gy = y0 + wy;
        gx = gx < 0 ? gx + lx : (gx >= lx ? gx - lx : gx);
        gy = gy < 0 ? gy + ly : (gy >= ly ? gy - ly : gy);
        in34[(wy + 1) * 34 + wx + 1] = is_in(B.field[(size_t)gy * lx + gx], B.thr, B.phase) ? 1 : 0;
    }
    tile_ccl(B, x0, y0, tw, th, L, rowm);

    const int np = B.npieces[tile];
    for (int i = t; i < np; i += DV_BLOCK) {
        const int r = B.pieces[(size_t)tile * DV_TILE_SITES + i];
        const int g = (y0 + (r >> 5)) * lx + x0 + (r & 31);
        const int G = B.parent[g];          // component root (compressed)
        const int gx = G % lx, gy = G / lx;
        const size_t seg = (size_t)gy * B.ntx + (gx >> 5);
        const uint32_t below = (1u << (gx & 31)) - 1u;
        const int rank = B.seg_prefix[seg] + __popc(B.seg_mask[seg] & below);
        prank[r] = rank;
        prx[r] = gx;
        pry[r] = gy;
        psx[r] = 0;
        psy[r] = 0;
        pn[r] = 0;
        if (G == g && rank < B.kmax) B.acc_root[rank] = G;
    }
    __syncthreads();

    const int cx = t & 31, ry = t >> 5;
    const int hix = lx - 1 - (lx >> 1), hiy = ly - 1 - (ly >> 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = ry + 8 * i, s = y * 32 + cx;
        if (cx >= tw || y >= th) continue;
        const int r = L[s];
        const size_t g = (size_t)(y0 + y) * lx + x0 + cx;
        if (B.keep_maps) B.labels[g] = r >= 0 ? prank[r] : -1;
        if (r < 0) continue;
        const int dx = wrap_off(x0 + cx - prx[r], lx);
        const int dy = wrap_off(y0 + y - pry[r], ly);
        atomicAdd(&psx[r], dx);
        atomicAdd(&psy[r], dy);
        atomicAdd(&pn[r], 1);
        // an adjacent inside site is a member; crossing the antipodal line of
        // the root makes the unwrapped coordinates jump by L - 1
        bool amb = false;
        const int w = (y + 1) * 34 + cx + 1;
        if (dx == hix) {
            if (B.conn == 8) amb = in34[w - 34 + 1] | in34[w + 1] | in34[w + 34 + 1];
            else amb = in34[w + 1];
        }
        if (dy == hiy) {
            if (B.conn == 8) amb |= in34[w + 34 - 1] | in34[w + 34] | in34[w + 34 + 1];
            else amb |= in34[w + 34];
        }
        if (amb && prank[r] < B.kmax) atomicOr(&B.acc_amb[prank[r]], 1);
    }
    __syncthreads();
    for (int i = t; i < np; i += DV_BLOCK) {
        const int r = B.pieces[(size_t)tile * DV_TILE_SITES + i];
        const int rank = prank[r];
        if (rank >= B.kmax) continue;
        atomicAdd((unsigned long long *)&B.acc_x[rank], (unsigned long long)(long long)psx[r]);
        atomicAdd((unsigned long long *)&B.acc_y[rank], (unsigned long long)(long long)psy[r]);
        atomicAdd(&B.acc_n[rank], pn[r]);
    }
}

}  // namespace

void launch_label(const Bufs &B, hipStream_t s, Prof &P) {
    const dim3 tiles(B.ntx, B.nty);
    P.begin(ST_TILE_CCL, s);
    hipLaunchKernelGGL(k_tile_ccl, tiles, dim3(DV_BLOCK), 0, s, B);
    P.end(ST_TILE_CCL, s);
    P.begin(ST_MERGE, s);
    hipLaunchKernelGGL(k_merge, tiles, dim3(64), 0, s, B);
    P.end(ST_MERGE, s);
    P.begin(ST_RESOLVE, s);
    hipLaunchKernelGGL(k_resolve, tiles, dim3(DV_BLOCK), 0, s, B);
    P.end(ST_RESOLVE, s);
    P.begin(ST_RANK_SCAN, s);
    hipLaunchKernelGGL(k_rank_scan, dim3(B.nty), dim3(DV_BLOCK), 0, s, B);
    P.end(ST_RANK_SCAN, s);
    P.begin(ST_RELABEL, s);
    hipLaunchKernelGGL(k_relabel, tiles, dim3(DV_BLOCK), 0, s, B);
    P.end(ST_RELABEL, s);
}
