// Centres, bucket grid, digital Voronoi colouring and Delaunay couples
// (Sec. 3.1 last step, Sec. 3.2.1 and Sec. 3.2.2 of the paper).
//
//   k_finalize      exact Q.8 and float64 centres from the integer sums;
//                   counts the centres of each bucket cell
//   k_grid          one block per frame builds the grid (cell offsets,
//                   centres by cell)
//   k_owner_edges   one block per tile: candidate centres from the grid,
//                   nearest centre of every site of the tile and its one-site
//                   ring (LDS), owner map, frame-gap vertex test and the first /
//                   second nearest-neighbour rules; the distinct couples of the
//                   tile go to the tile's couple list
//   k_rows          the couple lists into the adjacency rows with a lock-free
//                   set insert (rows are unordered sets, MAXLINK padded)
#include "dv_device.h"

namespace {

__device__ __forceinline__ long long floor_div(long long a, long long b) {
    long long q = a / b;
    if ((a % b) != 0 && a < 0) q -= 1;
    return q;
}

__device__ __forceinline__ long long pmod64(long long v, long long m) {
    const long long r = v % m;
    return r < 0 ? r + m : r;
}

// floor(256 S / W + 1/2) for W > 0 without forming 512 S (a weighted sum can
// use most of the 64 bits): with S = q W + r, 0 <= r < W, it is
// 256 q + floor((512 r + W) / (2 W)), and 512 r stays far below 2^63.
__device__ __forceinline__ long long q8_round(long long S, long long W) {
    const long long q = floor_div(S, W), r = S - q * W;
    return 256 * q + (512 * r + W) / (2 * W);
}

__global__ __launch_bounds__(1024) void k_finalize(const Bufs *__restrict__ D, Batch G) {
    const Bufs B = D[G.idx[blockIdx.z]];
    FrameState *fs = B.fs;
    const bool ok = fs->err == 0;
    const int K = fs->K_now;
    const CompBuf C = B.cur;
    const int t = threadIdx.x;
    if (ok) {
        int namb = 0;
        for (int k = blockIdx.x * blockDim.x + t; k < K; k += gridDim.x * blockDim.x) {
            const long long n = B.acc_n[k], sx = B.acc_x[k], sy = B.acc_y[k];
            const int root = B.acc_root[k], amb = B.acc_amb[k];
            B.acc_n[k] = 0;
            B.acc_x[k] = 0;
            B.acc_y[k] = 0;
            B.acc_amb[k] = 0;
            const int rx = root % B.lx, ry = root / B.lx;
            // weighted centres divide by the total weight, the others by n
            long long W = n;
            if (B.weighted) {
                W = B.acc_w[k];
                B.acc_w[k] = 0;
            }
            const int qx = (int)pmod64(256LL * rx + q8_round(sx, W), 256LL * B.lx);
            const int qy = (int)pmod64(256LL * ry + q8_round(sy, W), 256LL * B.ly);
            double fx = (double)rx + (double)sx / (double)W;
            double fy = (double)ry + (double)sy / (double)W;
            if (fx < 0) fx += B.lx; else if (fx >= B.lx) fx -= B.lx;
            if (fy < 0) fy += B.ly; else if (fy >= B.ly) fy -= B.ly;
            C.qx[k] = qx;
            C.qy[k] = qy;
            C.fx[k] = fx;
            C.fy[k] = fy;
            C.n[k] = (int)n;
            C.root[k] = root;
            C.amb[k] = amb;
            namb += amb;
            const int cell = (qy >> 13) * B.ntx + (qx >> 13);
            B.comp_cell[k] = cell;
            B.comp_slot[k] = atomicAdd(&B.cell_count[cell], 1);
            B.cnt[k] = 0;
            B.inv[k] = -1;
        }
        if (namb) atomicAdd(&fs->n_amb, namb);
    } else {
        // a rejected frame still leaves the sums it accumulated (ranks below
        // K_max) empty for the next frame
        const int KK = min(K, B.kmax);
        for (int k = blockIdx.x * blockDim.x + t; k < KK; k += gridDim.x * blockDim.x) {
            B.acc_n[k] = 0;
            B.acc_x[k] = 0;
            B.acc_y[k] = 0;
            B.acc_amb[k] = 0;
            if (B.weighted) B.acc_w[k] = 0;
        }
    }
}

// One block per frame: the bucket grid from the cell counts (offsets, centres
// by cell).  (A kernel of its own: a last-block ticket in k_finalize would
// need a device-wide release in every block.)
__global__ __launch_bounds__(1024) void k_grid(const Bufs *__restrict__ D, Batch G) {
    const Bufs B = D[G.idx[blockIdx.z]];
    __shared__ int wsum[16];
    const FrameState *fs = B.fs;
    if (fs->err) return;
    const int K = fs->K_now, t = threadIdx.x;
    const CompBuf C = B.cur;
    // (contiguous runs of up to 16 counts per thread: one pass for up to
    // 16384 cells)
    const int total = block_exclusive_scan_wide<16>(B.cell_count, B.cell_start, B.ncells, wsum);
    if (t == 0) B.cell_start[B.ncells] = total;
    __syncthreads();
#pragma unroll 4
    for (int k = t; k < K; k += blockDim.x) {
        const int pos = B.cell_start[B.comp_cell[k]] + B.comp_slot[k];
        B.cell_items[pos] = k;
        B.cell_q[pos] = make_int2(C.qx[k], C.qy[k]);
    }
}

// Frame of a site (Sec. 3.2.2), cyclic: spx, spxpy, spy, spymx, smx, smxmy,
// smy, smypx; inner-frame points a_k, b_k, c_k, d_k at (+-1/2, +-1/2) in Q.8.
// Written as expressions so that no table is read from memory.
__device__ __forceinline__ int frx(int k) { return (k == 0 || k == 1 || k == 7) ? 1 : (k == 2 || k == 6) ? 0 : -1; }
__device__ __forceinline__ int fry(int k) { return (k == 1 || k == 2 || k == 3) ? 1 : (k == 0 || k == 4) ? 0 : -1; }
__device__ __forceinline__ int inx(int r) { return (r == 1 || r == 2) ? -128 : 128; }
__device__ __forceinline__ int iny(int r) { return r >= 2 ? -128 : 128; }

// Lock-free set insert into a row (slots fill from the front; DV_EMPTY marks
// free slots).  Rows are 16-byte aligned (max_degree is a multiple of 4), so
// four slots are read per load.
__device__ __forceinline__ void row_insert(gint *row, int maxdeg, int v, FrameState *fs) {
    for (int i = 0; i < maxdeg; i += 4) {
        const dv_v4i q = *reinterpret_cast<const __attribute__((address_space(1))) dv_v4i *>(row + i);
        const int e[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (e[j] == v) return;
            if (e[j] == DV_EMPTY) {
                // claim the first free slot; on a lost race re-examine it
                for (int k = i + j; k < maxdeg; ++k) {
                    int old = DV_EMPTY;
                    __hip_atomic_compare_exchange_strong(row + k, &old, v, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (old == DV_EMPTY || old == v) return;
                }
                atomicOr(&fs->err, DV_E_DEGREE);
                return;
            }
        }
    }
    atomicOr(&fs->err, DV_E_DEGREE);
}

typedef short sh2 __attribute__((ext_vector_type(2)));   // packed 16-bit pair

// a.x b.x + a.y b.y + c on signed 16-bit pairs, exact in 32 bits.  Written
// as the three-operand instruction: the compiler's form of the builtin
// accumulates into its destination, which costs a copy of c for every use
// when c is shared by several products.
__device__ __forceinline__ int dot2_acc(sh2 a, sh2 b, int c) {
    int d;
    asm("v_dot2_i32_i16 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

#define PAIR_CAP 256    // couples a tile can collect in LDS before writing through
#define TMP_CAP 128     // centres kept from the first pass

#define WSITES 5      // ceil(34*34 / 256) window sites per thread
#define RCAP 256      // item ranges held in LDS per batch
#define IMG_MAX 9     // periodic images one centre can contribute (tiny lattices)
#define CAND_BATCH 8  // centres appended per batch (room for IMG_MAX images each)

// Shared state of one colouring tile.
struct OwnerLds {
    int own[34 * 34];
    // candidate centres as appended: tile-relative Q.8 image positions, label
    int cx[DV_CAND_CAP], cy[DV_CAND_CAP];
    int lab[DV_CAND_CAP];
    // the kept ones, ordered by label for evaluation: x, y, |c|^2 as doubles,
    // or as 32-bit integers when every kept one is near the tile (imode)
    union {
        struct { double sx[DV_CAND_CAP], sy[DV_CAND_CAP], sk[DV_CAND_CAP]; };
        // (ixy: x in the low 16 bits, y in the high 16, for the packed dot product)
        struct { int ixy[DV_CAND_CAP], ik[DV_CAND_CAP]; };
    };
    int sl[DV_CAND_CAP];
    uint8_t keep[DV_CAND_CAP];   // the candidate is not beaten everywhere in the window
    int nkeep;                   // candidates kept (the ordered list's length)
    int fast;                    // the one-pass candidate list of the usual case was built
    int far;                     // some kept candidate is beyond the 32-bit range
    int imode;                   // the ordered list holds 32-bit integers
    int ncand;
    int nchunks;   // times the list was evaluated and emptied before the end
    // item ranges of the cell rectangle being visited
    int r_e0[RCAP], r_pre[RCAP + 1];
    int nranges;
    unsigned long long best;
    int wsum[16];
    // centres seen in the first pass: label, Q.8 centre, squared distance
    // to the tile centre
    int tmp[TMP_CAP];
    union {
        int2 tmpq[TMP_CAP];
        // (after the candidate list is built) inner-frame queries of each
        // thread's sites, bit 4i + r as in the thread's own mask
        unsigned pendw[DV_BLOCK];
    };
    long long tmpd[TMP_CAP];
    int ntmp;
    int nout;      // distinct couples written to the tile's list
    // couples found by the tile, (a << 32 | b) with a < b
    unsigned long long pair[PAIR_CAP];
    int npair;
};

// Visit every item (index into the cell-ordered centre arrays) of the cells
// in rows sy x column ranges sx.  fn(e) is called by the block's threads in
// parallel, in batches of at most `batch` items; before each batch every
// thread calls before(m) with the batch size m (uniform control flow; all
// earlier fn calls have completed).
template <class Fn, class Before>
__device__ void visit_items(const Bufs &B, OwnerLds &S, const Span &sx, const Span &sy, int batch,
                            Fn fn, Before before) {
    const int t = threadIdx.x;
    const auto cs = gmem(B.cell_start);
    // rows of the rectangle, enumerated in order
    int nrows = 0;
    for (int i = 0; i < sy.n; ++i) nrows += sy.hi(i) - sy.lo(i) + 1;
    const int per_row = sx.n;
    for (int rb = 0; rb < nrows; rb += RCAP / 2) {
        const int nr = min(RCAP / 2, nrows - rb);
        const int nrng = nr * per_row;
        // range j -> (row index rb + j / per_row, column range j % per_row)
        int cnt = 0;
        if (t < nrng) {
            int ri = rb + t / per_row;
            const int n0 = sy.hi0 - sy.lo0 + 1;
            const int row = (ri < n0) ? sy.lo0 + ri : sy.lo1 + (ri - n0);
            const int c = t % per_row;
            const int e0 = cs[row * B.ntx + sx.lo(c)], e1 = cs[row * B.ntx + sx.hi(c) + 1];
            S.r_e0[t] = e0;
            cnt = e1 - e0;
        }
        // exclusive scan of the counts (nrng <= RCAP / 2 * 2 <= blockDim)
        {
            const int lane = t & 63, wid = t >> 6;
            const int x = wave_incl_sum(cnt);
            if (lane == 63) S.wsum[wid] = x;
            __syncthreads();
            int before = 0;
            for (int w = 0; w < wid; ++w) before += S.wsum[w];
            if (t < RCAP) S.r_pre[t] = before + x - cnt;
            if (t == (int)blockDim.x - 1) S.r_pre[RCAP] = before + x;
            __syncthreads();
        }
        const int total = S.r_pre[RCAP];
        for (int f0 = 0; f0 < total; f0 += batch) {
            const int m = min(batch, total - f0);
            before(m);
            for (int j = t; j < m; j += blockDim.x) {
                const int f = f0 + j;
                // range holding flat index f: last j with pre[j] <= f
                int lo = 0, hi = nrng - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (S.r_pre[mid] <= f) lo = mid; else hi = mid - 1;
                }
                fn(S.r_e0[lo] + (f - S.r_pre[lo]));
            }
            __syncthreads();
        }
    }
}

// Eight resident blocks per CU (register budget 64, 18.8 KB of LDS): the
// block's gather and barrier-bounded phases are latency chains that other
// resident blocks fill, which pays for the values that spill.
// GEOM: some entry of the launch has walls or obstacles; the periodic,
// unobstructed instance carries none of their tests.
template <bool GEOM>
__global__ __launch_bounds__(DV_BLOCK, 8) void k_owner_edges(const Bufs *__restrict__ D, Batch G) {
    const int e = entry_of(G.tbase, G.tpe, G.n, blockIdx.x);
    const Bufs &B = D[G.idx[e]];
    const int tile = blockIdx.x - G.tbase[e];
    __shared__ OwnerLds S;
    const int tx = tile % B.ntx, ty = tile / B.ntx;
    const bool ox = GEOM && B.open_x, oy = GEOM && B.open_y;
    // The usual candidate search reads the centres of the 7 x 7 cells around
    // the tile: first the bounds of their cell ranges (each row of cells of a
    // column span is one contiguous range of the cell-ordered arrays, at
    // most 7 x 2 ranges, a lane each in the first wave), then the centres.
    // The bounds are requested before anything else, so that their round
    // trip overlaps the frame header's.
    const int R0 = 3;
    const Span sx0 = span_cells(tx, R0, B.ntx, ox), sy0 = span_cells(ty, R0, B.nty, oy);
    const int n0y = sy0.hi0 - sy0.lo0 + 1, ncy = n0y + (sy0.n == 2 ? sy0.hi1 - sy0.lo1 + 1 : 0);
    const int nrng = ncy * sx0.n;
    int rb0 = 0, rb1 = 0;
    if ((int)threadIdx.x < nrng) {
        const int iy = threadIdx.x / sx0.n, c = threadIdx.x - iy * sx0.n;
        const int celly = iy < n0y ? sy0.lo0 + iy : sy0.lo1 + (iy - n0y);
        const auto cs = gmem(B.cell_start);
        rb0 = cs[celly * B.ntx + sx0.lo(c)];
        rb1 = cs[celly * B.ntx + sx0.hi(c) + 1];
    }
    FrameState *fs = B.fs;
    if (*gmem(&fs->err)) return;
    const int K = *gmem(&fs->K_now);
    gint *adj = gmem(B.cur.adj);
    const int x0 = tx * DV_TILE, y0 = ty * DV_TILE;
    const int tw = min(DV_TILE, B.lx - x0), th = min(DV_TILE, B.ly - y0);
    const int W = tw + 2, H = th + 2;
    const int t = threadIdx.x, lx = B.lx, ly = B.ly;
    // wrap periods (Q.8): the lattice period of a periodic axis; on a walled
    // axis a period that no distance reaches (images are not used there)
    const int MX = qperiod(lx, ox), MY = qperiod(ly, oy);
    const int OX = 256 * x0, OY = 256 * y0;   // tile origin (Q.8); coordinates below are relative

    // window sites of this thread: exact tile-relative Q.8 coordinates
    // (best value, owner) of the thread's window sites w = t + 256 i; the
    // site coordinates are rebuilt where needed (w / W by a multiply: w <
    // 1280 and W <= 34, so the 16-bit reciprocal is exact).  The float64
    // values are set by the first evaluation that uses them.
    double be[WSITES];
    int bl[WSITES];
    const int wmagic = (65536 + W - 1) / W;
#pragma unroll
    for (int i = 0; i < WSITES; ++i) bl[i] = DV_EMPTY;
    // the same sites as packed pairs wx | wy << 16: the first by the
    // reciprocal, each next one by adding 256 = wq W + wr (with a carry into
    // the row when wx reaches W)
    const int wq = DV_BLOCK / W, wr = DV_BLOCK - wq * W;
    auto site_pairs = [&](int P[WSITES]) {
        const int wy0 = (t * wmagic) >> 16;
        P[0] = (t - wy0 * W) | (wy0 << 16);
#pragma unroll
        for (int i = 1; i < WSITES; ++i) {
            const int q = P[i - 1] + (wr | (wq << 16));
            P[i] = (q & 0xffff) >= W ? q + (1 << 16) - W : q;
        }
    };
    // (the first wave reads these in program order, the others only after a
    // later barrier)
    if (t == 0) { S.ncand = 0; S.nchunks = 0; S.best = ~0ull; S.npair = 0; S.ntmp = 0; S.nout = 0; S.nkeep = 0; S.imode = 0; }

    // tile centre (absolute Q.8) and the window's relative x / y extent
    const int tcx = OX + 128 * (tw - 1), tcy = OY + 128 * (th - 1);
    const int wxlo = -256, wxhi = 256 * tw, wylo = -256, wyhi = 256 * th;

    // Nearest candidate of every window site.  Candidates that another
    // candidate beats everywhere in the window are dropped first: the
    // difference of the squared distances to two centres is affine in the
    // point, so when its minimum over the window rectangle (at the corner its
    // gradient picks) is positive, the other centre is strictly nearer at
    // every window site and inner-frame point, and the dropped one owns none
    // of them.  Some candidate always stays (strict domination has a minimal
    // element), and so does the owner of every point.  The test is exact in
    // float64: coordinates stay below 2^26 in magnitude (Q.8, images
    // included), so every square and sum is an integer below 2^53, and where
    // rounding could occur the value is far from zero.  The kept candidates
    // are ordered by label, so that a strict comparison already sends ties to
    // the lowest label; a later chunk (after an overflow) also compares
    // labels.
    // In the usual case every kept candidate lies within 23170 Q.8 units
    // (about 90 sites) of the tile origin on both axes: then |c|^2 < 2^30,
    // each product of a coordinate with a doubled point coordinate (at most
    // 16384 in magnitude) fits 24-bit operands, and every value below stays
    // inside 32-bit range, so the same exact comparison runs on integers.
    // That applies to the only evaluation of a tile (no overflow chunks);
    // otherwise the float64 form is used.
    auto eval_owners = [&](bool last, bool inited) {
        if (!inited) {
            if (t == 0) { S.nkeep = 0; S.far = 0; }
            __syncthreads();
        }
        const int nc = min(S.ncand, DV_CAND_CAP);
        if (nc <= 16) {   // the first wave: 4 lanes per candidate i, lane j of the group
                          // takes the rivals j, j + 4, ...
            if (t < 64) {
                const int i = t >> 2, gj = t & 3;
                bool beaten = false;
                if (i < nc) {
                    const double cx = (double)S.cx[i], cy = (double)S.cy[i];
                    const double cc = fma(cx, cx, cy * cy);
#pragma unroll 1
                    for (int j = gj; j < nc && !beaten; j += 4) {
                        if (j == i) continue;
                        const double jx = (double)S.cx[j], jy = (double)S.cy[j];
                        const double ax = 2.0 * (jx - cx), ay = 2.0 * (jy - cy);
                        const double f = fma(ax, ax >= 0.0 ? (double)wxlo : (double)wxhi,
                                             fma(ay, ay >= 0.0 ? (double)wylo : (double)wyhi,
                                                 cc - fma(jx, jx, jy * jy)));
                        beaten = f > 0.0;
                    }
                }
                const unsigned long long b = __ballot(beaten);
                const unsigned grp = (unsigned)(b >> (t & 60)) & 0xfu;
                const bool kept = gj == 0 && i < nc && !grp;
                if (gj == 0 && i < nc) S.keep[i] = grp ? 0 : 1;
                const bool farc = kept && (abs(S.cx[i]) > 23170 || abs(S.cy[i]) > 23170);
                const int nkept = __popcll(__ballot(kept));
                const bool anyfar = __ballot(farc) != 0ull;
                if (t == 0) {
                    S.nkeep = nkept;
                    S.far = anyfar ? 1 : 0;
                }
            }
        } else {   // 16 lanes per candidate i, lane j of the group takes the rivals j, j + 16, ...
            const int gi = t >> 4, gj = t & 15;
#pragma unroll 1
            for (int i0 = 0; i0 < nc; i0 += DV_BLOCK / 16) {
                const int i = i0 + gi;
                bool beaten = false;
                if (i < nc) {
                    const double cx = (double)S.cx[i], cy = (double)S.cy[i];
                    const double cc = fma(cx, cx, cy * cy);
#pragma unroll 1
                    for (int j = gj; j < nc && !beaten; j += 16) {
                        if (j == i) continue;
                        const double jx = (double)S.cx[j], jy = (double)S.cy[j];
                        // |w - c|^2 - |w - j|^2 = 2 w.(j - c) + |c|^2 - |j|^2
                        const double ax = 2.0 * (jx - cx), ay = 2.0 * (jy - cy);
                        const double f = fma(ax, ax >= 0.0 ? (double)wxlo : (double)wxhi,
                                             fma(ay, ay >= 0.0 ? (double)wylo : (double)wyhi,
                                                 cc - fma(jx, jx, jy * jy)));
                        beaten = f > 0.0;
                    }
                }
                const unsigned long long b = __ballot(beaten);
                const unsigned grp = (unsigned)(b >> (t & 48)) & 0xffffu;
                if (gj == 0 && i < nc) {
                    S.keep[i] = grp ? 0 : 1;
                    if (!grp) {
                        atomicAdd(&S.nkeep, 1);
                        if (abs(S.cx[i]) > 23170 || abs(S.cy[i]) > 23170) S.far = 1;
                    }
                }
            }
        }
        __syncthreads();
        const bool im = last && S.nchunks == 0 && !S.far;
        // kept candidate c with label lab goes to position r of the ordered list
        auto place = [&](int c, int r, int lab) {
            const int ix = S.cx[c], iy = S.cy[c];
            if (im) {
                S.ixy[r] = (int)(((unsigned)iy << 16) | ((unsigned)ix & 0xffffu));
                S.ik[r] = ix * ix + iy * iy;
            } else {
                const double x = (double)ix, y = (double)iy;
                S.sx[r] = x;
                S.sy[r] = y;
                S.sk[r] = x * x + y * y;
            }
            S.sl[r] = lab;
        };
        if (nc <= 64) {
            // the first wave, lane c holding candidate c: its position counts
            // the kept candidates before it by (label, index), visited one
            // kept candidate at a time
            if (t < 64) {
                const bool kc = t < nc && S.keep[t];
                const int lab = t < nc ? S.lab[t] : 0;
                int r = 0;
                for (unsigned long long m = __ballot(kc); m; m &= m - 1) {
                    const int j = (int)__builtin_ctzll(m);
                    const int l2 = __builtin_amdgcn_readlane(lab, j);
                    r += (l2 < lab || (l2 == lab && j < t)) ? 1 : 0;
                }
                if (kc) place(t, r, lab);
            }
        } else {
            for (int c = t; c < nc; c += DV_BLOCK) {
                if (!S.keep[c]) continue;
                const int lab = S.lab[c];
                int r = 0;
                for (int j = 0; j < nc; ++j) {
                    const int l2 = S.lab[j];
                    r += (S.keep[j] && (l2 < lab || (l2 == lab && j < c))) ? 1 : 0;
                }
                place(c, r, lab);
            }
        }
        if (t == 0) S.imode = im ? 1 : 0;
        __syncthreads();
        const int nk = S.nkeep;
        if (im) {
            // the only evaluation: strict comparison, ties to the first (lowest
            // label).  -2 w and the candidate are 16-bit pairs (|2 w| <= 16384,
            // |c| <= 23170), so e = -2 w . c + |c|^2 is one packed dot product
            // with exact 32-bit accumulation
            sh2 m2[WSITES];
            int bi[WSITES];
            {
                int P[WSITES];
                site_pairs(P);
#pragma unroll
                for (int i = 0; i < WSITES; ++i) {
                    // (-512 (wx - 1), -512 (wy - 1)) = ((1, 1) - (wx, wy)) * 512
                    m2[i] = (sh2{1, 1} - __builtin_bit_cast(sh2, P[i])) * (short)512;
                    bi[i] = INT_MAX;
                }
            }
            // candidates in order, two per step (the compiler does not unroll
            // a loop around inline assembly)
            auto cand = [&](int c) {
                const sh2 cq = __builtin_bit_cast(sh2, S.ixy[c]);
                const int kk = S.ik[c];
                const int lab = S.sl[c];
#pragma unroll
                for (int i = 0; i < WSITES; ++i) {
                    const int e = dot2_acc(m2[i], cq, kk);
                    const bool lt = e < bi[i];
                    bi[i] = lt ? e : bi[i];
                    bl[i] = lt ? lab : bl[i];
                }
            };
            int c = 0;
            for (; c + 1 < nk; c += 2) {
                cand(c);
                cand(c + 1);
            }
            if (c < nk) cand(c);
            return;
        }
        double m2x[WSITES], m2y[WSITES];
#pragma unroll
        for (int i = 0; i < WSITES; ++i) {
            const int w = t + i * DV_BLOCK;
            const int wy = (w * wmagic) >> 16, wx = w - wy * W;
            m2x[i] = -512.0 * (wx - 1);
            m2y[i] = -512.0 * (wy - 1);
        }
        if (S.nchunks == 0) {
#pragma unroll
            for (int i = 0; i < WSITES; ++i) be[i] = 1.0e300;
            for (int c = 0; c < nk; ++c) {
                const double cx = S.sx[c], cy = S.sy[c], kk = S.sk[c];
                const int lab = S.sl[c];
#pragma unroll
                for (int i = 0; i < WSITES; ++i) {
                    const double e = fma(m2x[i], cx, fma(m2y[i], cy, kk));
                    const bool lt = e < be[i];
                    be[i] = lt ? e : be[i];
                    bl[i] = lt ? lab : bl[i];
                }
            }
        } else {
            for (int c = 0; c < nk; ++c) {
                const double cx = S.sx[c], cy = S.sy[c], kk = S.sk[c];
                const int lab = S.sl[c];
#pragma unroll
                for (int i = 0; i < WSITES; ++i) {
                    const double e = fma(m2x[i], cx, fma(m2y[i], cy, kk));
                    if (e < be[i] || (e == be[i] && lab < bl[i])) { be[i] = e; bl[i] = lab; }
                }
            }
        }
    };

    // candidate list entry for centre e: every image of the centre that is the
    // minimum image of some window point (relative offset within [-M/2, M/2]).
    // The offset rx lies in (-MX, MX) and the window is at most one lattice
    // wide, so only the images k = -1 .. 2 can qualify.  On a walled axis
    // (M = 512 L) the centre itself always qualifies and a shifted copy only
    // for a centre on the first or last site line, seen from the tile at the
    // other wall: that copy is farther than the centre from every point inside
    // the domain (the only points whose colour is used), so it owns none.
    auto image_masks = [&](int rx, int ry, unsigned &mxk, unsigned &myk) {
        mxk = 0;
        myk = 0;
#pragma unroll
        for (int k = -1; k <= 2; ++k) {
            const int vx = rx + k * MX, vy = ry + k * MY;
            if (vx >= wxlo - MX / 2 && vx <= wxhi + MX / 2) mxk |= 1u << (k + 1);
            if (vy >= wylo - MY / 2 && vy <= wyhi + MY / 2) myk |= 1u << (k + 1);
        }
    };
    auto add_images = [&](int lab, int2 q) {
        const int rx = q.x - OX, ry = q.y - OY;
        unsigned mxk, myk;
        image_masks(rx, ry, mxk, myk);
        for (unsigned a = mxk; a; a &= a - 1) {
            const int cx = rx + (__ffs(a) - 2) * MX;
            for (unsigned b = myk; b; b &= b - 1) {
                const int cy = ry + (__ffs(b) - 2) * MY;
                const int slot = atomicAdd(&S.ncand, 1);
                if (slot >= DV_CAND_CAP) continue;   // overflow: caller falls back
                S.cx[slot] = cx;
                S.cy[slot] = cy;
                S.lab[slot] = lab;
            }
        }
    };
    // radius around the tile centre that holds every centre able to own a
    // window site or inner-frame point: bound + twice the window's half diagonal
    auto hdiag2 = [&]() {
        const double hx = 0.5 * (tw + 1), hy = 0.5 * (th + 1);
        return 2.0 * sqrt(hx * hx + hy * hy) + 2.0;
    };

    if (K > 0) {
        // --- usual case, one pass by the first wave: the 7x7 cells around the
        // tile give a bound (nearest centre seen) and, when they cover the
        // radius it implies, every candidate as well; the other waves wait at
        // the barrier
        if (t < 64) {
            // the centres of the square's cells, lane-parallel: one centre per
            // lane over the concatenated ranges whose bounds were requested
            // at the start; the bound is one wave minimum
            const int e0 = rb0, cnt = rb1 - rb0;
            const int inc = wave_incl_sum(cnt);
            const int total = wave_last(inc);
            const int pre = inc - cnt;
            unsigned long long dmin = ~0ull;
            // the lane's item of the first 64 stays in registers; later ones
            // (more than 64 centres in the square) go to LDS
            int2 q0 = make_int2(0, 0);
            int lab0 = 0;
            long long d0 = 0;
            for (int f0 = 0; f0 < total; f0 += 64) {
                const int f = f0 + t;
                // range of item f: the last one whose exclusive prefix is <= f
                int r = 0;
                for (int k = 1; k < nrng; ++k) r = __builtin_amdgcn_readlane(pre, k) <= f ? k : r;
                const int e = __shfl(e0, r, 64) + f - __shfl(pre, r, 64);
                if (f < total) {
                    const int2 q = ld_int2(B.cell_q, e);
                    const int lab = gmem(B.cell_items)[e];
                    const long long d = d2q(tcx, tcy, q.x, q.y, MX, MY);
                    dmin = min(dmin, (unsigned long long)d);
                    if (f0 == 0) {
                        q0 = q;
                        lab0 = lab;
                        d0 = d;
                    } else if (f < TMP_CAP) {
                        S.tmp[f] = lab;
                        S.tmpq[f] = q;
                        S.tmpd[f] = d;
                    }
                }
            }
            dmin = wave_min_u64(dmin);
            // the bound covers the candidates' radius: the list is built here
            bool fast = dmin != ~0ull && total <= TMP_CAP;
            double rq2 = 0.0;
            if (fast) {
                const double rho = sqrt((double)dmin) / 256.0 + hdiag2();
                const int wlx = lx - DV_TILE * (B.ntx - 1), wly = ly - DV_TILE * (B.nty - 1);
                const double cov_x = span_full(sx0, B.ntx) ? 1e30 : (double)(DV_TILE * (R0 - 1) + wlx);
                const double cov_y = span_full(sy0, B.nty) ? 1e30 : (double)(DV_TILE * (R0 - 1) + wly);
                fast = rho <= cov_x && rho <= cov_y;
                rq2 = (256.0 * rho) * (256.0 * rho);
            }
            if (fast) {
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                int nc = 0;   // list slots taken so far (every lane the same)
                for (int f0 = 0; f0 < total; f0 += 64) {
                    const int f = f0 + t;
                    int2 q = q0;
                    int lab = lab0;
                    long long d = d0;
                    if (f0 > 0 && f < total) {
                        q = S.tmpq[f];
                        lab = S.tmp[f];
                        d = S.tmpd[f];
                    }
                    unsigned mxk = 0, myk = 0;
                    int rx = 0, ry = 0;
                    if (f < total && (double)d <= rq2) {
                        rx = q.x - OX;
                        ry = q.y - OY;
                        image_masks(rx, ry, mxk, myk);
                    }
                    const int c = __popc(mxk) * __popc(myk);
                    const int x = wave_incl_sum(c);
                    int slot = nc + x - c;
                    for (unsigned a = mxk; a; a &= a - 1) {
                        const int cx = rx + (__ffs(a) - 2) * MX;
                        for (unsigned b = myk; b; b &= b - 1) {
                            if (slot < DV_CAND_CAP) {
                                S.cx[slot] = cx;
                                S.cy[slot] = ry + (__ffs(b) - 2) * MY;
                                S.lab[slot] = lab;
                            }
                            ++slot;
                        }
                    }
                    nc += wave_last(x);
                }
                if (t == 0) S.ncand = nc;
            }
            if (t == 0) {
                S.best = dmin;
                S.ntmp = total;
                S.fast = fast ? 1 : 0;
                S.nkeep = 0;
                S.far = 0;
            }
        }
        __syncthreads();
        const bool done = S.fast && S.ncand <= DV_CAND_CAP;
        if (!done) {
            // --- general case (from an empty list): a growing square of cells
            // for the bound, then every cell meeting the disc, evaluated in
            // LDS-sized chunks
            if (t == 0) S.ncand = 0;
            __syncthreads();
            for (int R = R0;; R *= 2) {
                if (S.best != ~0ull) break;
                const Span sx = span_cells(tx, 2 * R, B.ntx, ox), sy = span_cells(ty, 2 * R, B.nty, oy);
                visit_items(B, S, sx, sy, 1 << 30,
                            [&](int e) {
                                const int2 q = ld_int2(B.cell_q, e);
                                atomicMin(&S.best, (unsigned long long)d2q(tcx, tcy, q.x, q.y, MX, MY));
                            },
                            [](int) {});
                if (span_full(sx, B.ntx) && span_full(sy, B.nty)) break;
            }
            const double rho = sqrt((double)S.best) / 256.0 + hdiag2();
            const double rq2 = (256.0 * rho) * (256.0 * rho);
            const double px = tcx / 256.0, py = tcy / 256.0;
            const Span sx = span_sites((int)floor(px - rho), (int)floor(px + rho), lx, ox);
            const Span sy = span_sites((int)floor(py - rho), (int)floor(py + rho), ly, oy);
            visit_items(
                B, S, sx, sy, CAND_BATCH,
                [&](int e) {
                    const int2 q = ld_int2(B.cell_q, e);
                    if ((double)d2q(tcx, tcy, q.x, q.y, MX, MY) <= rq2) add_images(gmem(B.cell_items)[e], q);
                },
                [&](int m) {
                    // evaluate and empty the list when this batch could overflow it
                    if (S.ncand + m * IMG_MAX > DV_CAND_CAP) {
                        eval_owners(false, false);
                        __syncthreads();
                        if (t == 0) { S.ncand = 0; S.nchunks += 1; }
                        __syncthreads();
                    }
                });
        }
        eval_owners(true, done);
    }
    // window sites with no colour: beyond a wall, and obstacles.  (Without
    // either, a window 34 sites wide is stored as it is numbered.)
    if (!GEOM && W == 34) {
#pragma unroll
        for (int i = 0; i < WSITES; ++i)
            if (t + i * DV_BLOCK < W * H) S.own[t + i * DV_BLOCK] = bl[i];
    } else
#pragma unroll
    for (int i = 0; i < WSITES; ++i) {
        const int w = t + i * DV_BLOCK;
        const int wy = (w * wmagic) >> 16, wx = w - wy * W;
        if (w >= W * H) continue;
        int ax = x0 + wx - 1, ay = y0 + wy - 1;
        bool none = (ox && (ax < 0 || ax >= lx)) || (oy && (ay < 0 || ay >= ly));
        if (GEOM && B.obst && !none) {
            ax = ax < 0 ? ax + lx : (ax >= lx ? ax - lx : ax);
            ay = ay < 0 ? ay + ly : (ay >= ly ? ay - ly : ay);
            none = gmem(B.obst)[(size_t)ay * lx + ax] != 0;
        }
        S.own[wy * 34 + wx] = none ? DV_EMPTY : bl[i];
    }
    __syncthreads();

    // --- frame gaps and the neighbour rules.  The inner-frame points whose
    // colour decides a second-neighbour link are collected, then coloured
    // against the candidate list (or, after a candidate-list overflow, by the
    // exact grid search).
    const bool in_lds = S.nchunks == 0;
    const bool imode = S.imode;
    const int ncl = S.nkeep;   // the ordered list of the single chunk
    auto emit = [&](int a, int b) {
        const int slot = atomicAdd(&S.npair, 1);
        if (slot < PAIR_CAP) {
            S.pair[slot] = ((unsigned long long)(unsigned)a << 32) | (unsigned)b;
        } else {
            row_insert(adj + (size_t)a * B.maxdeg, B.maxdeg, b, fs);
            row_insert(adj + (size_t)b * B.maxdeg, B.maxdeg, a, fs);
        }
    };
    // thread t takes column t & 31 and the four rows 4 (t >> 5) .. + 3, so the
    // colours around its sites are one 6 x 3 block of the window
    const int cx = t & 31, ry = t >> 5, lane = t & 63;
    const int ys = 4 * ry;
    int g[6][3];
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) g[a][b] = S.own[(ys + a) * 34 + cx + b];
    // vertex sites of the thread (frame gaps >= 3): bit i for row ys + i.
    // (The map pointer and flag are read once: the stores could alias the
    // slot table as far as the compiler knows.)
    const bool keep_maps = B.keep_maps;
    const auto orow = gmem(B.owner) + ((size_t)(y0 + ys) * lx + x0 + cx);
    unsigned vmask = 0;
    if (!GEOM) {
        // The frame of the site in row ys + i is the border of rows i .. i + 2
        // of the block: its gaps are the changes along rows i and i + 2 and
        // down columns 0 and 2 (rows i to i + 1 and i + 1 to i + 2), each
        // change counted once for the thread's four sites.  (Without walls
        // and obstacles no frame point is MAXLINK once the site has a colour:
        // there is a centre, so every point has one.)
        int hr[6], vc[5];
#pragma unroll
        for (int a = 0; a < 6; ++a) hr[a] = (g[a][0] != g[a][1] ? 1 : 0) + (g[a][1] != g[a][2] ? 1 : 0);
#pragma unroll
        for (int a = 0; a < 5; ++a) vc[a] = (g[a][0] != g[a + 1][0] ? 1 : 0) + (g[a][2] != g[a + 1][2] ? 1 : 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int y = ys + i;
            if (cx >= tw || y >= th) continue;
            const int ckk = g[i + 1][1];
            if (keep_maps) orow[(size_t)i * lx] = ckk;
            // (with no centre every colour is MAXLINK and there are no gaps)
            const int gaps = hr[i] + hr[i + 2] + vc[i] + vc[i + 1];
            vmask |= gaps >= 3 ? 1u << i : 0u;
        }
    } else
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = ys + i;
        if (cx >= tw || y >= th) continue;
        const int ckk = g[i + 1][1];
        if (keep_maps) orow[(size_t)i * lx] = ckk;
        if (ckk == DV_EMPTY) continue;
        int f[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) f[k] = g[i + 1 + fry(k)][1 + frx(k)];
        // (a change next to a point without colour is no gap)
        int gaps = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int a = f[k], b = f[(k + 1) & 7];
            gaps += (a != b && a != DV_EMPTY && b != DV_EMPTY) ? 1 : 0;
        }
        vmask |= gaps >= 3 ? 1u << i : 0u;
    }
    // The neighbour rules at the wave's vertex sites, which are few: the
    // sites are listed in lane order (a wave prefix of the per-lane counts)
    // and each takes four lanes, lane r applying the first- and
    // second-neighbour rules of frame direction r (spx, spy, smx, smy rotated
    // by quarter turns).  A second-neighbour candidate goes to the mask of
    // the thread owning the site (bit 4i + r), read back below.
    // (a wave without vertex sites, the usual case, skips both steps)
    const int vcnt = __popc(vmask);
    const int vinc = wave_incl_sum(vcnt);
    const int vtotal = wave_last(vinc);
    if (vtotal > 0) {
        S.pendw[t] = 0u;
        const int cnt = vcnt, inc = vinc, total = vtotal;
        for (int p0 = 0; p0 < total; p0 += 16) {
            const int item = min(p0 + (lane >> 2), total - 1), r = lane & 3;
            // lane holding the item: the first one whose inclusive count exceeds it
            int L = 0;
            for (int step = 32; step > 0; step >>= 1)
                L += __shfl(inc, L + step - 1, 64) <= item ? step : 0;
            unsigned m = (unsigned)__shfl((int)vmask, L, 64);
            for (int k = item - (__shfl(inc, L, 64) - __shfl(cnt, L, 64)); k > 0; --k) m &= m - 1;
            const int i = __ffs(m) - 1;
            const int tl = (t & ~63) | L;
            const int c = (4 * (tl >> 5) + i + 1) * 34 + (tl & 31) + 1;
            const int k0 = 2 * r, k1 = (2 * r + 2) & 7, k7 = (2 * r + 7) & 7;
            const int ckk = S.own[c];
            const int tg = S.own[c + fry(k0) * 34 + frx(k0)];
            const int pa = S.own[c + fry(k1) * 34 + frx(k1)], pb = S.own[c + fry(k7) * 34 + frx(k7)];
            const int dg = S.own[c + fry(k0 + 1) * 34 + frx(k0 + 1)];
            if (p0 + (lane >> 2) < total) {
                if ((!GEOM || tg != DV_EMPTY) && pa != pb && tg != ckk) emit(min(ckk, tg), max(ckk, tg));
                if ((!GEOM || dg != DV_EMPTY) && dg != ckk && pa != pb && pa != tg)
                    atomicOr(&S.pendw[tl], 1u << (4 * i + r));
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const unsigned pend = S.pendw[t];   // bit 4i + r: site i needs the colour of inner-frame point r
        // Inner-frame queries, which are few: numbered within the wave (a wave
        // prefix of the per-lane counts) and answered one per lane, 64 at a time.
        const int qcnt = __popc(pend);
        const int qinc = wave_incl_sum(qcnt);
        const int qtotal = wave_last(qinc);
        for (int p0 = 0; p0 < qtotal; p0 += 64) {
            const int cnt = qcnt, inc = qinc, total = qtotal;
            const int item = min(p0 + lane, total - 1);
            // lane holding the item: the first one whose inclusive count exceeds it
            int L = 0;
            for (int step = 32; step > 0; step >>= 1)
                L += __shfl(inc, L + step - 1, 64) <= item ? step : 0;
            unsigned m = (unsigned)__shfl((int)pend, L, 64);
            for (int k = item - (__shfl(inc, L, 64) - __shfl(cnt, L, 64)); k > 0; --k) m &= m - 1;
            if (p0 + lane >= total) continue;
            const int bit = __ffs(m) - 1, r = bit & 3;
            const int tl = (t & ~63) | L;
            const int qsx = tl & 31, qsy = 4 * (tl >> 5) + (bit >> 2);
            int mq;
            if (in_lds && imode) {
                // (the packed form of the evaluation; |2 q| <= 16128 as for the sites)
                const sh2 q2 = sh2{(short)(-2 * (256 * qsx + inx(r))), (short)(-2 * (256 * qsy + iny(r)))};
                int bee = INT_MAX;
                mq = DV_EMPTY;
                // the single chunk is ordered by label: ties keep the first
                for (int k = 0; k < ncl; ++k) {
                    const int e = dot2_acc(q2, __builtin_bit_cast(sh2, S.ixy[k]), S.ik[k]);
                    const bool lt = e < bee;
                    bee = lt ? e : bee;
                    mq = lt ? S.sl[k] : mq;
                }
            } else if (in_lds) {
                const double qx = -2.0 * (256.0 * qsx + inx(r)), qy = -2.0 * (256.0 * qsy + iny(r));
                double bee = 1.0e300;
                mq = DV_EMPTY;
                // the single chunk is ordered by label: ties keep the first
                for (int k = 0; k < ncl; ++k) {
                    const double e = fma(qx, S.sx[k], fma(qy, S.sy[k], S.sk[k]));
                    const bool lt = e < bee;
                    bee = lt ? e : bee;
                    mq = lt ? S.sl[k] : mq;
                }
            } else {
                // (on a walled axis the point is inside: its diagonal
                // partner has a colour)
                int X = OX + 256 * qsx + inx(r), Y = OY + 256 * qsy + iny(r);
                if (X < 0) X += MX;
                if (Y < 0) Y += MY;
                mq = point_nearest(B, X, Y);
            }
            const int c = (qsy + 1) * 34 + qsx + 1;
            const int ckk = S.own[c];
            const int dg = S.own[c + fry(2 * r + 1) * 34 + frx(2 * r + 1)];
            if (mq == dg || mq == ckk) emit(min(ckk, dg), max(ckk, dg));
        }
    }
    __syncthreads();
    // --- distinct couples of the tile go to its list (k_rows fills the rows);
    // beyond the list's capacity they go into the rows directly
    // (a group of GL lanes per couple looks for an earlier copy; one wave holds
    // whole groups, and a ballot ORs the group's answers)
    const int np = min(S.npair, PAIR_CAP);
    int GL = 64;
    while (GL > 1 && np * GL > DV_BLOCK) GL >>= 1;
    const int sub = t & (GL - 1);
    const unsigned long long gmask = (GL == 64 ? ~0ull : ((1ull << GL) - 1ull)) << ((t & 63) & ~(GL - 1));
    for (int i0 = 0; i0 < np; i0 += DV_BLOCK / GL) {
        const int i = i0 + t / GL;
        unsigned long long key = 0;
        bool dup = false;
        if (i < np) {
            key = S.pair[i];
            for (int j = sub; j < i; j += GL)
                if (S.pair[j] == key) { dup = true; break; }
        }
        const bool first = i < np && !(__ballot(dup) & gmask);
        if (!first || sub != 0) continue;
        const int a = (int)(key >> 32), b = (int)(key & 0xffffffffu);
        const int slot = atomicAdd(&S.nout, 1);
        if (slot < DV_TILE_PAIRS) {
            st_int2(B.tpairs, (size_t)tile * DV_TILE_PAIRS + slot, a, b);
        } else {
            row_insert(adj + (size_t)a * B.maxdeg, B.maxdeg, b, fs);
            row_insert(adj + (size_t)b * B.maxdeg, B.maxdeg, a, fs);
        }
    }
    __syncthreads();
    if (t == 0) gmem(B.tpair_n)[tile] = min(S.nout, DV_TILE_PAIRS);
}

// Rows from the tiles' couple lists: ROW_LANES lanes per tile (a tile lists a few
// couples), one lane per couple end.  Rows are sets: a couple found by
// several tiles is stored once.
#define ROW_LANES 4
__global__ __launch_bounds__(256) void k_rows(const Bufs *__restrict__ D, Batch G) {
    const int gt = blockIdx.x * (256 / ROW_LANES) + (threadIdx.x / ROW_LANES);
    const int lane = threadIdx.x % ROW_LANES;
    if (gt >= G.tiles) return;
    const int e = entry_of(G.tbase, G.tpe, G.n, gt);
    const Bufs B = D[G.idx[e]];
    const int tile = gt - G.tbase[e];
    FrameState *fs = B.fs;
    if (fs->err) return;
    const int n = gmem(B.tpair_n)[tile];
    gint *adj = gmem(B.cur.adj);
    for (int j = lane; j < 2 * n; j += ROW_LANES) {
        const int2 p = ld_int2(B.tpairs, (size_t)tile * DV_TILE_PAIRS + (j >> 1));
        if (j & 1) row_insert(adj + (size_t)p.y * B.maxdeg, B.maxdeg, p.x, fs);
        else row_insert(adj + (size_t)p.x * B.maxdeg, B.maxdeg, p.y, fs);
    }
}

}  // namespace

void launch_voronoi(const Batch &G, hipStream_t s, Prof &P) {
    const int fgrid = (int)std::min<long long>((G.kmax + 1023) / 1024, 256);
    P.begin(ST_FINALIZE, s);
    hipLaunchKernelGGL(k_finalize, dim3(fgrid, 1, G.n), dim3(1024), 0, s, G.D, G);
    hipLaunchKernelGGL(k_grid, dim3(1, 1, G.n), dim3(1024), 0, s, G.D, G);
    P.end(ST_FINALIZE, s);
    P.begin(ST_OWNER_EDGES, s);
    if (G.geom) hipLaunchKernelGGL(k_owner_edges<true>, dim3(G.tiles), dim3(DV_BLOCK), 0, s, G.D, G);
    else hipLaunchKernelGGL(k_owner_edges<false>, dim3(G.tiles), dim3(DV_BLOCK), 0, s, G.D, G);
    P.end(ST_OWNER_EDGES, s);
    P.begin(ST_ROWS, s);
    hipLaunchKernelGGL(k_rows, dim3((G.tiles + 256 / ROW_LANES - 1) / (256 / ROW_LANES)), dim3(256), 0, s, G.D, G);
    P.end(ST_ROWS, s);
}
