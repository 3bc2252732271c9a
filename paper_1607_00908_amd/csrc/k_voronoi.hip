// Centres, bucket grid, digital Voronoi colouring and Delaunay couples
// (Sec. 3.1 last step, Sec. 3.2.1 and Sec. 3.2.2 of the paper).
//
//   k_finalize      exact Q.8 and float64 centres from the integer sums;
//                   counts the centres of each bucket cell
//   k_grid_scan     cell offsets (one block)
//   k_grid_scatter  centres ordered by cell
//   k_owner_edges   per tile: candidate centres from the grid, nearest centre
//                   of every site of the tile and its one-site ring (LDS),
//                   owner map, frame-gap vertex test and the first / second
//                   nearest-neighbour rules; couples go into the adjacency rows
//                   with a lock-free insert that drops duplicates
//   k_rows          sorts every row (the compression of the adjacency)
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

__global__ __launch_bounds__(256) void k_finalize(Bufs B) {
    DevState *st = B.st;
    if (st->err) return;
    const int K = st->K_now;
    const int now = 1 - st->sel;
    const CompBuf C = B.comp[now];
    int namb = 0;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
        const long long n = B.acc_n[k], sx = B.acc_x[k], sy = B.acc_y[k];
        const int root = B.acc_root[k], amb = B.acc_amb[k];
        B.acc_n[k] = 0;
        B.acc_x[k] = 0;
        B.acc_y[k] = 0;
        B.acc_amb[k] = 0;
        const int rx = root % B.lx, ry = root / B.lx;
        const int qx = (int)pmod64(256LL * rx + floor_div(512 * sx + n, 2 * n), 256LL * B.lx);
        const int qy = (int)pmod64(256LL * ry + floor_div(512 * sy + n, 2 * n), 256LL * B.ly);
        double fx = (double)rx + (double)sx / (double)n;
        double fy = (double)ry + (double)sy / (double)n;
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
    if (namb) atomicAdd(&st->n_amb, namb);
}

__global__ __launch_bounds__(1024) void k_grid_scan(Bufs B) {
    __shared__ int wsum[16];
    if (B.st->err) return;
    const int total = block_exclusive_scan(B.cell_count, B.cell_start, B.ncells, wsum);
    if (threadIdx.x == 0) B.cell_start[B.ncells] = total;
}

__global__ __launch_bounds__(256) void k_grid_scatter(Bufs B) {
    DevState *st = B.st;
    if (st->err) return;
    const int K = st->K_now;
    const CompBuf C = B.comp[1 - st->sel];
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
        const int pos = B.cell_start[B.comp_cell[k]] + B.comp_slot[k];
        B.cell_items[pos] = k;
        B.cell_q[pos] = make_int2(C.qx[k], C.qy[k]);
    }
}

// Frame of a site (Sec. 3.2.2), cyclic: spx, spxpy, spy, spymx, smx, smxmy,
// smy, smypx; inner-frame points a_k, b_k, c_k, d_k at (+-1/2, +-1/2).
__constant__ int FRX[8] = {1, 1, 0, -1, -1, -1, 0, 1};
__constant__ int FRY[8] = {0, 1, 1, 1, 0, -1, -1, -1};
__constant__ int INX[4] = {128, -128, -128, 128};
__constant__ int INY[4] = {128, 128, -128, -128};

__device__ __forceinline__ void row_insert(int *row, int maxdeg, int v, DevState *st) {
    for (int i = 0; i < maxdeg; ++i) {
        const int cur = row[i];
        if (cur == v) return;
        if (cur == DV_EMPTY) {
            const int old = atomicCAS(&row[i], DV_EMPTY, v);
            if (old == DV_EMPTY || old == v) return;
        }
    }
    atomicOr(&st->err, DV_E_DEGREE);
}

__device__ __forceinline__ void emit(const Bufs &B, int *adj, int a, int b) {
    row_insert(adj + (size_t)a * B.maxdeg, B.maxdeg, b, B.st);
    row_insert(adj + (size_t)b * B.maxdeg, B.maxdeg, a, B.st);
}

#define WSITES 5   // ceil(34*34 / 256) window sites per thread

__global__ __launch_bounds__(DV_BLOCK) void k_owner_edges(Bufs B) {
    __shared__ int own[34 * 34];
    __shared__ int cqx[DV_CAND_CAP], cqy[DV_CAND_CAP], clab[DV_CAND_CAP];
    __shared__ int ncand;
    __shared__ unsigned long long s_best;
    DevState *st = B.st;
    if (st->err) return;
    const int K = st->K_now;
    const int now = 1 - st->sel;
    int *adj = B.comp[now].adj;
    const int tx = blockIdx.x, ty = blockIdx.y;
    const int x0 = tx * DV_TILE, y0 = ty * DV_TILE;
    const int tw = min(DV_TILE, B.lx - x0), th = min(DV_TILE, B.ly - y0);
    const int W = tw + 2, H = th + 2;
    const int t = threadIdx.x, lx = B.lx, ly = B.ly;
    const int MX = 256 * lx, MY = 256 * ly;
    const int *cs = B.cell_start;

    long long bd[WSITES];
    int bl[WSITES], wX[WSITES], wY[WSITES];
#pragma unroll
    for (int i = 0; i < WSITES; ++i) {
        bd[i] = LLONG_MAX;
        bl[i] = DV_EMPTY;
        const int w = t + i * DV_BLOCK;
        const int wx = w % W - 1, wy = w / W - 1;
        wX[i] = 256 * pmod(x0 + wx, lx);
        wY[i] = 256 * pmod(y0 + wy, ly);
    }

    if (K > 0) {
        // --- a first bound on the distance from the tile centre to a centre
        const int tcx = 256 * x0 + 128 * (tw - 1), tcy = 256 * y0 + 128 * (th - 1);
        if (t == 0) s_best = ~0ull;
        __syncthreads();
        for (int R = 1;; R *= 2) {
            const Span sx = span_cells(tx, R, B.ntx), sy = span_cells(ty, R, B.nty);
            for (int ry = 0; ry < sy.n; ++ry)
                for (int row = sy.lo[ry]; row <= sy.hi[ry]; ++row)
                    for (int rx = 0; rx < sx.n; ++rx) {
                        const int e0 = cs[row * B.ntx + sx.lo[rx]], e1 = cs[row * B.ntx + sx.hi[rx] + 1];
                        for (int e = e0 + t; e < e1; e += DV_BLOCK) {
                            const int2 q = B.cell_q[e];
                            atomicMin(&s_best, (unsigned long long)d2q(tcx, tcy, q.x, q.y, MX, MY));
                        }
                    }
            __syncthreads();
            if (s_best != ~0ull || (span_full(sx, B.ntx) && span_full(sy, B.nty))) break;
            __syncthreads();
        }
        // --- every centre within r0 + 2h of the tile centre (h: half diagonal
        // of the tile plus its ring) can own a site or inner-frame point here
        const double hx = 0.5 * (tw + 1), hy = 0.5 * (th + 1);
        const double rho = sqrt((double)s_best) / 256.0 + 2.0 * sqrt(hx * hx + hy * hy) + 2.0;
        const double rq = 256.0 * rho;
        const double px = tcx / 256.0, py = tcy / 256.0;
        const Span sx = span_sites((int)floor(px - rho), (int)floor(px + rho), lx);
        const Span sy = span_sites((int)floor(py - rho), (int)floor(py + rho), ly);
        if (t == 0) ncand = 0;
        __syncthreads();
        // rows are visited one at a time; the LDS list is evaluated and
        // emptied whenever the next batch could overflow it
        for (int ry = 0; ry < sy.n; ++ry)
            for (int row = sy.lo[ry]; row <= sy.hi[ry]; ++row) {
                int a0 = 0, a1 = 0, b0 = 0, b1 = 0;
                a0 = cs[row * B.ntx + sx.lo[0]];
                a1 = cs[row * B.ntx + sx.hi[0] + 1];
                if (sx.n == 2) {
                    b0 = cs[row * B.ntx + sx.lo[1]];
                    b1 = cs[row * B.ntx + sx.hi[1] + 1];
                }
                const int na = a1 - a0, total = na + (b1 - b0);
                for (int base = 0; base < total; base += DV_CAND_CAP) {
                    const int m = min(DV_CAND_CAP, total - base);
                    if (ncand + m > DV_CAND_CAP) {
                        // evaluate and empty the list
                        const int nc = ncand;
                        for (int c = 0; c < nc; ++c) {
                            const int qx = cqx[c], qy = cqy[c], lab = clab[c];
#pragma unroll
                            for (int i = 0; i < WSITES; ++i) {
                                const long long d = d2q(wX[i], wY[i], qx, qy, MX, MY);
                                if (d < bd[i] || (d == bd[i] && lab < bl[i])) { bd[i] = d; bl[i] = lab; }
                            }
                        }
                        __syncthreads();
                        if (t == 0) ncand = 0;
                        __syncthreads();
                    }
                    for (int j = t; j < m; j += DV_BLOCK) {
                        const int f = base + j;
                        const int e = f < na ? a0 + f : b0 + (f - na);
                        const int2 q = B.cell_q[e];
                        const long long d = d2q(tcx, tcy, q.x, q.y, MX, MY);
                        if ((double)d <= rq * rq) {
                            const int slot = atomicAdd(&ncand, 1);
                            cqx[slot] = q.x;
                            cqy[slot] = q.y;
                            clab[slot] = B.cell_items[e];
                        }
                    }
                    __syncthreads();
                }
            }
        const int nc = ncand;
        for (int c = 0; c < nc; ++c) {
            const int qx = cqx[c], qy = cqy[c], lab = clab[c];
#pragma unroll
            for (int i = 0; i < WSITES; ++i) {
                const long long d = d2q(wX[i], wY[i], qx, qy, MX, MY);
                if (d < bd[i] || (d == bd[i] && lab < bl[i])) { bd[i] = d; bl[i] = lab; }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < WSITES; ++i) {
        const int w = t + i * DV_BLOCK;
        if (w < W * H) own[(w / W) * 34 + (w % W)] = bl[i];
    }
    __syncthreads();

    const int cx = t & 31, ry = t >> 5;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = ry + 8 * i;
        if (cx >= tw || y >= th) continue;
        const int c = (y + 1) * 34 + cx + 1;
        const int ck = own[c];
        if (B.keep_maps) B.owner[(size_t)(y0 + y) * lx + x0 + cx] = ck;
        if (ck == DV_EMPTY) continue;
        int f[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) f[k] = own[c + FRY[k] * 34 + FRX[k]];
        int gaps = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int a = f[k], b = f[(k + 1) & 7];
            gaps += (a != b && a != DV_EMPTY && b != DV_EMPTY) ? 1 : 0;
        }
        if (gaps < 3) continue;
        const int gx = x0 + cx, gy = y0 + y;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int tg = f[2 * r];
            const int pa = f[(2 * r + 2) & 7], pb = f[(2 * r + 7) & 7];
            if (tg != DV_EMPTY && pa != pb && tg != ck) emit(B, adj, min(ck, tg), max(ck, tg));
            const int dg = f[2 * r + 1];
            if (dg != DV_EMPTY && dg != ck && pa != pb && pa != tg) {
                int X = 256 * gx + INX[r], Y = 256 * gy + INY[r];
                if (X < 0) X += MX;
                if (Y < 0) Y += MY;
                const int m = point_nearest(B, X, Y);
                if (m == dg || m == ck) emit(B, adj, min(ck, dg), max(ck, dg));
            }
        }
    }
}

// Sort each row ascending; DV_EMPTY padding stays at the end.
__global__ __launch_bounds__(256) void k_rows(Bufs B) {
    DevState *st = B.st;
    if (st->err) return;
    const int K = st->K_now;
    const CompBuf C = B.comp[1 - st->sel];
    int e2 = 0;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
        int *row = C.adj + (size_t)k * B.maxdeg;
        int n = 0;
        while (n < B.maxdeg && row[n] != DV_EMPTY) ++n;
        for (int i = 1; i < n; ++i) {
            const int v = row[i];
            int j = i - 1;
            while (j >= 0 && row[j] > v) { row[j + 1] = row[j]; --j; }
            row[j + 1] = v;
        }
        C.deg[k] = n;
        e2 += n;
    }
    for (int o = 32; o > 0; o >>= 1) e2 += __shfl_down(e2, o, 64);
    if ((threadIdx.x & 63) == 0 && e2) atomicAdd(&st->E2_now, e2);
}

}  // namespace

void launch_voronoi(const Bufs &B, hipStream_t s, Prof &P) {
    const int kgrid = (int)std::min<long long>((B.kmax + 255) / 256, 1024);
    P.begin(ST_FINALIZE, s);
    hipLaunchKernelGGL(k_finalize, dim3(kgrid), dim3(256), 0, s, B);
    P.end(ST_FINALIZE, s);
    P.begin(ST_GRID_SCAN, s);
    hipLaunchKernelGGL(k_grid_scan, dim3(1), dim3(1024), 0, s, B);
    P.end(ST_GRID_SCAN, s);
    P.begin(ST_GRID_SCATTER, s);
    hipLaunchKernelGGL(k_grid_scatter, dim3(kgrid), dim3(256), 0, s, B);
    P.end(ST_GRID_SCATTER, s);
    P.begin(ST_OWNER_EDGES, s);
    hipLaunchKernelGGL(k_owner_edges, dim3(B.ntx, B.nty), dim3(DV_BLOCK), 0, s, B);
    P.end(ST_OWNER_EDGES, s);
    P.begin(ST_ROWS, s);
    hipLaunchKernelGGL(k_rows, dim3(kgrid), dim3(256), 0, s, B);
    P.end(ST_ROWS, s);
}
