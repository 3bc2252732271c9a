// Device helpers shared by the HIP sources of libdv: exact Q.8 distances
// (minimum image on periodic axes, plain on walled ones) and the bucket grid
// of centres (one cell per 32x32 tile).
#pragma once

#include "dv_internal.h"

// Global-memory view of a buffer pointer read from the slot table.  The table
// lives in device memory, so the compiler cannot tell that its pointers are
// global and would emit flat accesses, which also count against the LDS wait
// counter; accesses through this view are global instructions.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gmem(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}
using gint = __attribute__((address_space(1))) int;
typedef int dv_v4i __attribute__((ext_vector_type(4)));

// int2 element i of a buffer, through a global 64-bit access
__device__ __forceinline__ int2 ld_int2(const int2 *p, size_t i) {
    const unsigned long long v = gmem(reinterpret_cast<const unsigned long long *>(p))[i];
    return make_int2((int)(unsigned)v, (int)(unsigned)(v >> 32));
}
__device__ __forceinline__ void st_int2(int2 *p, size_t i, int a, int b) {
    gmem(reinterpret_cast<unsigned long long *>(p))[i] =
        (unsigned long long)(unsigned)a | ((unsigned long long)(unsigned)b << 32);
}

// ---- wave-wide operations through DPP lane moves --------------------------
// (every lane of the wave must be active).  Lane moves within rows of 16
// lanes (row_shr), then the last lane of a row broadcast into the rows above
// it (row_bcast:15 into rows 1 and 3, row_bcast:31 into rows 2 and 3); lanes
// without a source take the identity.  The control codes are those of the
// GFX9 data-parallel primitives.
#define DPP_ROW_SHR(n) (0x110 + (n))
#define DPP_WAVE_SHR1 0x138
#define DPP_ROW_BCAST15 0x142
#define DPP_ROW_BCAST31 0x143

// inclusive prefix sum over the lanes of the wave
__device__ __forceinline__ int wave_incl_sum(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_SHR(1), 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_SHR(2), 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_SHR(4), 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_SHR(8), 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_BCAST15, 0xa, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_BCAST31, 0xc, 0xf, false);
    return x;
}

// value of the last lane (a scalar)
__device__ __forceinline__ int wave_last(int x) { return __builtin_amdgcn_readlane(x, 63); }

// one step of wave_min_u64: the minimum with the value CTRL moves in
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long min_step_u64(unsigned long long v) {
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(-1, (int)(unsigned)v, CTRL, ROWS, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(-1, (int)(unsigned)(v >> 32), CTRL, ROWS, 0xf, false);
    const unsigned long long o = ((unsigned long long)hi << 32) | lo;
    return o < v ? o : v;
}

// minimum over the lanes of the wave, in every lane (unsigned 64-bit)
__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
    v = min_step_u64<DPP_ROW_SHR(1), 0xf>(v);
    v = min_step_u64<DPP_ROW_SHR(2), 0xf>(v);
    v = min_step_u64<DPP_ROW_SHR(4), 0xf>(v);
    v = min_step_u64<DPP_ROW_SHR(8), 0xf>(v);
    v = min_step_u64<DPP_ROW_BCAST15, 0xa>(v);
    v = min_step_u64<DPP_ROW_BCAST31, 0xc>(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

// value of the previous lane of the wave (lane 0: `first`)
__device__ __forceinline__ int wave_prev(int x, int first) {
    return __builtin_amdgcn_update_dpp(first, x, DPP_WAVE_SHR1, 0xf, 0xf, false);
}

// v in (-M, M) -> signed minimum image in [-M/2, M/2 - 1]  (M = 256 L, even)
__device__ __forceinline__ int wrap_q(int v, int M) {
    const int h = M >> 1;
    if (v >= h) v -= M;
    else if (v < -h) v += M;
    return v;
}

// Wrap period (Q.8) of an axis for distances: 256 L on a periodic axis.  On
// a walled axis 512 L: no difference of two in-domain points (|v| < 256 L)
// reaches half of it, so wrap_q leaves every difference as it is.
__device__ __forceinline__ int qperiod(int L, int open) { return open ? 512 * L : 256 * L; }

// squared distance between Q.8 points; X, Y, cx, cy in [0, 256 L); MX, MY
// wrap periods (qperiod)
__device__ __forceinline__ long long d2q(int X, int Y, int cx, int cy, int MX, int MY) {
    const int dx = wrap_q(X - cx, MX), dy = wrap_q(Y - cy, MY);
    return (long long)dx * dx + (long long)dy * dy;
}

__device__ __forceinline__ int pmod(int v, int m) {
    const int r = v % m;
    return r < 0 ? r + m : r;
}

// Up to two ranges of cell indices along one axis (accessors select between
// two scalars, so a Span never lives in scratch memory).
struct Span {
    int lo0, hi0, lo1, hi1;
    int n;
    __device__ __forceinline__ int lo(int i) const { return i ? lo1 : lo0; }
    __device__ __forceinline__ int hi(int i) const { return i ? hi1 : hi0; }
};

// Cells whose sites meet the site interval [a, b] (integers, a <= b): wrapped
// on a periodic axis, cut at the walls on an open one.
__device__ __forceinline__ Span span_sites(int a, int b, int L, int open) {
    Span s;
    const int ncell = (L + DV_TILE - 1) / DV_TILE;
    if (open) {
        a = max(a, 0);
        b = min(b, L - 1);
        s.lo1 = 0; s.hi1 = -1;
        if (a > b) { s.n = 0; s.lo0 = 0; s.hi0 = -1; }
        else { s.n = 1; s.lo0 = a / DV_TILE; s.hi0 = b / DV_TILE; }
        return s;
    }
    if (b - a >= L - 1) {
        s.n = 1; s.lo0 = 0; s.hi0 = ncell - 1; s.lo1 = 0; s.hi1 = -1;
        return s;
    }
    a = pmod(a, L);
    b = pmod(b, L);
    if (a <= b) {
        s.n = 1; s.lo0 = a / DV_TILE; s.hi0 = b / DV_TILE; s.lo1 = 0; s.hi1 = -1;
    } else {
        s.n = 2; s.lo0 = a / DV_TILE; s.hi0 = ncell - 1; s.lo1 = 0; s.hi1 = b / DV_TILE;
    }
    return s;
}

// Cells within Chebyshev cell distance R of cell c (no repeats; wrapped on a
// periodic axis, cut at the walls on an open one).
__device__ __forceinline__ Span span_cells(int c, int R, int ncell, int open) {
    Span s;
    if (open) {
        s.n = 1; s.lo0 = max(c - R, 0); s.hi0 = min(c + R, ncell - 1); s.lo1 = 0; s.hi1 = -1;
        return s;
    }
    if (2 * R + 1 >= ncell) {
        s.n = 1; s.lo0 = 0; s.hi0 = ncell - 1; s.lo1 = 0; s.hi1 = -1;
        return s;
    }
    const int a = c - R, b = c + R;
    if (a < 0) {
        s.n = 2; s.lo0 = a + ncell; s.hi0 = ncell - 1; s.lo1 = 0; s.hi1 = b;
    } else if (b >= ncell) {
        s.n = 2; s.lo0 = a; s.hi0 = ncell - 1; s.lo1 = 0; s.hi1 = b - ncell;
    } else {
        s.n = 1; s.lo0 = a; s.hi0 = b; s.lo1 = 0; s.hi1 = -1;
    }
    return s;
}

__device__ __forceinline__ bool span_full(const Span &s, int ncell) {
    return s.n == 1 && s.lo0 == 0 && s.hi0 == ncell - 1;
}

// Nearest now centre of the Q.8 point (X, Y) in [0, 256 lx) x [0, 256 ly),
// exact, ties to the lowest label, by the bucket grid.  K >= 1.  First a growing square of
// cells around the point's cell until a centre is seen; its distance bounds
// the answer, so every cell meeting the disc of that radius (+1 site) around
// the point is then scanned.
__device__ int point_nearest(const Bufs &B, int X, int Y) {
    const int MX = qperiod(B.lx, B.open_x), MY = qperiod(B.ly, B.open_y);
    const int cx = X >> 13, cy = Y >> 13;
    const auto cs = gmem(B.cell_start);
    long long bd = LLONG_MAX;
    for (int R = 1;; R *= 2) {
        const Span sx = span_cells(cx, R, B.ntx, B.open_x), sy = span_cells(cy, R, B.nty, B.open_y);
        for (int ry = 0; ry < sy.n; ++ry)
            for (int row = sy.lo(ry); row <= sy.hi(ry); ++row)
                for (int rx = 0; rx < sx.n; ++rx) {
                    const int e0 = cs[row * B.ntx + sx.lo(rx)], e1 = cs[row * B.ntx + sx.hi(rx) + 1];
                    for (int e = e0; e < e1; ++e) {
                        const int2 q = ld_int2(B.cell_q, e);
                        const long long d = d2q(X, Y, q.x, q.y, MX, MY);
                        if (d < bd) bd = d;
                    }
                }
        if (bd != LLONG_MAX || (span_full(sx, B.ntx) && span_full(sy, B.nty))) break;
    }
    // disc of radius sqrt(bd) + 1 site around the point
    const double rho = sqrt((double)bd) / 256.0 + 1.0;
    const double px = X / 256.0, py = Y / 256.0;
    const Span sx = span_sites((int)floor(px - rho), (int)floor(px + rho), B.lx, B.open_x);
    const Span sy = span_sites((int)floor(py - rho), (int)floor(py + rho), B.ly, B.open_y);
    long long best = LLONG_MAX;
    int bl = DV_EMPTY;
    for (int ry = 0; ry < sy.n; ++ry)
        for (int row = sy.lo(ry); row <= sy.hi(ry); ++row)
            for (int rx = 0; rx < sx.n; ++rx) {
                const int e0 = cs[row * B.ntx + sx.lo(rx)], e1 = cs[row * B.ntx + sx.hi(rx) + 1];
                for (int e = e0; e < e1; ++e) {
                    const int2 q = ld_int2(B.cell_q, e);
                    const long long d = d2q(X, Y, q.x, q.y, MX, MY);
                    const int lab = gmem(B.cell_items)[e];
                    if (d < best || (d == best && lab < bl)) { best = d; bl = lab; }
                }
            }
    return bl;
}

// Lexicographic (distance, label) minimum across a group of GL lanes (an
// aligned part of a wave).
template <int GL>
__device__ __forceinline__ void group_min_dl(long long &d, int &lab) {
    for (int o = GL / 2; o > 0; o >>= 1) {
        const long long d2 = __shfl_xor(d, o, 64);
        const int l2 = __shfl_xor(lab, o, 64);
        if (d2 < d || (d2 == d && l2 < lab)) { d = d2; lab = l2; }
    }
}

// Same search as point_nearest with a group of GL lanes (an aligned part of
// a wave) sharing the cells: lane j of the group takes the (row, column
// range) pairs j, j + GL, ...  Every lane of the group must call it with the
// same point; every lane of the group gets the answer.
template <int GL>
__device__ int group_nearest(const Bufs &B, int X, int Y) {
    const int MX = qperiod(B.lx, B.open_x), MY = qperiod(B.ly, B.open_y);
    const int cx = X >> 13, cy = Y >> 13;
    const int lane = threadIdx.x & (GL - 1);
    const auto cs = gmem(B.cell_start);
    long long bd = LLONG_MAX;
    int dummy = 0;
    for (int R = 1;; R *= 2) {
        const Span sx = span_cells(cx, R, B.ntx, B.open_x), sy = span_cells(cy, R, B.nty, B.open_y);
        const int n0 = sy.hi0 - sy.lo0 + 1, nrows = n0 + (sy.n == 2 ? sy.hi1 - sy.lo1 + 1 : 0);
        for (int j = lane; j < nrows * sx.n; j += GL) {
            const int ri = j / sx.n, c = j % sx.n;
            const int row = ri < n0 ? sy.lo0 + ri : sy.lo1 + (ri - n0);
            const int e0 = cs[row * B.ntx + sx.lo(c)], e1 = cs[row * B.ntx + sx.hi(c) + 1];
            for (int e = e0; e < e1; ++e) {
                const int2 q = ld_int2(B.cell_q, e);
                const long long d = d2q(X, Y, q.x, q.y, MX, MY);
                if (d < bd) bd = d;
            }
        }
        group_min_dl<GL>(bd, dummy);
        if (bd != LLONG_MAX || (span_full(sx, B.ntx) && span_full(sy, B.nty))) break;
    }
    const double rho = sqrt((double)bd) / 256.0 + 1.0;
    const double px = X / 256.0, py = Y / 256.0;
    const Span sx = span_sites((int)floor(px - rho), (int)floor(px + rho), B.lx, B.open_x);
    const Span sy = span_sites((int)floor(py - rho), (int)floor(py + rho), B.ly, B.open_y);
    const int n0 = sy.hi0 - sy.lo0 + 1, nrows = n0 + (sy.n == 2 ? sy.hi1 - sy.lo1 + 1 : 0);
    long long best = LLONG_MAX;
    int bl = DV_EMPTY;
    for (int j = lane; j < nrows * sx.n; j += GL) {
        const int ri = j / sx.n, c = j % sx.n;
        const int row = ri < n0 ? sy.lo0 + ri : sy.lo1 + (ri - n0);
        const int e0 = cs[row * B.ntx + sx.lo(c)], e1 = cs[row * B.ntx + sx.hi(c) + 1];
        for (int e = e0; e < e1; ++e) {
            const int2 q = ld_int2(B.cell_q, e);
            const long long d = d2q(X, Y, q.x, q.y, MX, MY);
            const int lab = gmem(B.cell_items)[e];
            if (d < best || (d == best && lab < bl)) { best = d; bl = lab; }
        }
    }
    group_min_dl<GL>(best, bl);
    return bl;
}

// Block-wide exclusive scan of in[0, n) into out[0, n); returns the total.
// Every thread of the block must call it.  blockDim.x is a multiple of 64.
__device__ int block_exclusive_scan(const int *in, int *out, int n, int *wsum /* LDS [16] */) {
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6, nw = blockDim.x >> 6;
    int carry = 0;
    for (int c0 = 0; c0 < n; c0 += blockDim.x) {
        const int i = c0 + t;
        const int v = i < n ? in[i] : 0;
        const int x = wave_incl_sum(v);
        __syncthreads();
        if (lane == 63) wsum[wid] = x;
        __syncthreads();
        int before = carry;
        for (int w = 0; w < wid; ++w) before += wsum[w];
        if (i < n) out[i] = before + x - v;
        int tot = 0;
        for (int w = 0; w < nw; ++w) tot += wsum[w];
        carry += tot;
    }
    return carry;
}

// The same, each thread taking a contiguous run of up to PER elements per
// pass (PER * blockDim.x elements a pass: one pass for the usual sizes), the
// loads of a run issued together.
template <int PER>
__device__ int block_exclusive_scan_wide(const int *in, int *out, int n, int *wsum /* LDS [16] */) {
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6, nw = blockDim.x >> 6;
    const int nthr = (int)blockDim.x;
    int carry = 0;
    for (int c0 = 0; c0 < n; c0 += nthr * PER) {
        const int m = min(n - c0, nthr * PER);
        const int per = (m + nthr - 1) / nthr;
        const int b = c0 + t * per;
        const int e = min(b + per, c0 + m);
        int v[PER];
        int sum = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            v[k] = b + k < e ? in[b + k] : 0;
            sum += v[k];
        }
        const int x = wave_incl_sum(sum);
        __syncthreads();
        if (lane == 63) wsum[wid] = x;
        __syncthreads();
        int before = carry + x - sum;
        for (int w = 0; w < wid; ++w) before += wsum[w];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (b + k < e) out[b + k] = before;
            before += v[k];
        }
        int tot = 0;
        for (int w = 0; w < nw; ++w) tot += wsum[w];
        carry += tot;
    }
    return carry;
}
