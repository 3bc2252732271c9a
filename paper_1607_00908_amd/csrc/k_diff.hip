// Isomorphism, translation, trigger and flips (Sec. 3.2.3 and 3.2.4).
//
//   k_match       Phi(p) = nearest now centre of past centre p (exact, ties to
//                 the lowest label) through the now bucket grid; preimage
//                 counts; inverse map
//   k_diff_count  one thread per now row n with exactly one preimage p: the
//                 past row of p translated through Phi (kept entries only,
//                 sorted) is compared with row n (kept entries only); counts
//                 the breaking (only past) and arising (only now) couples with
//                 the other end above n, and the local trigger of p
//   k_diff_scan   offsets of every row's flips (breaking first, then arising,
//                 each in (a, b) order)
//   k_diff_write  writes the flip records
//   k_commit      the frame becomes the past when it was accepted
#include "dv_device.h"

namespace {

__global__ __launch_bounds__(256) void k_match(Bufs B) {
    DevState *st = B.st;
    if (st->err || !st->past_valid) return;
    const int past = st->sel;
    const int KP = st->K[past], KN = st->K_now;
    const CompBuf P = B.comp[past];
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < KP; p += gridDim.x * blockDim.x) {
        if (KN == 0) { B.phi[p] = -1; continue; }
        const int n = point_nearest(B, P.qx[p], P.qy[p]);
        B.phi[p] = n;
        atomicAdd(&B.cnt[n], 1);
        B.inv[n] = p;
    }
}

#define MAXD 64   // largest supported row capacity

// Translated past row of p: pairs (Phi(q), q) for kept neighbours q, sorted by
// Phi(q).  Returns its length.
__device__ int translated_row(const Bufs &B, const CompBuf &P, int p, int *tv, int *tq) {
    const int *row = P.adj + (size_t)p * B.maxdeg;
    const int d = P.deg[p];
    int m = 0;
    for (int i = 0; i < d; ++i) {
        const int q = row[i];
        const int n = B.phi[q];
        if (n < 0 || B.cnt[n] != 1) continue;
        int j = m - 1;
        while (j >= 0 && tv[j] > n) { tv[j + 1] = tv[j]; tq[j + 1] = tq[j]; --j; }
        tv[j + 1] = n;
        tq[j + 1] = q;
        ++m;
    }
    return m;
}

__global__ __launch_bounds__(256) void k_diff_count(Bufs B) {
    DevState *st = B.st;
    if (st->err) return;
    const int KN = st->K_now;
    const int past = st->sel, now = 1 - past;
    const bool pv = st->past_valid != 0;
    const int KP = pv ? st->K[past] : 0;
    const CompBuf P = B.comp[past], N = B.comp[now];
    int exn = 0, exp_ = 0;
    const int stride = gridDim.x * blockDim.x;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    // dropped past points: Phi is reported as -1 (a concurrent reader of
    // phi[q] skips q either way)
    for (int p = tid; p < KP; p += stride) {
        const int n = B.phi[p];
        if (n < 0 || B.cnt[n] != 1) { B.trigger[p] = 0; B.phi[p] = -1; ++exp_; }
    }
    int tv[MAXD], tq[MAXD];
    for (int n = tid; n < KN; n += stride) {
        int cb = 0, ca = 0;
        if (pv) {
            if (B.cnt[n] != 1) {
                ++exn;
            } else {
                const int p = B.inv[n];
                const int m = translated_row(B, P, p, tv, tq);
                const int *row = N.adj + (size_t)n * B.maxdeg;
                const int d = N.deg[n];
                int i = 0, j = 0;
                bool differ = false;
                // merge of two sorted lists; now entries without exactly one
                // preimage are skipped
                while (i < m || j < d) {
                    if (j < d && B.cnt[row[j]] != 1) { ++j; continue; }
                    if (j >= d || (i < m && tv[i] < row[j])) {
                        differ = true;
                        if (tv[i] > n) ++cb;
                        ++i;
                    } else if (i >= m || row[j] < tv[i]) {
                        differ = true;
                        if (row[j] > n) ++ca;
                        ++j;
                    } else {
                        ++i;
                        ++j;
                    }
                }
                B.trigger[p] = differ ? 1 : 0;
            }
        }
        B.nb[n] = cb;
        B.na[n] = ca;
    }
    for (int o = 32; o > 0; o >>= 1) {
        exn += __shfl_down(exn, o, 64);
        exp_ += __shfl_down(exp_, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (exn) atomicAdd(&st->n_excl_now, exn);
        if (exp_) atomicAdd(&st->n_excl_past, exp_);
    }
}

__global__ __launch_bounds__(1024) void k_diff_scan(Bufs B) {
    __shared__ int wsum[16];
    DevState *st = B.st;
    if (st->err) return;
    const int KN = st->K_now;
    const int nbk = block_exclusive_scan(B.nb, B.ob, KN, wsum);
    __syncthreads();
    const int nar = block_exclusive_scan(B.na, B.oa, KN, wsum);
    if (threadIdx.x == 0) {
        st->n_break = nbk;
        st->n_flips = nbk + nar;
        st->global_trigger = (nbk + nar) > 0 ? 1 : 0;
    }
}

__global__ __launch_bounds__(256) void k_diff_write(Bufs B) {
    DevState *st = B.st;
    if (st->err || !st->past_valid) return;
    const int KN = st->K_now;
    const int past = st->sel, now = 1 - past;
    const CompBuf P = B.comp[past], N = B.comp[now];
    const int nbk = st->n_break;
    int tv[MAXD], tq[MAXD];
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < KN; n += gridDim.x * blockDim.x) {
        if (B.nb[n] == 0 && B.na[n] == 0) continue;
        const int p = B.inv[n];
        const int m = translated_row(B, P, p, tv, tq);
        const int *row = N.adj + (size_t)n * B.maxdeg;
        const int d = N.deg[n];
        int *fb = B.flips + (size_t)6 * B.ob[n];
        int *fa = B.flips + (size_t)6 * (nbk + B.oa[n]);
        int i = 0, j = 0;
        while (i < m || j < d) {
            if (j < d && B.cnt[row[j]] != 1) { ++j; continue; }
            if (j >= d || (i < m && tv[i] < row[j])) {
                if (tv[i] > n) {
                    fb[0] = n; fb[1] = tv[i]; fb[2] = p; fb[3] = tq[i]; fb[4] = -1; fb[5] = 0;
                    fb += 6;
                }
                ++i;
            } else if (i >= m || row[j] < tv[i]) {
                const int mm = row[j];
                if (mm > n) {
                    fa[0] = n; fa[1] = mm; fa[2] = p; fa[3] = B.inv[mm]; fa[4] = 1; fa[5] = 0;
                    fa += 6;
                }
                ++j;
            } else {
                ++i;
                ++j;
            }
        }
    }
}

__global__ void k_commit(Bufs B) {
    DevState *st = B.st;
    if (st->err) {
        st->status = 2;   // DV_ERR_CAPACITY
        st->n_flips = 0;
        st->n_break = 0;
        st->global_trigger = 0;
        return;
    }
    const int past = st->sel, now = 1 - past;
    st->K_past_cmp = st->past_valid ? st->K[past] : 0;
    st->K[now] = st->K_now;
    st->E[now] = st->E2_now / 2;
    st->sel = now;
    st->past_valid = 1;
    st->frame += 1;
    st->status = 0;
}

// ---- inspection: sorted couple list (a < b) of the current buffer ----------
__global__ __launch_bounds__(256) void k_edge_count(Bufs B, int *cntv) {
    DevState *st = B.st;
    const int cur = st->sel;
    const int K = st->K[cur];
    const CompBuf C = B.comp[cur];
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < K; a += gridDim.x * blockDim.x) {
        const int *row = C.adj + (size_t)a * B.maxdeg;
        int c = 0;
        for (int i = 0; i < C.deg[a]; ++i) c += row[i] > a ? 1 : 0;
        cntv[a] = c;
    }
}

__global__ __launch_bounds__(1024) void k_edge_scan(Bufs B, const int *cntv, int *offv, int *total) {
    __shared__ int wsum[16];
    const int K = B.st->K[B.st->sel];
    const int tot = block_exclusive_scan(cntv, offv, K, wsum);
    if (threadIdx.x == 0) *total = tot;
}

__global__ __launch_bounds__(256) void k_edge_write(Bufs B, const int *offv, int *ab) {
    DevState *st = B.st;
    const int cur = st->sel;
    const int K = st->K[cur];
    const CompBuf C = B.comp[cur];
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < K; a += gridDim.x * blockDim.x) {
        const int *row = C.adj + (size_t)a * B.maxdeg;
        int o = offv[a];
        for (int i = 0; i < C.deg[a]; ++i)
            if (row[i] > a) {
                ab[2 * o] = a;
                ab[2 * o + 1] = row[i];
                ++o;
            }
    }
}

}  // namespace

void launch_diff(const Bufs &B, hipStream_t s, Prof &P) {
    const int kgrid = (int)std::min<long long>((B.kmax + 255) / 256, 1024);
    P.begin(ST_MATCH, s);
    hipLaunchKernelGGL(k_match, dim3(kgrid), dim3(256), 0, s, B);
    P.end(ST_MATCH, s);
    P.begin(ST_DIFF_COUNT, s);
    hipLaunchKernelGGL(k_diff_count, dim3(kgrid), dim3(256), 0, s, B);
    P.end(ST_DIFF_COUNT, s);
    P.begin(ST_DIFF_SCAN, s);
    hipLaunchKernelGGL(k_diff_scan, dim3(1), dim3(1024), 0, s, B);
    P.end(ST_DIFF_SCAN, s);
    P.begin(ST_DIFF_WRITE, s);
    hipLaunchKernelGGL(k_diff_write, dim3(kgrid), dim3(256), 0, s, B);
    P.end(ST_DIFF_WRITE, s);
    P.begin(ST_COMMIT, s);
    hipLaunchKernelGGL(k_commit, dim3(1), dim3(1), 0, s, B);
    P.end(ST_COMMIT, s);
}

void launch_edge_list(const Bufs &B, int32_t *d_out_ab, int32_t *d_count, int32_t *d_scratch,
                      hipStream_t s) {
    const int kgrid = (int)std::min<long long>((B.kmax + 255) / 256, 1024);
    int *cntv = d_scratch, *offv = d_scratch + B.kmax;
    hipLaunchKernelGGL(k_edge_count, dim3(kgrid), dim3(256), 0, s, B, cntv);
    hipLaunchKernelGGL(k_edge_scan, dim3(1), dim3(1024), 0, s, B, (const int *)cntv, offv, d_count);
    hipLaunchKernelGGL(k_edge_write, dim3(kgrid), dim3(256), 0, s, B, (const int *)offv, d_out_ab);
}
