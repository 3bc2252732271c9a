// Comparison of every frame of a batch with its past (Sec. 3.2.3 and 3.2.4),
// one launch per step for the whole batch (frame = blockIdx.z).  The past of
// a frame is the last earlier frame of the batch that passed its stage checks
// (known on the device from the frame headers), else the shared past buffer,
// so the comparisons of a batch are independent of each other.
//
//   k_match   Phi(p) = nearest now centre of every past centre p, a group
//             of 16 lanes per point through the frame's bucket grid, exact,
//             ties to the lowest label; preimage counts of the now points.
//   k_diff    one wave per now label n.  The batch's last accepted frame
//             copies its components and rows into the spare past buffer (the
//             past of the next batch).  When n has exactly one preimage p,
//             lane j holds slot j of the now row of n and slot j of the past
//             row of p translated through Phi (kept entries only).  Rows are
//             sets, so membership is tested with wave shuffles.  A couple of
//             T(p) missing from R(n) is breaking, one of R(n) missing from
//             T(p) is arising; each is reported once, from the row of its
//             smaller now label, and staged in increasing order of the other
//             end.  The local trigger of p is set when the two rows differ.
//   k_events  (event classification only) one wave per changed row: active
//             neighbours in either graph, boundary points of either graph.
//   k_place   one block per frame: scans the per-row counts and places the
//             staged flips in canonical order (breaking first, then arising,
//             each by (a, b)) in the results page, and writes the frame's
//             record.  Kept past and now points correspond one to one, so the
//             number of dropped past points is K_past - (K_now - dropped now
//             points).
//   k_commit  every sequence of the launch: its spare past buffer becomes the
//             past when any of its frames was accepted.
#include "dv_device.h"

namespace {

// past components of frame i: slot j's frame, or the shared buffer
struct PastOf {
    CompBuf C;
    int K;
    bool valid;
};

// (every lane of the calling wave must make the call)

__device__ __forceinline__ PastOf past_of_slot(const Bufs *D, const Batch &G, int i, int j) {
    PastOf r;
    if (j >= 0) {
        r.C = D[G.idx[j]].cur;
        r.K = D[G.idx[j]].fs->K_now;
        r.valid = true;
    } else {
        const SeqState *st = D[G.idx[i]].st;
        r.C = D[G.idx[i]].past[st->sel];
        r.K = st->past_valid ? st->K[st->sel] : 0;
        r.valid = st->past_valid != 0;
    }
    return r;
}

// Past of frame i (every lane of the calling wave must make the call: lane j
// loads entry j); for one-block-per-frame kernels.
__device__ __forceinline__ PastOf past_of(const Bufs *D, const Batch &G, int i,
                                          unsigned long long accepted) {
    return past_of_slot(D, G, i, past_slot(accepted, i));
}

// (by the scalar walk: the per-row kernels run many waves per frame)
__device__ __forceinline__ PastOf past_of(const Bufs *D, const Batch &G, int i) {
    return past_of_slot(D, G, i, past_slot_walk(D, G, i));
}

#define MATCH_LANES 16
__global__ __launch_bounds__(256) void k_match(const Bufs *__restrict__ D, Batch G) {
    const Bufs B = D[G.idx[blockIdx.z]];
    if (B.fs->err) return;
    const PastOf P = past_of(D, G, blockIdx.z);
    if (!P.valid) return;
    const int KP = P.K, KN = B.fs->K_now;
    // a group of MATCH_LANES lanes per past centre (the search of one point
    // rarely visits more cells than that)
    const int lane = threadIdx.x & (MATCH_LANES - 1);
    const int ng = blockDim.x / MATCH_LANES;
    for (int p = blockIdx.x * ng + (threadIdx.x / MATCH_LANES); p < KP; p += gridDim.x * ng) {
        int n = -1;
        if (KN > 0) n = group_nearest<MATCH_LANES>(B, gmem(P.C.qx)[p], gmem(P.C.qy)[p]);
        if (lane == 0) {
            gmem(B.phi)[p] = n;
            if (n >= 0) {
                atomicAdd(&B.cnt[n], 1);
                gmem(B.inv)[n] = p;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_diff(const Bufs *__restrict__ Dt, Batch G) {
    __shared__ int s_red[4][4];
    const int i = blockIdx.z;
    const Bufs &B = Dt[G.idx[i]];
    FrameState *fs = B.fs;
    if (fs->err) return;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int KN = fs->K_now;
    const PastOf PO = past_of(Dt, G, i);
    const bool pv = PO.valid;
    const CompBuf P = PO.C, N = B.cur, Q = B.past[1 - B.st->sel];
    // the sequence's last accepted frame of the launch leaves its copy for the
    // next launch
    bool keep = true;
    for (int q = i + 1; q < G.n; ++q)
        if (Dt[G.idx[q]].seq == B.seq && Dt[G.idx[q]].fs->err == 0) keep = false;
    const int D = B.maxdeg;
    int e2 = 0, exn = 0, tb = 0, ta = 0;
    const int nwaves = gridDim.x * (blockDim.x >> 6);
    for (int n = blockIdx.x * (blockDim.x >> 6) + wid; n < KN; n += nwaves) {
        const int m = lane < D ? gmem(N.adj)[(size_t)n * D + lane] : DV_EMPTY;
        if (keep) {
            if (lane < D) gmem(Q.adj)[(size_t)n * D + lane] = m;
            switch (lane) {
                case 0: Q.qx[n] = N.qx[n]; break;
                case 1: Q.qy[n] = N.qy[n]; break;
                case 2: Q.fx[n] = N.fx[n]; break;
                case 3: Q.fy[n] = N.fy[n]; break;
                case 4: Q.n[n] = N.n[n]; break;
                case 5: Q.root[n] = N.root[n]; break;
                case 6: Q.amb[n] = N.amb[n]; break;
                default: break;
            }
        }
        const int cn = gmem(B.cnt)[n];
        const int p = gmem(B.inv)[n];
        const int dR = __popcll(__ballot(m != DV_EMPTY));
        if (lane == 0) e2 += dR;
        int cb = 0, ca = 0, actv = 0;
        if (pv && cn != 1) {
            if (lane == 0) ++exn;
        } else if (pv) {
            const int q = lane < D ? gmem(P.adj)[(size_t)p * D + lane] : DV_EMPTY;
            const int dT = __popcll(__ballot(q != DV_EMPTY));
            const int mv = (m != DV_EMPTY && gmem(B.cnt)[m] == 1) ? m : DV_EMPTY;
            int tv = DV_EMPTY;
            if (q != DV_EMPTY) {
                const int nn = gmem(B.phi)[q];
                if (nn >= 0 && gmem(B.cnt)[nn] == 1) tv = nn;
            }
            // slots are filled from the front: the first dR (dT) lanes
            bool tin = false, min_ = false;
            for (int k = 0; k < dR; ++k) tin |= (__shfl(mv, k, 64) == tv);
            for (int k = 0; k < dT; ++k) min_ |= (__shfl(tv, k, 64) == mv);
            const bool brk = tv != DV_EMPTY && !tin;
            const bool ari = mv != DV_EMPTY && !min_;
            const unsigned long long dmask = __ballot(brk || ari);
            if (lane == 0) gmem(B.trigger)[p] = dmask ? 1 : 0;
            actv = dmask ? 1 : 0;
            // each couple once, from the row of its smaller now label
            const bool bo = brk && tv > n, ao = ari && mv > n;
            cb = __popcll(__ballot(bo));
            ca = __popcll(__ballot(ao));
            gint *stg = gmem(B.stage) + (size_t)n * (2 * D) * 6;
            const int bv = bo ? tv : DV_EMPTY, av = ao ? mv : DV_EMPTY;
            int rb = 0, ra = 0;
            for (int k = 0; k < dT; ++k) rb += (__shfl(bv, k, 64) < bv) ? 1 : 0;
            for (int k = 0; k < dR; ++k) ra += (__shfl(av, k, 64) < av) ? 1 : 0;
            if (bo) {
                gint *r = stg + 6 * rb;
                r[0] = n; r[1] = tv; r[2] = p; r[3] = q; r[4] = -1; r[5] = 0;
            }
            if (ao) {
                gint *r = stg + 6 * (D + ra);
                r[0] = n; r[1] = mv; r[2] = p; r[3] = gmem(B.inv)[mv]; r[4] = 1; r[5] = 0;
            }
        }
        if (lane == 0) {
            gmem(B.nb)[n] = cb;
            gmem(B.na)[n] = ca;
            tb += cb;
            ta += ca;
            if (B.classify) gmem(B.act)[n] = actv;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        e2 += __shfl_down(e2, o, 64);
        exn += __shfl_down(exn, o, 64);
        tb += __shfl_down(tb, o, 64);
        ta += __shfl_down(ta, o, 64);
    }
    if (lane == 0) {
        s_red[0][wid] = e2;
        s_red[1][wid] = exn;
        s_red[2][wid] = tb;
        s_red[3][wid] = ta;
    }
    __syncthreads();
    if (t == 0) {
        int a = 0, b = 0, c = 0, d = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            a += s_red[0][w];
            b += s_red[1][w];
            c += s_red[2][w];
            d += s_red[3][w];
        }
        if (a) atomicAdd(&fs->E2_acc, a);
        if (b) atomicAdd(&fs->excl_acc, b);
        // flip totals of the frame: the next launch places every frame's flips
        // after those of the frames before it in the results page
        if (c) atomicAdd(&fs->nb_acc, c);
        if (d) atomicAdd(&fs->na_acc, d);
    }
}

// Event classification (Sec. 3.2.4), one wave per active now label n (an end
// of a flip): the active points connected to n in either graph, and whether
// n is a boundary point of the now graph and of the translated past graph
// (one of its couples has ends sharing fewer than two neighbours).  Both
// graphs keep only points with exactly one preimage, as in k_diff.  The
// wave's two rows sit in LDS for the membership tests of its lanes.
__global__ __launch_bounds__(256) void k_events(const Bufs *__restrict__ Dt, Batch G) {
    __shared__ int rowR[4][64], rowT[4][64];
    const int i = blockIdx.z;
    const Bufs B = Dt[G.idx[i]];
    const FrameState *fs = B.fs;
    if (!B.classify || fs->err) return;
    const PastOf PO = past_of(Dt, G, i);
    if (!PO.valid) return;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int KN = fs->K_now, D = B.maxdeg;
    const CompBuf P = PO.C, N = B.cur;
    const auto cnt = gmem(B.cnt), phi = gmem(B.phi), inv = gmem(B.inv), act = gmem(B.act);
    const int nwaves = gridDim.x * (blockDim.x >> 6);
    for (int n = blockIdx.x * (blockDim.x >> 6) + wid; n < KN; n += nwaves) {
        if (!act[n]) continue;
        const int m = lane < D ? gmem(N.adj)[(size_t)n * D + lane] : DV_EMPTY;
        const int mv = (m != DV_EMPTY && cnt[m] == 1) ? m : DV_EMPTY;
        const int p = inv[n];
        const int q = lane < D ? gmem(P.adj)[(size_t)p * D + lane] : DV_EMPTY;
        int tv = DV_EMPTY;
        if (q != DV_EMPTY) {
            const int nn = phi[q];
            if (nn >= 0 && cnt[nn] == 1) tv = nn;
        }
        rowR[wid][lane] = mv;
        rowT[wid][lane] = tv;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        bool tin = false;
        for (int k = 0; k < D; ++k) tin |= (tv != DV_EMPTY && rowR[wid][k] == tv);
        const bool aR = mv != DV_EMPTY && act[mv];
        const bool aT = tv != DV_EMPTY && !tin && act[tv];
        const int count = __popcll(__ballot(aR)) + __popcll(__ballot(aT));
        // a couple (n, x) is a boundary couple when n and x share fewer than
        // two neighbours; x's row is read from memory, n's from LDS
        bool bN = false, bP = false;
        if (mv != DV_EMPTY) {
            int c = 0;
            for (int k = 0; k < D && c < 2; ++k) {
                const int x = gmem(N.adj)[(size_t)mv * D + k];
                if (x == DV_EMPTY) break;
                if (cnt[x] != 1) continue;
                for (int j = 0; j < D; ++j)
                    if (rowR[wid][j] == x) { ++c; break; }
            }
            bN = c < 2;
        }
        if (tv != DV_EMPTY) {
            const int pt = inv[tv];
            int c = 0;
            for (int k = 0; k < D && c < 2; ++k) {
                const int q2 = gmem(P.adj)[(size_t)pt * D + k];
                if (q2 == DV_EMPTY) break;
                const int x = phi[q2];
                if (x < 0 || cnt[x] != 1) continue;
                for (int j = 0; j < D; ++j)
                    if (rowT[wid][j] == x) { ++c; break; }
            }
            bP = c < 2;
        }
        const bool anyN = __ballot(bN) != 0ull, anyP = __ballot(bP) != 0ull;
        if (lane == 0) {
            gmem(B.ecnt)[n] = count;
            gmem(B.ebnd)[n] = (anyN ? 1 : 0) | (anyP ? 2 : 0);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// flags of a placed flip record (a, b, pa, pb, kind, flags)
__device__ __forceinline__ int event_flags(const Bufs &B, int a, int b, int kind) {
    const auto ecnt = gmem(B.ecnt), ebnd = gmem(B.ebnd);
    int f = (ecnt[a] >= 3 && ecnt[b] >= 3) ? 1 : 0;
    const int bit = kind < 0 ? 2 : 1;
    if ((ebnd[a] & bit) && (ebnd[b] & bit)) f |= 2;
    return f;
}

// n 8-byte words from src to dst (distinct buffers), four loads in flight
__device__ __forceinline__ void copy_words(const int2 *__restrict__ src, int2 *__restrict__ dst, int n) {
    const auto s = gmem(reinterpret_cast<const unsigned long long *>(src));
    const auto d = gmem(reinterpret_cast<unsigned long long *>(dst));
    int j = 0;
    for (; j + 4 <= n; j += 4) {
        const unsigned long long a0 = s[j], a1 = s[j + 1], a2 = s[j + 2], a3 = s[j + 3];
        d[j] = a0;
        d[j + 1] = a1;
        d[j + 2] = a2;
        d[j + 3] = a3;
    }
    for (; j < n; ++j) d[j] = s[j];
}

// rows per thread of k_place's one-pass form (K up to 16 x 1024 rows)
#define PLACE_PER 16
__global__ __launch_bounds__(1024) void k_place(const Bufs *__restrict__ Dt, Batch G) {
    __shared__ int wsum[16], wsb2[16];
    __shared__ int s_before[2];
    const int i = blockIdx.z;
    const Bufs &B = Dt[G.idx[i]];
    FrameState *fs = B.fs;
    const int t = threadIdx.x;
    // results page of the frame: the flips of the page before it are those
    // the page held before the launch and those of the earlier accepted frames
    // of the same sequence in the launch (all of one sequence share one page);
    // lane j of the first wave takes entry j (at most 64 entries)
    if (t < 64) {
        int nfl = 0, acc = 0;
        if (t < i) {
            const Bufs &Bj = Dt[G.idx[t]];
            const FrameState *fj = Bj.fs;
            if (Bj.seq == B.seq && fj->err == 0) {
                nfl = fj->nb_acc + fj->na_acc;
                acc = 1;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            nfl += __shfl_xor(nfl, o, 64);
            acc += __shfl_xor(acc, o, 64);
        }
        if (t == 0) {
            s_before[0] = nfl;
            s_before[1] = acc;
        }
    }
    __syncthreads();
    const uint32_t ps = G.pslot[i];
    const int pg = DV_PG_PAGE(ps);
    const SeqState *sq0 = B.st;
    const int base = (DV_PG_FRESH(ps) ? 0 : sq0->pg_fill[pg]) + s_before[0];
    long long frame_no = sq0->frame + s_before[1];
    int *const flips = B.pg_flips[pg] + (size_t)6 * base;
    if (fs->err) {
        if (t == 0) {
            fs->status = 2;   // DV_ERR_CAPACITY; the frame is not a past
            fs->n_flips = 0;
            fs->n_break = 0;
            fs->n_excl_past = 0;
            fs->n_excl_now = 0;
            fs->global_trigger = 0;
            fs->K_past = 0;
            fs->E_now = 0;
        }
    } else {
        ++frame_no;
        const int KN = fs->K_now;
        const PastOf PO = past_of(Dt, G, i, accepted_entries(Dt, G, B.seq));
        const int D = B.maxdeg;
        // row n's staged flips to their places in the frame's list; records
        // are 24 bytes, copied as 8-byte words with the loads issued together
        auto place_row = [&](int n, int cb, int ca, int offb, int offa) {
            const int *stg = B.stage + (size_t)n * (2 * D) * 6;
            int *fb = flips + (size_t)6 * offb;
            int *fa = flips + (size_t)6 * offa;
            copy_words(reinterpret_cast<const int2 *>(stg), reinterpret_cast<int2 *>(fb), 3 * cb);
            copy_words(reinterpret_cast<const int2 *>(stg + 6 * D), reinterpret_cast<int2 *>(fa), 3 * ca);
            if (B.classify) {
                for (int j = 0; j < cb; ++j) fb[6 * j + 5] = event_flags(B, fb[6 * j], fb[6 * j + 1], -1);
                for (int j = 0; j < ca; ++j) fa[6 * j + 5] = event_flags(B, fa[6 * j], fa[6 * j + 1], 1);
            }
        };
        int nbk, nar;
        if (KN <= PLACE_PER * (int)blockDim.x) {
            // one pass: thread t holds the counts of a contiguous run of rows
            // (their loads issued together), both prefix sums are one block
            // scan, and the copies start from the registers
            const int per = (KN + blockDim.x - 1) / blockDim.x;
            const int b0 = t * per, e0 = min(b0 + per, KN);
            int vb[PLACE_PER], va[PLACE_PER];
            int sb = 0, sa = 0;
#pragma unroll
            for (int k = 0; k < PLACE_PER; ++k) {
                vb[k] = b0 + k < e0 ? gmem(B.nb)[b0 + k] : 0;
                va[k] = b0 + k < e0 ? gmem(B.na)[b0 + k] : 0;
                sb += vb[k];
                sa += va[k];
            }
            const int lane = t & 63, wid = t >> 6, nw = blockDim.x >> 6;
            const int xb = wave_incl_sum(sb), xa = wave_incl_sum(sa);
            if (lane == 63) {
                wsum[wid] = xb;
                wsb2[wid] = xa;
            }
            __syncthreads();
            int offb = xb - sb, offa = xa - sa;
            nbk = 0;
            nar = 0;
            for (int w = 0; w < nw; ++w) {
                const int pb = wsum[w], pa = wsb2[w];
                offb += w < wid ? pb : 0;
                offa += w < wid ? pa : 0;
                nbk += pb;
                nar += pa;
            }
            offa += nbk;   // arising flips follow every breaking one
#pragma unroll
            for (int k = 0; k < PLACE_PER; ++k) {
                if ((vb[k] | va[k]) != 0) place_row(b0 + k, vb[k], va[k], offb, offa);
                offb += vb[k];
                offa += va[k];
            }
        } else {
            nbk = block_exclusive_scan_wide<16>(B.nb, B.ob, KN, wsum);
            __syncthreads();
            nar = block_exclusive_scan_wide<16>(B.na, B.oa, KN, wsum);
            __syncthreads();
            for (int n = t; n < KN; n += blockDim.x) {
                const int cb = B.nb[n], ca = B.na[n];
                if (cb == 0 && ca == 0) continue;
                place_row(n, cb, ca, B.ob[n], nbk + B.oa[n]);
            }
        }
        if (t == 0) {
            const int KP = PO.valid ? PO.K : 0;
            const int excl = fs->excl_acc;
            fs->status = 0;
            fs->K_past = KP;
            fs->E_now = fs->E2_acc / 2;
            fs->n_excl_now = excl;
            fs->n_excl_past = PO.valid ? KP - (KN - excl) : 0;
            fs->n_break = nbk;
            fs->n_flips = nbk + nar;
            fs->global_trigger = (nbk + nar) > 0 ? 1 : 0;
        }
    }
    if (t == 0) {
        // the frame's result record (host memory, read after the launch)
        FrameOut r;
        r.frame = frame_no;
        r.status = fs->status;
        r.K = fs->K_now;
        r.E = fs->E_now;
        r.n_flips = fs->n_flips;
        r.n_break = fs->n_break;
        r.excl_past = fs->n_excl_past;
        r.excl_now = fs->n_excl_now;
        r.amb = fs->n_amb;
        r.trigger = fs->global_trigger;
        r.flip_off = base;
        r.pad[0] = r.pad[1] = r.pad[2] = 0;
        B.pg_info[pg][DV_PG_POS(ps)] = r;
    }
}

// Commit of every sequence of the launch, after k_place (a kernel of its own:
// a last-block ticket in k_place would need a device-wide release in every
// block).  Lane k of one wave takes entry k and commits its sequence when k is
// the sequence's last entry in the launch: the spare past buffer becomes the
// past when any of its frames was accepted; the entries' values reach the
// other lanes by shuffles.
__global__ __launch_bounds__(64) void k_commit(const Bufs *__restrict__ Dt, Batch G) {
    const int nb_frames = G.n;
    const int k = threadIdx.x;
    int q = -1, ok = 0, nfl = 0, Kn = 0, E2 = 0;
    if (k < nb_frames) {
        const Bufs &Bk = Dt[G.idx[k]];
        const FrameState *fk = Bk.fs;
        q = Bk.seq;
        ok = fk->err == 0;
        if (ok) {
            nfl = fk->nb_acc + fk->na_acc;
            Kn = fk->K_now;
            E2 = fk->E2_acc;
        }
    }
    bool last = k < nb_frames;
    int acc = 0, sum = 0, Ka = -1, E2a = 0;
    for (int j = 0; j < nb_frames; ++j) {
        const int qj = __shfl(q, j, 64), okj = __shfl(ok, j, 64), nj = __shfl(nfl, j, 64);
        const int Kj = __shfl(Kn, j, 64), Ej = __shfl(E2, j, 64);
        if (j > k && qj == q) last = false;
        if (j <= k && qj == q && okj) {
            ++acc;
            sum += nj;
            Ka = Kj;
            E2a = Ej;
        }
    }
    if (last) {
        SeqState *sq = Dt[G.idx[k]].st;
        const uint32_t pk = G.pslot[k];
        const int p = DV_PG_PAGE(pk);
        sq->pg_fill[p] = (DV_PG_FRESH(pk) ? 0 : sq->pg_fill[p]) + sum;
        if (acc > 0) {
            const int nxt = 1 - sq->sel;
            sq->K[nxt] = Ka;
            sq->E[nxt] = E2a / 2;
            sq->sel = nxt;
            sq->past_valid = 1;
            sq->frame += acc;
        }
    }
}

// Phi of the most recent comparison with dropped past points as -1 (inspection).
__global__ __launch_bounds__(256) void k_phi_out(const Bufs *__restrict__ D, int slot, int *out) {
    const Bufs &B = D[slot];
    const int KP = B.fs->K_past;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < KP; p += gridDim.x * blockDim.x) {
        const int n = B.phi[p];
        out[p] = (n >= 0 && B.cnt[n] == 1) ? n : -1;
    }
}

// ---- inspection: sorted couple list (a < b) of the past buffer -------------
__global__ __launch_bounds__(256) void k_edge_count(const Bufs *__restrict__ D, int *cntv) {
    const Bufs &B = D[0];
    const SeqState *st = B.st;
    const int cur = st->sel;
    const int K = st->K[cur];
    const CompBuf C = B.past[cur];
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < K; a += gridDim.x * blockDim.x) {
        const int *row = C.adj + (size_t)a * B.maxdeg;
        int c = 0;
        for (int i = 0; i < B.maxdeg && row[i] != DV_EMPTY; ++i) c += row[i] > a ? 1 : 0;
        cntv[a] = c;
    }
}

__global__ __launch_bounds__(1024) void k_edge_scan(const Bufs *__restrict__ D, const int *cntv,
                                                    int *offv, int *total) {
    __shared__ int wsum[16];
    const SeqState *st = D[0].st;
    const int K = st->K[st->sel];
    const int tot = block_exclusive_scan(cntv, offv, K, wsum);
    if (threadIdx.x == 0) *total = tot;
}

// entries above a, written in increasing order (rows are unordered sets)
__global__ __launch_bounds__(256) void k_edge_write(const Bufs *__restrict__ D, const int *offv,
                                                     int *ab) {
    const Bufs &B = D[0];
    const SeqState *st = B.st;
    const int cur = st->sel;
    const int K = st->K[cur];
    const CompBuf C = B.past[cur];
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < K; a += gridDim.x * blockDim.x) {
        const int *row = C.adj + (size_t)a * B.maxdeg;
        const int o = offv[a];
        for (int i = 0; i < B.maxdeg && row[i] != DV_EMPTY; ++i) {
            const int v = row[i];
            if (v <= a) continue;
            int rank = 0;
            for (int j = 0; j < B.maxdeg && row[j] != DV_EMPTY; ++j)
                rank += (row[j] > a && row[j] < v) ? 1 : 0;
            ab[2 * (o + rank)] = a;
            ab[2 * (o + rank) + 1] = v;
        }
    }
}

}  // namespace

void launch_compare(const Batch &G, hipStream_t s, Prof &P) {
    // one wave per row, grid-stride: a quarter of K_max waves per frame
    // (K is usually well below K_max)
    const int grid = (int)std::max<long long>(1, std::min<long long>((G.kmax + 15) / 16, 512));
    P.begin(ST_MATCH, s);
    // (k_match: MATCH_LANES lanes per point, so a quarter of the blocks)
    const int mgrid = (int)std::max<long long>(1, std::min<long long>((G.kmax + 63) / 64, 512));
    hipLaunchKernelGGL(k_match, dim3(mgrid, 1, G.n), dim3(256), 0, s, G.D, G);
    P.end(ST_MATCH, s);
    P.begin(ST_DIFF, s);
    hipLaunchKernelGGL(k_diff, dim3(grid, 1, G.n), dim3(256), 0, s, G.D, G);
    P.end(ST_DIFF, s);
    if (G.classify) {
        P.begin(ST_EVENTS, s);
        hipLaunchKernelGGL(k_events, dim3(grid, 1, G.n), dim3(256), 0, s, G.D, G);
        P.end(ST_EVENTS, s);
    }
    P.begin(ST_PLACE, s);
    hipLaunchKernelGGL(k_place, dim3(1, 1, G.n), dim3(1024), 0, s, G.D, G);
    hipLaunchKernelGGL(k_commit, dim3(1), dim3(64), 0, s, G.D, G);
    P.end(ST_PLACE, s);
}

void launch_phi_out(const Bufs &H, const Bufs *D, int slot, int32_t *d_out, hipStream_t s) {
    const int grid = (int)std::min<long long>((H.kmax + 255) / 256, 1024);
    hipLaunchKernelGGL(k_phi_out, dim3(grid), dim3(256), 0, s, D, slot, d_out);
}

void launch_edge_list(const Bufs &H, const Bufs *D, int32_t *d_out_ab, int32_t *d_count,
                      int32_t *d_scratch, hipStream_t s) {
    const int kgrid = (int)std::min<long long>((H.kmax + 255) / 256, 1024);
    int *cntv = d_scratch, *offv = d_scratch + H.kmax;
    hipLaunchKernelGGL(k_edge_count, dim3(kgrid), dim3(256), 0, s, D, cntv);
    hipLaunchKernelGGL(k_edge_scan, dim3(1), dim3(1024), 0, s, D, (const int *)cntv, offv, d_count);
    hipLaunchKernelGGL(k_edge_write, dim3(kgrid), dim3(256), 0, s, D, (const int *)offv, d_out_ab);
}
