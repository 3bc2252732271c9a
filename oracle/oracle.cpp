// CPU oracle for the per-frame detection of topological changes in dynamic
// lattice Voronoi diagrams (Bernaschi, Lulli, Sbragaglia, arXiv:1607.00908).
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
// definition the HIP path is checked against.  Only the tests, the smoke entry
// and the benchmark's CPU-baseline leg may load it; the product path never does.
// It shares no code, header or table with the HIP path.
//
// Every step follows the paper (section numbers below) in the paper's order:
//   Sec. 3.1    threshold, cluster labelling, sizes, centres of mass
//   Sec. 3.2.1  digital Voronoi colouring by squared Euclidean distance
//   Sec. 3.2.2  frame gaps, first/second nearest-neighbour rules, compression
//   Sec. 3.2.3  kinematic isomorphism Phi_{P->N}, translation, row compare,
//               exclusion of appearing / disappearing points
//   Sec. 3.2.4  breaking / arising couples
// Readings where the paper is silent or ambiguous are stated at each step.
//
// Geometry (Sec. 3.2.1 obstacles, Sec. 3.2.2 frame on the domain boundary):
// every axis is periodic unless its bit is set in `open` (bit 0 = x, bit 1 =
// y).  On an open axis there is no wrap: components do not connect across
// the domain edge, offsets and distances are plain differences, and frame
// points beyond the edge read as MAXLINK (the frame keeps only neighbours
// inside the domain; a dropped point makes no gap).  `obst` (nullable, one
// byte per site, row-major) marks obstacle sites: they belong to no component
// and their colour is MAXLINK.  Inner-frame points are coloured by the
// nearest-centre rule alone (the obstacle field lives on the sites).
//
// Single-threaded except the per-site nearest-centre loops, which may use
// OpenMP over sites (each site is computed independently by the same loop).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <set>
#include <utility>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

const int32_t MAXLINK = 0x77777777;  // colour of "no cell" (Sec. 3.2.1 footnote)

// Signed minimum-image offset on a ring of length L:
// ((v + floor(L/2)) mod L) - floor(L/2), so the result lies in
// [-floor(L/2), L - 1 - floor(L/2)].
int64_t wrap_signed(int64_t v, int64_t L) {
    const int64_t h = L / 2;
    int64_t r = (v + h) % L;
    if (r < 0) r += L;
    return r - h;
}

int64_t pos_mod(int64_t v, int64_t m) {
    int64_t r = v % m;
    return r < 0 ? r + m : r;
}

// floor(a / b) for b > 0
int64_t floor_div(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b) != 0 && a < 0) q -= 1;
    return q;
}

// ---------------------------------------------------------------------------
// Sec. 3.1: a site belongs to a droplet when rho is above the threshold (the
// emulsion case, Sec. 4 footnote on phi_conc) or to a bubble when rho is below
// it.  Reading: strict comparison, so rho == threshold and NaN are outside.
// ---------------------------------------------------------------------------
bool inside(float rho, float thr, int phase) {
    return phase == 0 ? (rho > thr) : (rho < thr);
}

struct UF {
    std::vector<int32_t> p;
    explicit UF(size_t n) : p(n) { for (size_t i = 0; i < n; ++i) p[i] = (int32_t)i; }
    int32_t find(int32_t a) {
        while (p[a] != a) { p[a] = p[p[a]]; a = p[a]; }
        return a;
    }
    void unite(int32_t a, int32_t b) {
        a = find(a); b = find(b);
        if (a == b) return;
        if (a < b) p[b] = a; else p[a] = b;
    }
};

// Neighbour offsets: 8-connectivity = the D2Q9 lattice directions (Sec. 3.1,
// "moving along the directions of the Lattice Boltzmann model"); 4 optional.
const int NB8[8][2] = {{1, 0}, {1, 1}, {0, 1}, {-1, 1}, {-1, 0}, {-1, -1}, {0, -1}, {1, -1}};
const int NB4[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};

// Sec. 3.2.1: colour = label of the nearest centre by squared Euclidean
// distance.  Reading: exact integer distance between Q.8 points with the
// periodic minimum image on periodic axes and the plain difference on open
// ones; ties go to the lowest label; no centre -> MAXLINK.  On a periodic
// axis the query point is first brought into [0, 256 L); then every
// difference to a centre lies in (-256 L, 256 L) and one conditional shift
// gives the same minimum image as wrap_signed.
int32_t nearest_centre(int64_t X, int64_t Y, int K, const int32_t* qx, const int32_t* qy,
                       int lx, int ly, int open) {
    const int64_t MX = 256LL * lx, MY = 256LL * ly, hx = MX / 2, hy = MY / 2;
    const bool ox = open & 1, oy = open & 2;
    if (!ox) X = pos_mod(X, MX);
    if (!oy) Y = pos_mod(Y, MY);
    int32_t best = MAXLINK;
    int64_t bd = INT64_MAX;
    for (int i = 0; i < K; ++i) {
        int64_t dx = X - qx[i], dy = Y - qy[i];
        if (!ox) { if (dx >= MX - hx) dx -= MX; else if (dx < -hx) dx += MX; }
        if (!oy) { if (dy >= MY - hy) dy -= MY; else if (dy < -hy) dy += MY; }
        const int64_t d = dx * dx + dy * dy;
        if (d < bd) { bd = d; best = i; }
    }
    return best;
}

// Site (x, y) moved by (dx, dy): false when it leaves the domain across an
// open axis; otherwise (xx, yy) is the site, wrapped on periodic axes.
bool step(int64_t x, int64_t y, int dx, int dy, int lx, int ly, int open, int64_t& xx, int64_t& yy) {
    xx = x + dx;
    yy = y + dy;
    if (open & 1) { if (xx < 0 || xx >= lx) return false; } else xx = pos_mod(xx, lx);
    if (open & 2) { if (yy < 0 || yy >= ly) return false; } else yy = pos_mod(yy, ly);
    return true;
}

// Offset between two coordinates of one axis: minimum image when periodic.
int64_t axis_off(int64_t v, int64_t L, bool is_open) { return is_open ? v : wrap_signed(v, L); }

// Frame of site k (Sec. 3.2.2).  The naming figure is missing; reading from
// the mnemonics: s = "site", p/m = plus/minus along x/y.  Cyclic order:
// spx, spxpy, spy, spymx, smx, smxmy, smy, smypx.
const int FRAME[8][2] = {{1, 0}, {1, 1}, {0, 1}, {-1, 1}, {-1, 0}, {-1, -1}, {0, -1}, {1, -1}};
// Inner frame a_k, b_k, c_k, d_k.  Reading: the half-integer points between k
// and its diagonal neighbours spxpy, spymx, smxmy, smypx, in Q.8 offsets.
const int INNER[4][2] = {{128, 128}, {-128, 128}, {-128, -128}, {128, -128}};

// Rules of Sec. 3.2.2 applied at site (x, y) with colours f[0..7] of its frame
// and colour ck of the site itself.  mid(r) returns the colour of inner-frame
// point r (evaluated only when the other conditions hold).  Emits undirected
// couples {min, max} into out.
template <class Mid>
void site_rules(int32_t ck, const int32_t f[8], Mid mid, std::set<std::pair<int32_t, int32_t>>& out) {
    if (ck == MAXLINK) return;
    // gaps: consecutive frame points of different colour, obstacles not counted
    int gaps = 0;
    for (int i = 0; i < 8; ++i) {
        const int32_t a = f[i], b = f[(i + 1) & 7];
        if (a != b && a != MAXLINK && b != MAXLINK) ++gaps;
    }
    if (gaps < 3) return;  // bulk (0) or cell boundary (2): not a vertex
    for (int r = 0; r < 4; ++r) {
        // first nearest neighbour, written in the paper for spx, rotated by
        // r quarter turns (index +2 per turn): target f[2r]; long-diagonal
        // check between f[2r+2] and f[2r+7]
        const int32_t t = f[2 * r];
        const int32_t pa = f[(2 * r + 2) & 7], pb = f[(2 * r + 7) & 7];
        if (t != MAXLINK && pa != pb && t != ck)
            out.insert({std::min(ck, t), std::max(ck, t)});
        // second nearest neighbour, written for spxpy, rotated likewise:
        // target f[2r+1]; long diagonal f[2r+2] vs f[2r+7]; short diagonal
        // f[2r+2] vs f[2r]; inner-frame point r decides.
        const int32_t d = f[2 * r + 1];
        const int32_t side0 = f[2 * r];
        if (d != MAXLINK && d != ck && pa != pb && pa != side0) {
            const int32_t m = mid(r);
            if (m == d || m == ck)
                out.insert({std::min(ck, d), std::max(ck, d)});
        }
    }
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
// Sec. 3.1 -- cluster labelling.  Connected sets of inside sites (periodic
// axes wrap, open axes do not; obstacle sites are never inside).
// Reading: labels 0..K-1 are given in increasing order of each component's
// smallest linear index y*lx + x; outside sites get -1.  Sequential
// union-find over the sites in raster order.
// Returns K.
// ---------------------------------------------------------------------------
int32_t or_label(const float* field, int32_t lx, int32_t ly, float thr, int32_t phase,
                 int32_t conn, const uint8_t* obst, int32_t open, int32_t* labels) {
    const int64_t N = (int64_t)lx * ly;
    std::vector<uint8_t> in(N);
    for (int64_t s = 0; s < N; ++s)
        in[s] = (inside(field[s], thr, phase) && !(obst && obst[s])) ? 1 : 0;
    UF uf((size_t)N);
    const int (*nb)[2] = conn == 4 ? NB4 : NB8;
    const int nn = conn == 4 ? 4 : 8;
    for (int32_t y = 0; y < ly; ++y)
        for (int32_t x = 0; x < lx; ++x) {
            const int64_t s = (int64_t)y * lx + x;
            if (!in[s]) continue;
            for (int k = 0; k < nn; ++k) {
                int64_t xx, yy;
                if (!step(x, y, nb[k][0], nb[k][1], lx, ly, open, xx, yy)) continue;
                const int64_t t = yy * lx + xx;
                if (in[t]) uf.unite((int32_t)s, (int32_t)t);
            }
        }
    std::vector<int32_t> lab(N, -1);
    int32_t K = 0;
    for (int64_t s = 0; s < N; ++s) {
        if (!in[s]) { labels[s] = -1; continue; }
        const int32_t r = uf.find((int32_t)s);
        if (lab[r] < 0) lab[r] = K++;  // first visit in raster order = smallest index
        labels[s] = lab[r];
    }
    return K;
}

// ---------------------------------------------------------------------------
// Sec. 3.1 -- sizes and centres of mass: "sum the coordinates of the points
// of the bubble and divide by its size" (unweighted; the density-weighted
// definition of Sec. 2 is not what the procedure computes).
// Reading for the torus: offsets are taken relative to the component's
// smallest-index site r with the signed minimum image (plain differences on
// an open axis, where the mod below changes nothing), so
//   S = sum_s wrap(s - r),  centre = r + S/n  (mod L).
// Q.8 (units of 1/256 site) = 256 r + round_half_up(256 S / n), i.e.
//   256 r + floor((512 S + n) / (2 n))  mod 256 L,   exact integers.
// The float64 centre is r + (double)S/(double)n, wrapped once into [0, L).
// A component is "ambiguous" when two adjacent member sites get unwrapped
// coordinates more than one site apart (it crosses its own antipodal line);
// only a periodic axis can do that.
// Outputs (length K): n, root (linear index), qx, qy, fx, fy, amb (0/1).
// ---------------------------------------------------------------------------
void or_centroids(const int32_t* labels, int32_t lx, int32_t ly, int32_t conn, int32_t open, int32_t K,
                  int32_t* n_out, int32_t* root_out, int32_t* qx, int32_t* qy,
                  double* fx, double* fy, int32_t* amb) {
    const int64_t N = (int64_t)lx * ly;
    std::vector<int64_t> rootv(K, -1), n(K, 0), sx(K, 0), sy(K, 0);
    std::vector<int32_t> a(K, 0);
    for (int64_t s = 0; s < N; ++s) {
        const int32_t l = labels[s];
        if (l >= 0 && rootv[l] < 0) rootv[l] = s;
    }
    const int (*nb)[2] = conn == 4 ? NB4 : NB8;
    const int nn = conn == 4 ? 4 : 8;
    for (int32_t y = 0; y < ly; ++y)
        for (int32_t x = 0; x < lx; ++x) {
            const int32_t l = labels[(int64_t)y * lx + x];
            if (l < 0) continue;
            const int64_t rx = rootv[l] % lx, ry = rootv[l] / lx;
            const bool ox = open & 1, oy = open & 2;
            const int64_t ux = rx + axis_off(x - rx, lx, ox), uy = ry + axis_off(y - ry, ly, oy);
            n[l] += 1;
            sx[l] += ux - rx;
            sy[l] += uy - ry;
            for (int k = 0; k < nn; ++k) {
                int64_t xx, yy;
                if (!step(x, y, nb[k][0], nb[k][1], lx, ly, open, xx, yy)) continue;
                if (labels[yy * lx + xx] != l) continue;
                const int64_t vx = rx + axis_off(xx - rx, lx, ox), vy = ry + axis_off(yy - ry, ly, oy);
                if (vx - ux > 1 || ux - vx > 1 || vy - uy > 1 || uy - vy > 1) a[l] = 1;
            }
        }
    for (int32_t l = 0; l < K; ++l) {
        const int64_t rx = rootv[l] % lx, ry = rootv[l] / lx;
        n_out[l] = (int32_t)n[l];
        root_out[l] = (int32_t)rootv[l];
        qx[l] = (int32_t)pos_mod(256 * rx + floor_div(512 * sx[l] + n[l], 2 * n[l]), 256LL * lx);
        qy[l] = (int32_t)pos_mod(256 * ry + floor_div(512 * sy[l] + n[l], 2 * n[l]), 256LL * ly);
        double cx = (double)rx + (double)sx[l] / (double)n[l];
        double cy = (double)ry + (double)sy[l] / (double)n[l];
        if (cx < 0) cx += lx; else if (cx >= lx) cx -= lx;
        if (cy < 0) cy += ly; else if (cy >= ly) cy -= ly;
        fx[l] = cx;
        fy[l] = cy;
        amb[l] = a[l];
    }
}

// ---------------------------------------------------------------------------
// Sec. 2 (centroid equation with a density) -- the weighted variant of the
// centres: the centroid of a component with the field as its density,
// z = sum(w_s * y_s) / sum(w_s) over the member sites, y_s the member's
// position unwrapped as above (minimum image from the root on a periodic
// axis).  Reading: the density of a site is the field value rho_s quantised
// to 1/256, w_s = floor(256 rho_s + 1/2), computed in float64 from the
// float32 value, and clamped to [1, 65535] so that every site weighs
// something and every sum stays exact in 64-bit integers.  The Q.8 centre
// rounds 256 * sum(w dx) / sum(w) half up, as the unweighted one does with
// n; the float64 centre is root + (double)sum(w dx) / (double)sum(w).  With
// all weights equal this is the unweighted centre.  Sizes stay member counts.
// ---------------------------------------------------------------------------
int32_t quantised_weight(float rho) {
    const double v = std::floor(256.0 * (double)rho + 0.5);
    if (!(v >= 1.0)) return 1;      // (NaN cannot be inside)
    if (v > 65535.0) return 65535;
    return (int32_t)v;
}

int64_t round_half_up_q8(int64_t S, int64_t W) {
    // floor(256 S / W + 1/2) = floor((512 S + W) / (2 W)), in 128-bit integers
    const __int128 num = (__int128)512 * S + W, den = (__int128)2 * W;
    __int128 q = num / den;
    if ((num % den) != 0 && num < 0) q -= 1;
    return (int64_t)q;
}

void or_centroids_weighted(const int32_t* labels, const float* field, int32_t lx, int32_t ly,
                           int32_t open, int32_t K, int32_t* root_out, int32_t* qx, int32_t* qy,
                           double* fx, double* fy, int64_t* wsum) {
    const int64_t N = (int64_t)lx * ly;
    std::vector<int64_t> rootv(K, -1), W(K, 0), sx(K, 0), sy(K, 0);
    for (int64_t s = 0; s < N; ++s) {
        const int32_t l = labels[s];
        if (l >= 0 && rootv[l] < 0) rootv[l] = s;
    }
    const bool ox = open & 1, oy = open & 2;
    for (int32_t y = 0; y < ly; ++y)
        for (int32_t x = 0; x < lx; ++x) {
            const int64_t s = (int64_t)y * lx + x;
            const int32_t l = labels[s];
            if (l < 0) continue;
            const int64_t rx = rootv[l] % lx, ry = rootv[l] / lx;
            const int64_t w = quantised_weight(field[s]);
            W[l] += w;
            sx[l] += w * axis_off(x - rx, lx, ox);
            sy[l] += w * axis_off(y - ry, ly, oy);
        }
    for (int32_t l = 0; l < K; ++l) {
        const int64_t rx = rootv[l] % lx, ry = rootv[l] / lx;
        root_out[l] = (int32_t)rootv[l];
        qx[l] = (int32_t)pos_mod(256 * rx + round_half_up_q8(sx[l], W[l]), 256LL * lx);
        qy[l] = (int32_t)pos_mod(256 * ry + round_half_up_q8(sy[l], W[l]), 256LL * ly);
        double cx = (double)rx + (double)sx[l] / (double)W[l];
        double cy = (double)ry + (double)sy[l] / (double)W[l];
        if (cx < 0) cx += lx; else if (cx >= lx) cx -= lx;
        if (cy < 0) cy += ly; else if (cy >= ly) cy -= ly;
        fx[l] = cx;
        fy[l] = cy;
        wsum[l] = W[l];
    }
}

// ---------------------------------------------------------------------------
// Sec. 3.2.1 -- digital Voronoi colouring: one evaluation per site over all
// centres.  owner[y*lx + x] = nearest_centre(256x, 256y), MAXLINK on obstacles.
// ---------------------------------------------------------------------------
void or_owner(int32_t lx, int32_t ly, int32_t open, const uint8_t* obst, int32_t K,
              const int32_t* qx, const int32_t* qy, int32_t* owner, int32_t nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int32_t y = 0; y < ly; ++y)
        for (int32_t x = 0; x < lx; ++x)
            owner[(int64_t)y * lx + x] = (obst && obst[(int64_t)y * lx + x])
                                             ? MAXLINK
                                             : nearest_centre(256LL * x, 256LL * y, K, qx, qy, lx, ly, open);
    (void)nthreads;
}

// Colour of an arbitrary Q.8 point (used by tests for single sites / midpoints).
int32_t or_colour_at(int64_t X, int64_t Y, int32_t lx, int32_t ly, int32_t open, int32_t K,
                     const int32_t* qx, const int32_t* qy) {
    return nearest_centre(X, Y, K, qx, qy, lx, ly, open);
}

// ---------------------------------------------------------------------------
// Sec. 3.2.2 -- Delaunay couples from Voronoi-vertex sites, on a full colour
// map.  Inner-frame colours are evaluated on demand with the same nearest-
// centre rule; frame points beyond an open edge read as MAXLINK.  The
// compressed adjacency (sort + unique of the rows) is the
// ordered set of undirected couples (a < b).  Writes up to cap couples as
// (a, b) pairs into ab and returns the total count E.
// ---------------------------------------------------------------------------
int32_t or_edges(int32_t lx, int32_t ly, int32_t open, int32_t K, const int32_t* qx,
                 const int32_t* qy, const int32_t* owner, int32_t* ab, int32_t cap) {
    std::set<std::pair<int32_t, int32_t>> E;
    for (int32_t y = 0; y < ly; ++y)
        for (int32_t x = 0; x < lx; ++x) {
            int32_t f[8];
            for (int i = 0; i < 8; ++i) {
                int64_t xx, yy;
                f[i] = step(x, y, FRAME[i][0], FRAME[i][1], lx, ly, open, xx, yy) ? owner[yy * lx + xx]
                                                                                   : MAXLINK;
            }
            const int32_t ck = owner[(int64_t)y * lx + x];
            auto mid = [&](int r) {
                return nearest_centre(256LL * x + INNER[r][0], 256LL * y + INNER[r][1], K, qx, qy, lx, ly,
                                      open);
            };
            site_rules(ck, f, mid, E);
        }
    int32_t e = 0;
    for (const auto& p : E) {
        if (e < cap) { ab[2 * e] = p.first; ab[2 * e + 1] = p.second; }
        ++e;
    }
    return e;
}

// Same rules restricted to the sites of the window [x0, x0+w) x [y0, y0+h)
// (inside the domain), colouring the window and its one-site ring by brute
// force (ring sites beyond an open edge and obstacle sites are MAXLINK).
// Used to check large lattices one region at a time.
int32_t or_edges_window(int32_t lx, int32_t ly, int32_t open, const uint8_t* obst, int32_t K,
                        const int32_t* qx, const int32_t* qy, int32_t x0, int32_t y0, int32_t w,
                        int32_t h, int32_t* ab, int32_t cap, int32_t nthreads) {
    const int32_t W = w + 2, H = h + 2;
    std::vector<int32_t> c((size_t)W * H);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 2)
#endif
    for (int32_t j = 0; j < H; ++j)
        for (int32_t i = 0; i < W; ++i) {
            int64_t x, y;
            int32_t col = MAXLINK;
            if (step(x0, y0, i - 1, j - 1, lx, ly, open, x, y) && !(obst && obst[y * lx + x]))
                col = nearest_centre(256 * x, 256 * y, K, qx, qy, lx, ly, open);
            c[(size_t)j * W + i] = col;
        }
    (void)nthreads;
    std::set<std::pair<int32_t, int32_t>> E;
    for (int32_t j = 1; j <= h; ++j)
        for (int32_t i = 1; i <= w; ++i) {
            int32_t f[8];
            for (int q = 0; q < 8; ++q) f[q] = c[(size_t)(j + FRAME[q][1]) * W + (i + FRAME[q][0])];
            const int32_t ck = c[(size_t)j * W + i];
            const int64_t x = pos_mod(x0 - 1 + i, lx), y = pos_mod(y0 - 1 + j, ly);
            auto mid = [&](int r) {
                return nearest_centre(256 * x + INNER[r][0], 256 * y + INNER[r][1], K, qx, qy, lx, ly, open);
            };
            site_rules(ck, f, mid, E);
        }
    int32_t e = 0;
    for (const auto& p : E) {
        if (e < cap) { ab[2 * e] = p.first; ab[2 * e + 1] = p.second; }
        ++e;
    }
    return e;
}

// ---------------------------------------------------------------------------
// Sec. 3.2.3 -- kinematic isomorphism: each past centre is matched to the
// nearest now centre ("comparing the two sets of centers of mass").
// Reading: exact Q.8 squared distance (minimum image on periodic axes), ties
// to the lowest now label, no distance cut-off.  cnt[n] = number of past
// labels mapped to n.  With KN == 0 every phi is -1.
// ---------------------------------------------------------------------------
void or_match(int32_t lx, int32_t ly, int32_t open, int32_t KP, const int32_t* pqx, const int32_t* pqy,
              int32_t KN, const int32_t* nqx, const int32_t* nqy, int32_t* phi, int32_t* cnt) {
    for (int32_t n = 0; n < KN; ++n) cnt[n] = 0;
    for (int32_t p = 0; p < KP; ++p) {
        if (KN == 0) { phi[p] = -1; continue; }
        const int32_t m = nearest_centre(pqx[p], pqy[p], KN, nqx, nqy, lx, ly, open);
        phi[p] = m;
        cnt[m] += 1;
    }
}

// ---------------------------------------------------------------------------
// Sec. 3.2.3 / 3.2.4 -- translation, exclusion and breaking / arising couples.
// A past point p is kept when Phi(p) has exactly one preimage (a bubble that
// disappeared makes Phi non-injective); a now point n is kept when it has
// exactly one preimage (an appearing bubble has none).  Reading: couples that
// touch an excluded point are dropped from both graphs before comparing.
//   E_P' = { canon(Phi p, Phi q) : (p,q) in E_P, p and q kept }
//   E_N' = { (n,m) in E_N : n and m kept }
//   breaking = E_P' \ E_N' (kind -1), arising = E_N' \ E_P' (kind +1)
// Flip record = (a, b, pa, pb, kind, flags) with a < b now labels and
// Phi(pa) = a, Phi(pb) = b.  Order: breaking then arising, each by (a, b).
// The paper's additional active-point filter is not applied (flags = 0).
// local_trigger[p] (length KP) = 1 when the translated row of kept p differs
// from the row of Phi(p) in E_N'.  Returns the number of flips F; writes
// min(F, cap) records of 6 int32.  counts[0..2] = excluded past, excluded now,
// global trigger.
// ---------------------------------------------------------------------------
int32_t or_diff(int32_t KP, int32_t EP, const int32_t* past_ab, const int32_t* phi,
                int32_t KN, int32_t EN, const int32_t* now_ab, const int32_t* cnt,
                int32_t* flips, int32_t cap, int32_t* local_trigger, int32_t* counts) {
    std::vector<int32_t> inv(KN, -1);
    std::vector<char> keepP(KP, 0), keepN(KN, 0);
    int32_t exP = 0, exN = 0;
    for (int32_t p = 0; p < KP; ++p) {
        keepP[p] = (phi[p] >= 0 && cnt[phi[p]] == 1) ? 1 : 0;
        if (keepP[p]) inv[phi[p]] = p; else ++exP;
    }
    for (int32_t n = 0; n < KN; ++n) {
        keepN[n] = cnt[n] == 1 ? 1 : 0;
        if (!keepN[n]) ++exN;
    }
    typedef std::pair<int32_t, int32_t> E2;
    std::set<E2> Pp, Nn;
    std::vector<std::set<int32_t>> rowP(KP), rowN(KN);
    for (int32_t e = 0; e < EP; ++e) {
        const int32_t p = past_ab[2 * e], q = past_ab[2 * e + 1];
        if (!keepP[p] || !keepP[q]) continue;
        const int32_t a = phi[p], b = phi[q];
        Pp.insert({std::min(a, b), std::max(a, b)});
        rowP[p].insert(b);
        rowP[q].insert(a);
    }
    for (int32_t e = 0; e < EN; ++e) {
        const int32_t n = now_ab[2 * e], m = now_ab[2 * e + 1];
        if (!keepN[n] || !keepN[m]) continue;
        Nn.insert({n, m});
        rowN[n].insert(m);
        rowN[m].insert(n);
    }
    std::vector<E2> brk, ari;
    std::set_difference(Pp.begin(), Pp.end(), Nn.begin(), Nn.end(), std::back_inserter(brk));
    std::set_difference(Nn.begin(), Nn.end(), Pp.begin(), Pp.end(), std::back_inserter(ari));
    int32_t F = 0;
    auto emit = [&](const E2& e, int32_t kind) {
        if (F < cap) {
            int32_t* r = flips + 6 * F;
            r[0] = e.first; r[1] = e.second;
            r[2] = inv[e.first]; r[3] = inv[e.second];
            r[4] = kind; r[5] = 0;
        }
        ++F;
    };
    for (const auto& e : brk) emit(e, -1);
    for (const auto& e : ari) emit(e, +1);
    int32_t g = 0;
    for (int32_t p = 0; p < KP; ++p) {
        int32_t t = 0;
        if (keepP[p]) t = rowP[p] != rowN[phi[p]] ? 1 : 0;
        if (local_trigger) local_trigger[p] = t;
        g |= t;
    }
    counts[0] = exP;
    counts[1] = exN;
    counts[2] = g;
    return F;
}

}  // extern "C"
