// CPU oracle for 3D power (weighted Voronoi) cells -- TEST INFRASTRUCTURE ONLY.
//
// Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
// load this library.  It shares no code with the GPU path and is deliberately
// plain: FP64 arithmetic, brute-force candidate enumeration, O(V^2) clipping.
//
// What it computes (paper, Sec. 3, Eq. 1): for site p_i with weight w_i,
//     C_i = B  intersected with  { x : |x-p_i|^2 - w_i <= |x-p_j|^2 - w_j  for all j != i }
// where B is the clip box.  Written in the frame centred on p_i, every
// constraint is the half-space  a_ij . y <= b_ij  with  a_ij = p_j - p_i  and
// b_ij = (|a_ij|^2 + w_i - w_j) / 2;  b_ij / |a_ij| is the signed distance of
// the bisecting (radical) plane from p_i (paper, Sec. 4.2, Eq. 2).
//
// Candidate enumeration: all j != i are sorted by that plane distance d_ij and
// clipped in increasing order; once d_ij exceeds the largest vertex distance R
// of the current cell no remaining plane can reach the cell, because every
// point of the cell lies within R of p_i (this is the isotropic security
// radius of Levy and Bonneel, which the paper cites as prior art in Sec. 4.2.1;
// the paper's own directional BVH walk is what the GPU path implements).
//
// Clipping (paper, Sec. 4.1 and supplementary Sec. B): vertices strictly on
// the positive side of a_h.y - b_h are removed, zero is kept; each new vertex
// lies on an edge joining a kept and a removed vertex and is the intersection
// of the new plane with the two planes that edge lies on.  Edges are found by
// brute force (two vertices of a simple polytope are joined by an edge iff
// they share two planes).  Vertex positions are always recomputed from their
// three planes (Cramer's rule), never interpolated.
//
// Readings of points the paper leaves open (each is listed in the design notes):
//   * initial cell = the clip box (supplementary Sec. B uses the AABB of the
//     point set; a caller-supplied box generalises it); box planes carry codes
//     -1..-6 = x_min, x_max, y_min, y_max, z_min, z_max;
//   * coincident sites (a_ij = 0): among sites sharing one position the one
//     with the largest weight keeps its cell (ties: lowest original index);
//     the others ("losers") have empty cells, and their planes are dropped
//     from every other cell -- they are implied by the winner's plane, which
//     is identical (equal weights) or strictly tighter (larger weight);
//   * a facet counts as a neighbour only if the plane carries >= 3 vertices
//     (positive area); touching planes (all s <= 0) never clip;
//   * an empty cell has no vertices, facets or neighbours, volume 0 and
//     centroid equal to its site.
//
// Per cell it also reports a robustness margin: the smallest distance from a
// final vertex to any non-incident plane, divided by an error scale of that
// vertex and plane (see margin_of_cell).  Cells whose margin is at least a
// threshold tau are "certified": their combinatorics cannot change under
// relative perturbations well below tau, so any correct implementation must
// reproduce them exactly.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

enum { OF_EMPTY = 1, OF_DEGENERATE = 2, OF_COINCIDENT = 4 };

struct Plane {
    double a[3];
    double b;
    int64_t code;  // original site index (>= 0) or box code -1..-6
    double sig;    // size of the terms b is formed from, in distance units
};

struct Vert {
    double y[3];   // position relative to the cell's site
    int p[3];      // local plane indices
};

struct Poly {
    std::vector<Plane> pl;
    std::vector<Vert> v;
    bool empty = false;
    bool degenerate = false;
};

inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
inline double norm3(const double* a) { return std::sqrt(dot3(a, a)); }

// Intersection point of three planes a.y = b (Cramer's rule).
bool solve3(const Plane& A, const Plane& B, const Plane& C, double* y) {
    double bc[3], ca[3], ab[3];
    cross3(B.a, C.a, bc);
    cross3(C.a, A.a, ca);
    cross3(A.a, B.a, ab);
    double det = dot3(A.a, bc);
    if (det == 0.0) return false;
    for (int k = 0; k < 3; ++k) y[k] = (A.b * bc[k] + B.b * ca[k] + C.b * ab[k]) / det;
    return true;
}

// Sites in FP64 (FP32 inputs are widened exactly; an FP64 entry point lets
// finite differences perturb them below FP32 resolution).
struct Input {
    const double* xyz;
    const double* w;  // may be null (Voronoi)
    int64_t n;
    double box[6];   // lo.xyz, hi.xyz
    std::vector<char> loser;  // coincident site whose cell is empty
};

inline double site_w(const Input& in, int64_t j) { return in.w ? (double)in.w[j] : 0.0; }

// The clip box as six half-spaces in the frame of site p, and its 8 corners.
void init_box(Poly& P, const double* p, const double* box) {
    P.pl.clear();
    P.v.clear();
    P.empty = false;
    P.degenerate = false;
    for (int ax = 0; ax < 3; ++ax) {
        Plane lo{}, hi{};
        lo.a[ax] = -1.0;
        lo.b = p[ax] - box[ax];
        lo.code = -(2 * ax + 1);
        lo.sig = std::fabs(lo.b);
        hi.a[ax] = 1.0;
        hi.b = box[3 + ax] - p[ax];
        hi.code = -(2 * ax + 2);
        hi.sig = std::fabs(hi.b);
        P.pl.push_back(lo);
        P.pl.push_back(hi);
    }
    for (int c = 0; c < 8; ++c) {
        Vert v;
        for (int ax = 0; ax < 3; ++ax) {
            int side = (c >> ax) & 1;
            v.p[ax] = 2 * ax + side;
            v.y[ax] = (side ? box[3 + ax] : box[ax]) - p[ax];
        }
        P.v.push_back(v);
    }
}

int shared_planes(const Vert& u, const Vert& v, int* out) {
    int k = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (u.p[i] == v.p[j]) out[k++] = u.p[i];
    return k;
}

// Clip P by the half-space h.a . y <= h.b.  Returns true if the cell changed.
bool clip(Poly& P, const Plane& h) {
    if (P.empty) return false;
    const size_t nv = P.v.size();
    std::vector<double> s(nv);
    bool any_out = false, all_out = true;
    const double an = norm3(h.a);
    for (size_t k = 0; k < nv; ++k) {
        s[k] = dot3(h.a, P.v[k].y) - h.b;
        if (s[k] > 0) any_out = true; else all_out = false;
        // an exact or nearly exact zero marks a configuration that is not in
        // general position
        if (std::fabs(s[k]) <= 1e-12 * (an * norm3(P.v[k].y) + std::fabs(h.b))) P.degenerate = true;
    }
    if (!any_out) return false;
    if (all_out) {
        P.empty = true;
        P.v.clear();
        return true;
    }
    const int hidx = (int)P.pl.size();
    P.pl.push_back(h);
    std::vector<Vert> next;
    next.reserve(nv + 8);
    for (size_t k = 0; k < nv; ++k)
        if (s[k] <= 0) next.push_back(P.v[k]);
    for (size_t u = 0; u < nv; ++u) {
        if (s[u] > 0) continue;
        for (size_t r = 0; r < nv; ++r) {
            if (s[r] <= 0) continue;
            int sh[9];
            if (shared_planes(P.v[u], P.v[r], sh) != 2) continue;
            Vert nvx;
            nvx.p[0] = hidx;
            nvx.p[1] = sh[0];
            nvx.p[2] = sh[1];
            if (!solve3(P.pl[hidx], P.pl[sh[0]], P.pl[sh[1]], nvx.y)) {
                P.degenerate = true;
                continue;
            }
            if (s[u] == 0) P.degenerate = true;  // new vertex coincides with a kept one
            next.push_back(nvx);
        }
    }
    P.v.swap(next);
    return true;
}

struct Cand {
    double d;     // signed distance of the bisecting plane from the site
    int64_t j;
};

// Plane of candidate j in the frame of site i.
Plane make_plane(const Input& in, int64_t i, int64_t j) {
    Plane h;
    double d2 = 0;
    for (int k = 0; k < 3; ++k) {
        h.a[k] = (double)in.xyz[3 * j + k] - (double)in.xyz[3 * i + k];
        d2 += h.a[k] * h.a[k];
    }
    h.b = 0.5 * (d2 + (site_w(in, i) - site_w(in, j)));
    h.code = j;
    h.sig = (d2 + std::fabs(site_w(in, i) - site_w(in, j))) / (2.0 * std::sqrt(d2));
    return h;
}

struct CellOut {
    int flags = 0;
    double margin = 0;
    double vol = 0;
    double cen[3] = {0, 0, 0};
    std::vector<int64_t> nbr;
    std::vector<double> vpos;     // 3 per vertex, global coordinates
    std::vector<int64_t> vcode;   // 3 per vertex, ascending
    std::vector<int64_t> fcode;   // per facet, ascending
    std::vector<int64_t> fsize;   // vertices per facet
    std::vector<int64_t> fv;      // cell-local vertex indices, CCW seen from outside
};

// Enumerate candidates for site i in increasing plane distance and clip until
// no further plane can reach the cell.  Returns the number of candidates
// examined (those with d <= reach are left at the front of `cand`).
struct Builder {
    const Input& in;
    std::vector<Cand> cand;
    size_t sorted_upto = 0;

    explicit Builder(const Input& input) : in(input) {}

    // Fill `cand` with all j != i except coincident losers.  Returns false
    // if site i itself is a coincident loser (empty cell).
    bool gather(int64_t i, bool& coincident) {
        cand.clear();
        sorted_upto = 0;
        coincident = false;
        const double wi = site_w(in, i);
        const double px = in.xyz[3 * i], py = in.xyz[3 * i + 1], pz = in.xyz[3 * i + 2];
        for (int64_t j = 0; j < in.n; ++j) {
            if (j == i) continue;
            double ax = (double)in.xyz[3 * j] - px, ay = (double)in.xyz[3 * j + 1] - py,
                   az = (double)in.xyz[3 * j + 2] - pz;
            double d2 = ax * ax + ay * ay + az * az;
            if (d2 == 0.0) coincident = true;
            if (in.loser[j] || d2 == 0.0) continue;
            double D = std::sqrt(d2);
            cand.push_back({(d2 + (wi - site_w(in, j))) / (2.0 * D), j});
        }
        return !in.loser[i];
    }

    // Make sure cand[0 .. k) is sorted and holds the k smallest distances.
    void ensure_sorted(size_t k) {
        if (k <= sorted_upto) return;
        size_t want = std::max(k, std::max<size_t>(2 * sorted_upto, 64));
        want = std::min(want, cand.size());
        auto less = [](const Cand& x, const Cand& y) { return x.d < y.d || (x.d == y.d && x.j < y.j); };
        std::partial_sort(cand.begin() + sorted_upto, cand.begin() + want, cand.end(), less);
        sorted_upto = want;
    }
};

double max_radius(const Poly& P) {
    double r2 = 0;
    for (const Vert& v : P.v) r2 = std::max(r2, dot3(v.y, v.y));
    return std::sqrt(r2);
}

// Build the polytope of site i (clipping only, no outputs).  Returns the
// number of sorted candidates that were examined.
size_t build_poly(const Input& in, Builder& B, int64_t i, double wshift, Poly& P, int& flags) {
    double p[3] = {(double)in.xyz[3 * i], (double)in.xyz[3 * i + 1], (double)in.xyz[3 * i + 2]};
    init_box(P, p, in.box);
    bool coincident = false;
    bool alive = B.gather(i, coincident);
    if (coincident) flags |= OF_COINCIDENT;
    if (!alive) {
        P.empty = true;
        P.v.clear();
        return 0;
    }
    size_t t = 0;
    double R = max_radius(P);
    for (;; ++t) {
        B.ensure_sorted(t + 1);
        if (t >= B.cand.size()) break;
        // a weight raised by wshift >= 0 only moves planes outward (by
        // wshift / (2 D)), so the unshifted order still bounds the rest
        if (B.cand[t].d > R) break;
        Plane h = make_plane(in, i, B.cand[t].j);
        h.b += 0.5 * wshift;
        if (clip(P, h)) {
            if (P.empty) break;
            R = max_radius(P);
        }
    }
    return t;
}

// Error scale of a vertex: |inverse of the matrix of unit normals| times the
// size of the quantities it is solved from.
double vertex_error_scale(const Poly& P, const Vert& v) {
    double m[3][3], dist = 0;
    for (int r = 0; r < 3; ++r) {
        const Plane& pl = P.pl[v.p[r]];
        double an = norm3(pl.a);
        for (int c = 0; c < 3; ++c) m[r][c] = pl.a[c] / an;
        dist = std::max(dist, pl.sig);
    }
    double c0[3], c1[3], c2[3];
    cross3(m[1], m[2], c0);
    cross3(m[2], m[0], c1);
    cross3(m[0], m[1], c2);
    double det = std::fabs(dot3(m[0], c0));
    if (det == 0) return INFINITY;
    double fro = std::sqrt(dot3(c0, c0) + dot3(c1, c1) + dot3(c2, c2)) / det;
    return fro * (dist + norm3(v.y));
}

// Robustness margin of a non-empty cell (see the header comment): the least
// distance from a final vertex v to a non-incident plane k, divided by
// sigma(v,k) = e_v + |v| + sig_k.  A candidate whose plane distance d_k
// satisfies d_k - R >= tau_m * (e_max + R + sig_k) cannot go below tau_m
// (every vertex is within R of the site) and is skipped cheaply.
double margin_of_cell(const Input& in, Builder& B, int64_t i, const Poly& P) {
    const double tau_m = 1e-3;
    std::vector<double> ev(P.v.size());
    double emax = 0, R = 0;
    for (size_t k = 0; k < P.v.size(); ++k) {
        ev[k] = vertex_error_scale(P, P.v[k]);
        emax = std::max(emax, ev[k]);
        R = std::max(R, norm3(P.v[k].y));
    }
    if (!std::isfinite(emax)) return 0.0;
    double margin = tau_m;
    auto visit = [&](const Plane& h) {
        double an = norm3(h.a);
        double dk = h.sig;
        for (size_t k = 0; k < P.v.size(); ++k) {
            const Vert& v = P.v[k];
            bool incident = false;
            for (int r = 0; r < 3; ++r)
                if (P.pl[v.p[r]].code == h.code) incident = true;
            if (incident) continue;
            double dist = (h.b - dot3(h.a, v.y)) / an;
            double sigma = ev[k] + norm3(v.y) + dk;
            margin = std::min(margin, dist / sigma);
        }
    };
    double p[3] = {(double)in.xyz[3 * i], (double)in.xyz[3 * i + 1], (double)in.xyz[3 * i + 2]};
    Poly boxp;
    init_box(boxp, p, in.box);
    for (const Plane& h : boxp.pl) visit(h);
    for (const Cand& c : B.cand) {
        if (c.d - R > tau_m * (emax + R)) {
            Plane h = make_plane(in, i, c.j);
            if (c.d - R >= tau_m * (emax + R + h.sig)) continue;
            visit(h);
        } else {
            visit(make_plane(in, i, c.j));
        }
    }
    return std::max(margin, 0.0);
}

void finalize(const Input& in, int64_t i, const Poly& P, CellOut& out) {
    double p[3] = {(double)in.xyz[3 * i], (double)in.xyz[3 * i + 1], (double)in.xyz[3 * i + 2]};
    if (P.empty || P.v.empty()) {
        out.flags |= OF_EMPTY;
        out.vol = 0;
        for (int k = 0; k < 3; ++k) out.cen[k] = p[k];
        return;
    }
    const size_t nv = P.v.size();
    // canonical vertex order: by ascending code triple
    std::vector<std::array<int64_t, 3>> key(nv);
    for (size_t k = 0; k < nv; ++k) {
        for (int r = 0; r < 3; ++r) key[k][r] = P.pl[P.v[k].p[r]].code;
        std::sort(key[k].begin(), key[k].end());
    }
    std::vector<size_t> order(nv);
    for (size_t k = 0; k < nv; ++k) order[k] = k;
    std::sort(order.begin(), order.end(), [&](size_t x, size_t y) { return key[x] < key[y]; });
    std::vector<size_t> rank(nv);
    for (size_t k = 0; k < nv; ++k) rank[order[k]] = k;
    for (size_t k = 0; k < nv; ++k) {
        const Vert& v = P.v[order[k]];
        for (int r = 0; r < 3; ++r) {
            out.vpos.push_back(p[r] + v.y[r]);
            out.vcode.push_back(key[order[k]][r]);
        }
    }
    // live planes, ascending code
    std::vector<int> live;
    for (size_t q = 0; q < P.pl.size(); ++q) {
        bool used = false;
        for (const Vert& v : P.v)
            if (v.p[0] == (int)q || v.p[1] == (int)q || v.p[2] == (int)q) used = true;
        if (used) live.push_back((int)q);
    }
    std::sort(live.begin(), live.end(), [&](int x, int y) { return P.pl[x].code < P.pl[y].code; });
    // reference point for the tetrahedral fan: first canonical vertex
    const double* ref = P.v[order[0]].y;
    double vol6 = 0, mom[3] = {0, 0, 0}, vol_facets = 0;
    for (int q : live) {
        const Plane& pl = P.pl[q];
        std::vector<size_t> ring;
        for (size_t k = 0; k < nv; ++k) {
            const Vert& v = P.v[k];
            if (v.p[0] == q || v.p[1] == q || v.p[2] == q) ring.push_back(k);
        }
        if (ring.size() < 3) {
            // a plane touching the cell in an edge or a point is no facet
            out.flags |= OF_DEGENERATE;
            continue;
        }
        // order the facet's vertices counter-clockwise seen from outside
        // (looking against the outward normal a)
        double c[3] = {0, 0, 0};
        for (size_t k : ring)
            for (int r = 0; r < 3; ++r) c[r] += P.v[k].y[r] / ring.size();
        double an = norm3(pl.a), nrm[3] = {pl.a[0] / an, pl.a[1] / an, pl.a[2] / an};
        double e1[3], e2[3];
        {
            double t[3];
            // any direction not parallel to the normal
            double ax[3] = {0, 0, 0};
            int m = 0;
            for (int r = 1; r < 3; ++r)
                if (std::fabs(nrm[r]) < std::fabs(nrm[m])) m = r;
            ax[m] = 1;
            cross3(nrm, ax, t);
            double tn = norm3(t);
            for (int r = 0; r < 3; ++r) e1[r] = t[r] / tn;
            cross3(nrm, e1, e2);
        }
        std::vector<std::pair<double, size_t>> ang;
        for (size_t k : ring) {
            double d[3] = {P.v[k].y[0] - c[0], P.v[k].y[1] - c[1], P.v[k].y[2] - c[2]};
            ang.push_back({std::atan2(dot3(d, e2), dot3(d, e1)), k});
        }
        std::sort(ang.begin(), ang.end());
        // rotate to start at the smallest canonical index
        size_t start = 0;
        for (size_t t = 1; t < ang.size(); ++t)
            if (rank[ang[t].second] < rank[ang[start].second]) start = t;
        out.fcode.push_back(pl.code);
        out.fsize.push_back((int64_t)ang.size());
        for (size_t t = 0; t < ang.size(); ++t) out.fv.push_back((int64_t)rank[ang[(start + t) % ang.size()].second]);
        if (pl.code >= 0) out.nbr.push_back(pl.code);
        // facet area and the facet form of the volume, V = sum_f h_f A_f / 3
        double area2 = 0;
        for (size_t t = 0; t < ang.size(); ++t) {
            const double* u = P.v[ang[t].second].y;
            const double* w = P.v[ang[(t + 1) % ang.size()].second].y;
            double du[3] = {u[0] - c[0], u[1] - c[1], u[2] - c[2]};
            double dw[3] = {w[0] - c[0], w[1] - c[1], w[2] - c[2]};
            double cr[3];
            cross3(du, dw, cr);
            area2 += dot3(cr, nrm);
        }
        double h = (pl.b - dot3(pl.a, ref)) / an;
        vol_facets += h * 0.5 * area2 / 3.0;
        // tetrahedra (ref, f0, f_t, f_t+1) for the centroid
        const double* f0 = P.v[ang[0].second].y;
        for (size_t t = 1; t + 1 < ang.size(); ++t) {
            const double* f1 = P.v[ang[t].second].y;
            const double* f2 = P.v[ang[t + 1].second].y;
            double a0[3], a1[3], a2[3], cr[3];
            for (int r = 0; r < 3; ++r) {
                a0[r] = f0[r] - ref[r];
                a1[r] = f1[r] - ref[r];
                a2[r] = f2[r] - ref[r];
            }
            cross3(a1, a2, cr);
            double det = dot3(a0, cr);
            vol6 += det;
            for (int r = 0; r < 3; ++r) mom[r] += det * (a0[r] + a1[r] + a2[r]) / 4.0;
        }
    }
    (void)vol_facets;
    out.vol = vol6 / 6.0;
    for (int r = 0; r < 3; ++r) out.cen[r] = p[r] + ref[r] + (vol6 != 0 ? mom[r] / vol6 : 0.0);
}

struct Result {
    std::vector<CellOut> cells;
};

double nearest_distance(const Input& in, const Builder& B, int64_t i) {
    // smallest Euclidean distance to another (non-coincident) site
    double best = INFINITY;
    for (const Cand& c : B.cand) {
        Plane h = make_plane(in, i, c.j);
        best = std::min(best, norm3(h.a));
    }
    return best;
}

}  // namespace

extern "C" {

static void* run_impl(const double* xyz, const double* w, int64_t n, const double* box, const int64_t* cells, int64_t m,
                     int want_margin, int nthreads);

// Compute cells `cells[0..m)` (all n cells if cells == NULL).  `box` is
// [lo.xyz, hi.xyz] in FP64.  Returns an opaque handle, or NULL on bad input.
// `want_margin` = 0 skips the robustness margin (faster).
void* orc_run(const float* xyz, const float* w, int64_t n, const double* box, const int64_t* cells, int64_t m,
              int want_margin, int nthreads) {
    if (n <= 0 || !xyz || !box) return nullptr;
    std::vector<double> x((size_t)(3 * n)), ww;
    for (int64_t k = 0; k < 3 * n; ++k) x[(size_t)k] = (double)xyz[k];
    if (w) {
        ww.resize((size_t)n);
        for (int64_t k = 0; k < n; ++k) ww[(size_t)k] = (double)w[k];
    }
    return run_impl(x.data(), w ? ww.data() : nullptr, n, box, cells, m, want_margin, nthreads);
}

// The same with FP64 sites and weights.
void* orc_run64(const double* xyz, const double* w, int64_t n, const double* box, const int64_t* cells, int64_t m,
                int want_margin, int nthreads) {
    if (n <= 0 || !xyz || !box) return nullptr;
    return run_impl(xyz, w, n, box, cells, m, want_margin, nthreads);
}

static void* run_impl(const double* xyz, const double* w, int64_t n, const double* box, const int64_t* cells, int64_t m,
                     int want_margin, int nthreads) {
    Input in{xyz, w, n, {box[0], box[1], box[2], box[3], box[4], box[5]}, {}};
    // coincident sites: sort by position, the heaviest of each run of equal
    // positions (lowest index among equals) is the only one that keeps a cell
    in.loser.assign((size_t)n, 0);
    {
        std::vector<int64_t> ord((size_t)n);
        for (int64_t k = 0; k < n; ++k) ord[(size_t)k] = k;
        auto pos_less = [&](int64_t x, int64_t y) {
            for (int c = 0; c < 3; ++c)
                if (xyz[3 * x + c] != xyz[3 * y + c]) return xyz[3 * x + c] < xyz[3 * y + c];
            return x < y;
        };
        std::sort(ord.begin(), ord.end(), pos_less);
        for (size_t a = 0; a < ord.size();) {
            size_t b = a + 1;
            while (b < ord.size() && xyz[3 * ord[b]] == xyz[3 * ord[a]] && xyz[3 * ord[b] + 1] == xyz[3 * ord[a] + 1] &&
                   xyz[3 * ord[b] + 2] == xyz[3 * ord[a] + 2])
                ++b;
            if (b - a > 1) {
                size_t win = a;
                for (size_t t = a + 1; t < b; ++t) {
                    double wt = w ? (double)w[ord[t]] : 0.0, ww = w ? (double)w[ord[win]] : 0.0;
                    if (wt > ww || (wt == ww && ord[t] < ord[win])) win = t;
                }
                for (size_t t = a; t < b; ++t)
                    if (t != win) in.loser[(size_t)ord[t]] = 1;
            }
            a = b;
        }
    }
    Result* res = new Result;
    const int64_t count = cells ? m : n;
    res->cells.resize((size_t)count);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        Builder B(in);
        Poly P;
#pragma omp for schedule(dynamic, 4)
        for (int64_t t = 0; t < count; ++t) {
            int64_t i = cells ? cells[t] : t;
            CellOut& out = res->cells[(size_t)t];
            int flags = 0;
            build_poly(in, B, i, 0.0, P, flags);
            out.flags = flags;
            if (P.degenerate) out.flags |= OF_DEGENERATE;
            finalize(in, i, P, out);
            if (want_margin) {
                if (out.flags & (OF_DEGENERATE | OF_COINCIDENT)) {
                    out.margin = 0;
                } else if (out.flags & OF_EMPTY) {
                    // robustly empty at level tau: still empty after raising
                    // w_i by tau (l^2 + |w_i|), l = nearest-site distance
                    double l = nearest_distance(in, B, i);
                    if (!std::isfinite(l)) l = 0;
                    out.margin = 0.0;
                    const double levels[4] = {1e-3, 1e-5, 1e-7, 1e-10};
                    for (double tau : levels) {
                        double shift = tau * (l * l + std::fabs(site_w(in, i)));
                        Poly Q;
                        int f2 = 0;
                        build_poly(in, B, i, shift, Q, f2);
                        if (Q.empty || Q.v.empty()) {
                            out.margin = tau;
                            break;
                        }
                    }
                } else {
                    out.margin = margin_of_cell(in, B, i, P);
                }
            }
        }
    }
    return res;
}

// Totals: [neighbours, vertices, facets, facet-vertices].
void orc_sizes(const void* h, int64_t* tot) {
    const Result* r = (const Result*)h;
    int64_t a = 0, b = 0, c = 0, d = 0;
    for (const CellOut& o : r->cells) {
        a += o.nbr.size();
        b += o.vcode.size() / 3;
        c += o.fcode.size();
        d += o.fv.size();
    }
    tot[0] = a;
    tot[1] = b;
    tot[2] = c;
    tot[3] = d;
}

// Copy results into caller arrays (sizes from orc_sizes; m = number of cells).
// Offsets are CSR (m+1 entries); fv holds cell-local vertex indices.
void orc_fetch(const void* h, int64_t* nbr_off, int64_t* nbr, int64_t* vert_off, double* vert, int64_t* vert_code,
               int64_t* facet_off, int64_t* facet_code, int64_t* fv_off, int64_t* fv, double* vol, double* cen,
               int32_t* flags, double* margin) {
    const Result* r = (const Result*)h;
    int64_t a = 0, b = 0, c = 0, d = 0;
    nbr_off[0] = vert_off[0] = facet_off[0] = fv_off[0] = 0;
    for (size_t t = 0; t < r->cells.size(); ++t) {
        const CellOut& o = r->cells[t];
        for (int64_t x : o.nbr) nbr[a++] = x;
        for (size_t k = 0; k < o.vcode.size(); ++k) {
            vert[3 * b + k] = o.vpos[k];
            vert_code[3 * b + k] = o.vcode[k];
        }
        b += o.vcode.size() / 3;
        for (size_t f = 0; f < o.fcode.size(); ++f) {
            facet_code[c] = o.fcode[f];
            fv_off[c + 1] = fv_off[c] + o.fsize[f];
            ++c;
        }
        for (int64_t x : o.fv) fv[d++] = x;
        nbr_off[t + 1] = a;
        vert_off[t + 1] = b;
        facet_off[t + 1] = c;
        vol[t] = o.vol;
        for (int k = 0; k < 3; ++k) cen[3 * t + k] = o.cen[k];
        flags[t] = o.flags;
        margin[t] = o.margin;
    }
}

void orc_free(void* h) { delete (Result*)h; }

}  // extern "C"
