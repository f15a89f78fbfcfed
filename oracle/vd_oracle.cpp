// CPU oracle for 3D power (weighted Voronoi) cells -- TEST INFRASTRUCTURE ONLY.
//
// Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
// load this library.  It shares no code with the GPU path and is deliberately
// plain: FP64 arithmetic, candidates in increasing plane distance (brute force
// or a k-d tree, same sequence), O(V^2) clipping.
//
// What it computes (paper, Sec. 3, Eq. 1): for site p_i with weight w_i,
//     C_i = B  intersected with  { x : |x-p_i|^2 - w_i <= |x-p_j|^2 - w_j  for all j != i }
// where B is the clip box.  Written in the frame centred on p_i, every
// constraint is the half-space  a_ij . y <= b_ij  with  a_ij = p_j - p_i  and
// b_ij = (|a_ij|^2 + w_i - w_j) / 2;  b_ij / |a_ij| is the signed distance of
// the bisecting (radical) plane from p_i (paper, Sec. 4.2, Eq. 2).
//
// Candidate enumeration: all j != i are taken in increasing plane distance
// d_ij (ties: lower index first) and clipped in that order; once d_ij exceeds
// the largest vertex distance R of the current cell no remaining plane can
// reach the cell, because every point of the cell lies within R of p_i (this
// is the isotropic security radius of Levy and Bonneel, which the paper cites
// as prior art in Sec. 4.2.1; the paper's own directional BVH walk is what the
// GPU path implements).  Two ways to produce that order: brute force (every
// site's d_ij, partially sorted), or a best-first walk of a median-split k-d
// tree whose nodes also hold the largest weight below them, keyed by the
// lower bound d_B/2 + min(0, w_i - w_max)/(2 d_B) of d_ij over a node at
// distance d_B (Sec. 4.2.2's bound with an isotropic radius).  The walk emits
// exactly the brute-force sequence (a node is expanded before any site whose
// d_ij is not below its key), so both modes give bit-identical results.
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
    std::vector<char> twin;   // some other site has the same position
    int64_t moved = -1;       // a site moved since the k-d tree was built (or -1)
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

// Median-split k-d tree over the sites (leaves of at most kKdLeaf sites);
// every node stores the bounding box and the largest weight of its sites.
constexpr int kKdLeaf = 8;
struct KdNode {
    double lo[3], hi[3];
    double wmax;
    int64_t begin, end;   // range of `perm`
    int64_t left, right;  // children (-1: leaf)
};
struct KdTree {
    std::vector<KdNode> nodes;
    std::vector<int64_t> perm;
};

// Builds the subtree over perm[b, e) and returns its node index.  Large
// ranges build their two halves as OpenMP tasks (the tree and the input are
// passed by pointer, which a task copies as a plain value).
int64_t kd_build_range(const Input* in, KdTree* T, int64_t b, int64_t e) {
    KdNode nd;
    for (int k = 0; k < 3; ++k) {
        nd.lo[k] = INFINITY;
        nd.hi[k] = -INFINITY;
    }
    nd.wmax = -INFINITY;
    for (int64_t q = b; q < e; ++q) {
        const int64_t j = T->perm[(size_t)q];
        for (int k = 0; k < 3; ++k) {
            nd.lo[k] = std::min(nd.lo[k], in->xyz[3 * j + k]);
            nd.hi[k] = std::max(nd.hi[k], in->xyz[3 * j + k]);
        }
        nd.wmax = std::max(nd.wmax, site_w(*in, j));
    }
    nd.begin = b;
    nd.end = e;
    nd.left = nd.right = -1;
    int64_t id;
#pragma omp critical(kd_nodes)
    {
        id = (int64_t)T->nodes.size();
        T->nodes.push_back(nd);
    }
    if (e - b <= kKdLeaf) return id;
    int ax = 0;
    for (int k = 1; k < 3; ++k)
        if (nd.hi[k] - nd.lo[k] > nd.hi[ax] - nd.lo[ax]) ax = k;
    const int64_t mid = b + (e - b) / 2;
    const double* xyz = in->xyz;
    std::nth_element(T->perm.begin() + b, T->perm.begin() + mid, T->perm.begin() + e,
                     [xyz, ax](int64_t x, int64_t y) { return xyz[3 * x + ax] < xyz[3 * y + ax]; });
    int64_t l = -1, r = -1;
    if (e - b > 65536) {
#pragma omp task shared(l) firstprivate(in, T, b, mid)
        l = kd_build_range(in, T, b, mid);
#pragma omp task shared(r) firstprivate(in, T, mid, e)
        r = kd_build_range(in, T, mid, e);
#pragma omp taskwait
    } else {
        l = kd_build_range(in, T, b, mid);
        r = kd_build_range(in, T, mid, e);
    }
#pragma omp critical(kd_nodes)
    {
        T->nodes[(size_t)id].left = l;
        T->nodes[(size_t)id].right = r;
    }
    return id;
}

void kd_build(const Input& in, KdTree& T) {
    T.perm.resize((size_t)in.n);
    for (int64_t j = 0; j < in.n; ++j) T.perm[(size_t)j] = j;
    T.nodes.reserve((size_t)(4 * in.n / kKdLeaf + 16));
    const Input* ip = &in;
    KdTree* tp = &T;
#pragma omp parallel
#pragma omp single
    kd_build_range(ip, tp, 0, in.n);
}

// Distance from p to a node's box.
double box_distance(const KdNode& nd, const double* p) {
    double d2 = 0;
    for (int k = 0; k < 3; ++k) {
        const double t = std::max(std::max(nd.lo[k] - p[k], p[k] - nd.hi[k]), 0.0);
        d2 += t * t;
    }
    return std::sqrt(d2);
}

// Lower bound, over the sites j of a node at distance dB from p_i, of
// (|a|^2 (1 - tau) + g(w_i - w_j)) / (2 |a|) with g(x) = x (1 - tau) for x >= 0
// and x (1 + tau) below; tau = 0 gives the plane distance d_ij.  The function
// of t = |a| >= dB is t (1 - tau)/2 + g/(2t), increasing when g < 0, and g is
// increasing in w_i - w_j >= w_i - w_max.  Rounded down by a relative margin
// far above FP64 rounding, so that the key never exceeds a computed d_ij.
double node_key(const KdNode& nd, const double* p, double wi, double tau) {
    const double dB = box_distance(nd, p);
    const double c = std::min(0.0, wi - nd.wmax) * (1.0 + tau);
    double lb;
    if (c < 0.0) lb = dB > 0.0 ? 0.5 * dB * (1.0 - tau) + c / (2.0 * dB) : -INFINITY;
    else lb = 0.5 * dB * (1.0 - tau);
    return lb - 1e-9 * std::fabs(lb);
}

// Candidates for site i in increasing plane distance (ties: lower index).
struct Builder {
    const Input& in;
    const KdTree* kd;  // null: brute force
    int64_t i = -1;
    double p[3] = {0, 0, 0}, wi = 0;
    // brute force: every candidate, sorted lazily
    std::vector<Cand> cand;
    size_t sorted_upto = 0, pos = 0;
    // k-d tree: heap of nodes (kind 0) and sites (kind 1)
    struct Entry {
        double key;
        int kind;
        int64_t id;
    };
    std::vector<Entry> heap;

    Builder(const Input& input, const KdTree* tree) : in(input), kd(tree) {}

    static bool after(const Entry& x, const Entry& y) {  // heap order: smallest (key, kind, id) on top
        if (x.key != y.key) return x.key > y.key;
        if (x.kind != y.kind) return x.kind > y.kind;
        return x.id > y.id;
    }

    // Plane distance of candidate j (the same expression in both modes).
    double dist_of(int64_t j, double* d2out) const {
        const double ax = in.xyz[3 * j] - p[0], ay = in.xyz[3 * j + 1] - p[1], az = in.xyz[3 * j + 2] - p[2];
        const double d2 = ax * ax + ay * ay + az * az;
        *d2out = d2;
        return (d2 + (wi - site_w(in, j))) / (2.0 * std::sqrt(d2));
    }

    // Start the enumeration for site i.  Returns false if site i is a
    // coincident loser (empty cell); `coincident` tells whether some other
    // site has the same position.
    bool start(int64_t site, bool& coincident) {
        i = site;
        for (int k = 0; k < 3; ++k) p[k] = in.xyz[3 * i + k];
        wi = site_w(in, i);
        coincident = in.twin[(size_t)i] != 0;
        cand.clear();
        heap.clear();
        sorted_upto = pos = 0;
        if (!kd) {
            for (int64_t j = 0; j < in.n; ++j) {
                if (j == i || in.loser[(size_t)j]) continue;
                double d2;
                const double d = dist_of(j, &d2);
                if (d2 == 0.0) continue;
                cand.push_back({d, j});
            }
        } else {
            heap.push_back({node_key(kd->nodes[0], p, wi, 0.0), 0, 0});
            // a moved site may lie outside the node boxes: it is a candidate of its own
            const int64_t mv = in.moved;
            if (mv >= 0 && mv != i && !in.loser[(size_t)mv]) {
                double d2;
                const double d = dist_of(mv, &d2);
                if (d2 != 0.0) heap.push_back({d, 1, mv});
                std::push_heap(heap.begin(), heap.end(), after);
            }
        }
        return !in.loser[(size_t)i];
    }

    // The next candidate; false when none is left.
    bool next(Cand& c) {
        if (!kd) {
            ensure_sorted(pos + 1);
            if (pos >= cand.size()) return false;
            c = cand[pos++];
            return true;
        }
        while (!heap.empty()) {
            std::pop_heap(heap.begin(), heap.end(), after);
            const Entry e = heap.back();
            heap.pop_back();
            if (e.kind == 1) {
                c = {e.key, e.id};
                return true;
            }
            const KdNode& nd = kd->nodes[(size_t)e.id];
            if (nd.left < 0) {
                for (int64_t q = nd.begin; q < nd.end; ++q) {
                    const int64_t j = kd->perm[(size_t)q];
                    if (j == i || in.loser[(size_t)j] || j == in.moved) continue;
                    double d2;
                    const double d = dist_of(j, &d2);
                    if (d2 == 0.0) continue;
                    heap.push_back({d, 1, j});
                    std::push_heap(heap.begin(), heap.end(), after);
                }
            } else {
                for (int64_t ch : {nd.left, nd.right}) {
                    heap.push_back({node_key(kd->nodes[(size_t)ch], p, wi, 0.0), 0, ch});
                    std::push_heap(heap.begin(), heap.end(), after);
                }
            }
        }
        return false;
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

    // Calls f(candidate) for every candidate j (all of them in brute force);
    // with the k-d tree at least for every j whose
    // d_ij - tau sig_ij < T (sig_ij = (|a|^2 + |w_i - w_j|) / (2 |a|)).
    template <typename F>
    void for_each(double T, double tau, F f) {
        if (!kd) {
            for (const Cand& c : cand) f(c);
            return;
        }
        const double Tr = T + 1e-6 * std::fabs(T);
        std::vector<int64_t> stack{0};
        while (!stack.empty()) {
            const KdNode& nd = kd->nodes[(size_t)stack.back()];
            stack.pop_back();
            if (node_key(nd, p, wi, tau) >= Tr) continue;
            if (nd.left >= 0) {
                stack.push_back(nd.left);
                stack.push_back(nd.right);
                continue;
            }
            for (int64_t q = nd.begin; q < nd.end; ++q) {
                const int64_t j = kd->perm[(size_t)q];
                if (j == i || in.loser[(size_t)j] || j == in.moved) continue;
                double d2;
                const double d = dist_of(j, &d2);
                if (d2 == 0.0) continue;
                f(Cand{d, j});
            }
        }
        const int64_t mv = in.moved;
        if (mv >= 0 && mv != i && !in.loser[(size_t)mv]) {
            double d2;
            const double d = dist_of(mv, &d2);
            if (d2 != 0.0) f(Cand{d, mv});
        }
    }

    // Smallest distance |p_j - p_i| to another (non-coincident, non-loser) site.
    double nearest() {
        double best2 = INFINITY;
        auto consider = [&](int64_t j) {
            if (j == i || in.loser[(size_t)j]) return;
            double d2;
            dist_of(j, &d2);
            if (d2 != 0.0) best2 = std::min(best2, d2);
        };
        if (!kd) {
            for (const Cand& c : cand) consider(c.j);
            return std::sqrt(best2);
        }
        if (in.moved >= 0) consider(in.moved);
        std::vector<std::pair<double, int64_t>> pq{{0.0, 0}};
        while (!pq.empty()) {
            std::pop_heap(pq.begin(), pq.end(), std::greater<>());
            const auto e = pq.back();
            pq.pop_back();
            if (e.first * e.first > best2) break;
            const KdNode& nd = kd->nodes[(size_t)e.second];
            if (nd.left < 0) {
                for (int64_t q = nd.begin; q < nd.end; ++q)
                    if (kd->perm[(size_t)q] != in.moved) consider(kd->perm[(size_t)q]);
            } else {
                for (int64_t ch : {nd.left, nd.right}) {
                    pq.push_back({box_distance(kd->nodes[(size_t)ch], p), ch});
                    std::push_heap(pq.begin(), pq.end(), std::greater<>());
                }
            }
        }
        return std::sqrt(best2);
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
    bool alive = B.start(i, coincident);
    if (coincident) flags |= OF_COINCIDENT;
    if (!alive) {
        P.empty = true;
        P.v.clear();
        return 0;
    }
    size_t t = 0;
    double R = max_radius(P);
    Cand c;
    for (;; ++t) {
        if (!B.next(c)) break;
        // a weight raised by wshift >= 0 only moves planes outward (by
        // wshift / (2 D)), so the unshifted order still bounds the rest
        if (c.d > R) break;
        Plane h = make_plane(in, i, c.j);
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
    // (the k-d tree enumerates every candidate with d - tau_m sig below
    // R + tau_m (emax + R), which includes every one not skipped here)
    B.for_each(R + tau_m * (emax + R), tau_m, [&](const Cand& c) {
        if (c.d - R > tau_m * (emax + R)) {
            Plane h = make_plane(in, i, c.j);
            if (c.d - R >= tau_m * (emax + R + h.sig)) return;
            visit(h);
        } else {
            visit(make_plane(in, i, c.j));
        }
    });
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

// Everything the cells of one input share: FP64 copies of the sites and
// weights, the coincident-site marks, and the k-d tree (when used).
struct Session {
    std::vector<double> xyz, w;
    Input in;
    KdTree tree;
    bool use_kd = false;
};

Session* open_session(const double* xyz, const double* w, int64_t n, const double* box, int nthreads, int mode) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    Session* sp = new Session;
    Session& S = *sp;
    S.xyz.assign(xyz, xyz + 3 * n);
    if (w) S.w.assign(w, w + n);
    S.in = Input{S.xyz.data(), w ? S.w.data() : nullptr, n, {box[0], box[1], box[2], box[3], box[4], box[5]}, {}, {},
                 -1};
    xyz = S.xyz.data();
    w = w ? S.w.data() : nullptr;
    // coincident sites: sort by position, the heaviest of each run of equal
    // positions (lowest index among equals) is the only one that keeps a cell
    S.in.loser.assign((size_t)n, 0);
    S.in.twin.assign((size_t)n, 0);
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
                for (size_t t = a; t < b; ++t) S.in.twin[(size_t)ord[t]] = 1;
                size_t win = a;
                for (size_t t = a + 1; t < b; ++t) {
                    double wt = w ? (double)w[ord[t]] : 0.0, ww = w ? (double)w[ord[win]] : 0.0;
                    if (wt > ww || (wt == ww && ord[t] < ord[win])) win = t;
                }
                for (size_t t = a; t < b; ++t)
                    if (t != win) S.in.loser[(size_t)ord[t]] = 1;
            }
            a = b;
        }
    }
    S.use_kd = mode == 2 || (mode == 0 && n > 20000);
    if (S.use_kd) kd_build(S.in, S.tree);
    return sp;
}

Result* compute(Session& S, const int64_t* cells, int64_t m, int want_margin) {
    const Input& in = S.in;
    const int64_t n = in.n;
    Result* res = new Result;
    const int64_t count = cells ? m : n;
    res->cells.resize((size_t)count);
#pragma omp parallel
    {
        Builder B(in, S.use_kd ? &S.tree : nullptr);
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
                    double l = B.nearest();
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

}  // namespace

extern "C" {

// Compute cells `cells[0..m)` (all n cells if cells == NULL).  `box` is
// [lo.xyz, hi.xyz] in FP64.  Returns an opaque handle, or NULL on bad input.
// `want_margin` = 0 skips the robustness margin (faster).  `mode`: candidate
// enumeration, 1 brute force, 2 k-d tree, 0 brute force up to 20000 sites and
// the k-d tree above (the results are identical).
void* orc_run(const float* xyz, const float* w, int64_t n, const double* box, const int64_t* cells, int64_t m,
              int want_margin, int nthreads, int mode) {
    if (n <= 0 || !xyz || !box || mode < 0 || mode > 2) return nullptr;
    std::vector<double> x((size_t)(3 * n)), ww;
    for (int64_t k = 0; k < 3 * n; ++k) x[(size_t)k] = (double)xyz[k];
    if (w) {
        ww.resize((size_t)n);
        for (int64_t k = 0; k < n; ++k) ww[(size_t)k] = (double)w[k];
    }
    Session* S = open_session(x.data(), w ? ww.data() : nullptr, n, box, nthreads, mode);
    Result* r = compute(*S, cells, m, want_margin);
    delete S;
    return r;
}

// The same with FP64 sites and weights.
void* orc_run64(const double* xyz, const double* w, int64_t n, const double* box, const int64_t* cells, int64_t m,
                int want_margin, int nthreads, int mode) {
    if (n <= 0 || !xyz || !box || mode < 0 || mode > 2) return nullptr;
    Session* S = open_session(xyz, w, n, box, nthreads, mode);
    Result* r = compute(*S, cells, m, want_margin);
    delete S;
    return r;
}

// A session keeps FP64 sites (and the k-d tree) for many calls, each of which
// may move one site first (finite differences): orc_session_cells computes
// the cells `cells[0..m)` with site `moved` (or none, if negative) at
// moved_xyzw[0..2] with weight moved_xyzw[3], and puts it back afterwards.
// The moved site must not coincide with another site.  Not thread-safe.
void* orc_session_open(const double* xyz, const double* w, int64_t n, const double* box, int nthreads, int mode) {
    if (n <= 0 || !xyz || !box || mode < 0 || mode > 2) return nullptr;
    return open_session(xyz, w, n, box, nthreads, mode);
}

void* orc_session_cells(void* h, const int64_t* cells, int64_t m, int want_margin, int64_t moved,
                        const double* moved_xyzw) {
    Session& S = *(Session*)h;
    if (moved >= S.in.n || (moved >= 0 && (!moved_xyzw || S.in.twin[(size_t)moved]))) return nullptr;
    double keep[4] = {0, 0, 0, 0};
    if (moved >= 0) {
        for (int k = 0; k < 3; ++k) {
            keep[k] = S.xyz[(size_t)(3 * moved + k)];
            S.xyz[(size_t)(3 * moved + k)] = moved_xyzw[k];
        }
        if (!S.w.empty()) {
            keep[3] = S.w[(size_t)moved];
            S.w[(size_t)moved] = moved_xyzw[3];
        }
        S.in.moved = moved;
    }
    Result* r = compute(S, cells, m, want_margin);
    if (moved >= 0) {
        for (int k = 0; k < 3; ++k) S.xyz[(size_t)(3 * moved + k)] = keep[k];
        if (!S.w.empty()) S.w[(size_t)moved] = keep[3];
        S.in.moved = -1;
    }
    return r;
}

void orc_session_close(void* h) { delete (Session*)h; }

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
