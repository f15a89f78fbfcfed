// Backward pass: gradients of cell volumes, centroids and vertex positions
// with respect to site positions and weights, through the combinatorics of
// the last build (its staged cell records are the checkpoint; nothing is
// re-clipped).
//
// In the frame of site p_i a cell is {y : a_f . y <= b_f} (paper Sec. 3,
// Eq. 1: a_f = p_j - p_i, b_f = (|a_f|^2 + w_i - w_j) / 2 for the plane of
// site j; a box face has a_f = +-e_k).  Moving plane f by (da_f, db_f) moves
// the points y of its facet along the outward normal by
// (db_f - da_f . y) / |a_f|, so with A_f, Y_f and S_f = int_F y y^T dA the
// area, centroid and second moment of facet f:
//     dV = sum_f (A_f db_f - A_f Y_f . da_f) / |a_f|
//     dm = sum_f (A_f Y_f db_f - S_f da_f) / |a_f|,   m = int_C y dV,
// and c = p_i + m / V.  A vertex is x = p_i + M^-1 b (rows of M: the normals
// of its three planes), so a gradient g on x gives d/db = M^-T g and
// d/da_k = -(M^-T g)_k y.  The plane parameters then carry the gradient to
// the sites: da_f = dp_j - dp_i, db_f = a_f . da_f + (dw_i - dw_j) / 2, or
// db_f = -a_f . dp_i for a box face.
//
// Layout: one wave per cell, lanes over its facets.  Each lane walks its
// facet's vertex ring (staged by the forward pass) and recomputes the ring's
// vertices in FP64 from their three planes, which is cheaper than storing
// them.  A first walk gives V and m (pyramids with apex at the site), the
// second the facet integrals and the gradient of each plane.  The gradient
// a cell sends to neighbour j is stored with the facet; each site then sums
// what its neighbours sent it, in ascending neighbour order (deterministic).
// Shares stay in FP64 until that sum: around thin cells (tight clusters) the
// shares of two neighbouring cells are many orders of magnitude larger than
// the site gradient they cancel to.
// A facet whose neighbour does not list the cell back (possible only on
// configurations FP32 cannot decide) is added with an atomic instead.
// When the box is the sites' own bounding box its faces move with the
// extreme sites (b = p_i,k - min_j p_j,k for a lower face, max_j p_j,k - p_i,k
// for an upper one): the sum over all cells of dL/db of each face goes to the
// site on that face with the lowest index, summed in a fixed order.
#include <mutex>

#include "vd_internal.h"

namespace vd {
namespace {

struct CellRec {
    const float4* V;
    const uint64_t* T64;
    const int32_t* C;
    const uint16_t* FS;
    const uint16_t* FV;
};

__device__ inline CellRec record_of(const BwdArgs& a, uint32_t k) {
    const uint32_t loc = a.loc[k], tier = loc >> 30;
    const Stage st = tier == 0 ? a.stage[0] : (tier == 1 ? a.stage[1] : (tier == 2 ? a.stage[2] : a.stage[3]));
    const int64_t slot = loc & 0x3FFFFFFFu;
    const int64_t cap = st.cap;
    CellRec r;
    r.V = st.vert + slot * cap;
    r.T64 = st.tri64 ? st.tri64 + slot * cap : nullptr;
    r.C = st.code + slot * cap;
    r.FS = st.fsize + slot * cap;
    r.FV = st.fv + slot * 3 * cap;
    return r;
}

__device__ inline void ranks_of(const CellRec& r, uint32_t u, uint32_t* t) {
    if (r.T64) {
        const uint64_t x = r.T64[u];
        t[0] = (uint32_t)(x & 0x1FFFFFu);
        t[1] = (uint32_t)((x >> 21) & 0x1FFFFFu);
        t[2] = (uint32_t)((x >> 42) & 0x1FFFFFu);
    } else {
        const uint32_t x = __float_as_uint(r.V[u].w);
        t[0] = x & 1023u;
        t[1] = (x >> 10) & 1023u;
        t[2] = (x >> 20) & 1023u;
    }
}

struct Site {
    double p[3];
    double w;
};

// Plane of facet code `code` in the frame of site s, FP64 from the FP32 inputs.
__device__ inline void plane_of(const BwdArgs& a, const Site& s, int32_t code, double* n, double* b) {
    if (code >= 0) {
        const float4 q = a.pts[a.inv[code]];
        n[0] = (double)q.x - s.p[0];
        n[1] = (double)q.y - s.p[1];
        n[2] = (double)q.z - s.p[2];
        *b = 0.5 * (n[0] * n[0] + n[1] * n[1] + n[2] * n[2] + (s.w - (double)q.w));
    } else {
        const int c = -code - 1, ax = c >> 1, side = c & 1;
        n[0] = n[1] = n[2] = 0.0;
        n[ax] = side ? 1.0 : -1.0;
        *b = side ? ((double)a.bbox[3 + ax] - s.p[ax]) : (s.p[ax] - (double)a.bbox[ax]);
    }
}

__device__ inline void cross(const double* u, const double* v, double* o) {
    o[0] = u[1] * v[2] - u[2] * v[1];
    o[1] = u[2] * v[0] - u[0] * v[2];
    o[2] = u[0] * v[1] - u[1] * v[0];
}
__device__ inline double dot(const double* u, const double* v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; }

// A vertex of the cell: its position y (frame of the site), the rows of M
// and their cofactors (so that M^-T g = (c_k . g) / det), and its ranks.
struct Vtx {
    double y[3];
    double c[3][3];
    double det;
    uint32_t t[3];
};

__device__ inline void vertex(const BwdArgs& a, const Site& s, const CellRec& r, uint32_t u, Vtx* v) {
    ranks_of(r, u, v->t);
    double n[3][3], b[3];
    for (int k = 0; k < 3; ++k) plane_of(a, s, r.C[v->t[k]], n[k], &b[k]);
    cross(n[1], n[2], v->c[0]);
    cross(n[2], n[0], v->c[1]);
    cross(n[0], n[1], v->c[2]);
    v->det = dot(n[0], v->c[0]);
    const double inv = v->det != 0.0 ? 1.0 / v->det : 0.0;
    for (int q = 0; q < 3; ++q) v->y[q] = (b[0] * v->c[0][q] + b[1] * v->c[1][q] + b[2] * v->c[2][q]) * inv;
}

__device__ inline double wsum(double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Is `who` among the neighbours of cell j (original ids)?  Binary search of
// the ascending site codes at the end of j's facet list.
__device__ inline int64_t find_facet(const BwdArgs& a, uint32_t j, int32_t who) {
    const CellRec r = record_of(a, a.inv[j]);
    const int F = (int)a.cnt_f[j], nn = (int)a.cnt_n[j];
    int lo = F - nn, hi = F - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int32_t c = r.C[mid];
        if (c == who) return mid;
        if (c < who) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

__global__ __launch_bounds__(256) void k_bwd_cells(BwdArgs a) {
    const int ln = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    double bx[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // dL/db of the box faces of this lane's facets
    for (int64_t i = wave; i < a.n; i += nwaves) {
        const uint32_t k = a.inv[i];
        const float4 ps = a.pts[k];
        double gc[3] = {0.0, 0.0, 0.0};
        if (a.g_cen)
            for (int q = 0; q < 3; ++q) gc[q] = (double)a.g_cen[3 * i + q];
        const double gv = a.g_vol ? (double)a.g_vol[i] : 0.0;
        const int nv = (int)a.cnt_v[i], F = (int)a.cnt_f[i];
        if (nv == 0) {
            // empty cell: V = 0 and c = p_i
            if (ln == 0) a.gself[i] = make_double4(gc[0], gc[1], gc[2], 0.0);
            continue;
        }
        Site s;
        s.p[0] = ps.x; s.p[1] = ps.y; s.p[2] = ps.z;
        s.w = ps.w;
        const CellRec r = record_of(a, k);
        const float* gvert = a.g_vert ? a.g_vert + 3 * a.off_v[i] : nullptr;

        // first walk: V and m from the pyramids (site, facet)
        double V = 0.0, m[3] = {0.0, 0.0, 0.0};
        {
            uint32_t carry = 0;
            for (int f0 = 0; f0 < F; f0 += 64) {
                const int f = f0 + ln;
                const uint32_t sz = f < F ? (uint32_t)r.FS[f] : 0u;
                uint32_t x = sz;
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t y = __shfl_up(x, o);
                    if (ln >= o) x += y;
                }
                if (f < F && sz >= 3) {
                    const uint32_t base = carry + x - sz;
                    double n[3], b;
                    plane_of(a, s, r.C[f], n, &b);
                    const double D = sqrt(dot(n, n));
                    const double nh[3] = {n[0] / D, n[1] / D, n[2] / D};
                    Vtx v0, v1, v2;
                    vertex(a, s, r, r.FV[base], &v0);
                    vertex(a, s, r, r.FV[base + 1], &v1);
                    double A = 0.0, AY[3] = {0.0, 0.0, 0.0};
                    for (uint32_t t = 2; t < sz; ++t) {
                        vertex(a, s, r, r.FV[base + t], &v2);
                        double e1[3], e2[3], cr[3];
                        for (int q = 0; q < 3; ++q) {
                            e1[q] = v1.y[q] - v0.y[q];
                            e2[q] = v2.y[q] - v0.y[q];
                        }
                        cross(e1, e2, cr);
                        const double at = 0.5 * dot(cr, nh);
                        A += at;
                        for (int q = 0; q < 3; ++q) AY[q] += at * (v0.y[q] + v1.y[q] + v2.y[q]) * (1.0 / 3.0);
                        v1 = v2;
                    }
                    V += b * A / (3.0 * D);
                    for (int q = 0; q < 3; ++q) m[q] += b * AY[q] / (4.0 * D);
                }
                carry += (uint32_t)__shfl(x, 63);
            }
            V = wsum(V);
            for (int q = 0; q < 3; ++q) m[q] = wsum(m[q]);
        }
        // L = gv V + gc . (p_i + m / V): dL/dV and dL/dm
        double alpha = 0.0, gam[3] = {0.0, 0.0, 0.0};
        if (V != 0.0) {
            alpha = gv - dot(gc, m) / (V * V);
            for (int q = 0; q < 3; ++q) gam[q] = gc[q] / V;
        }
        // second walk: facet integrals, plane gradients, scatter to sites
        double self_p[3] = {0.0, 0.0, 0.0}, self_w = 0.0;
        {
            uint32_t carry = 0;
            for (int f0 = 0; f0 < F; f0 += 64) {
                const int f = f0 + ln;
                const uint32_t sz = f < F ? (uint32_t)r.FS[f] : 0u;
                uint32_t x = sz;
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t y = __shfl_up(x, o);
                    if (ln >= o) x += y;
                }
                if (f < F && sz >= 3) {
                    const uint32_t base = carry + x - sz;
                    const int32_t code = r.C[f];
                    double n[3], b;
                    plane_of(a, s, code, n, &b);
                    const double D = sqrt(dot(n, n));
                    const double nh[3] = {n[0] / D, n[1] / D, n[2] / D};
                    double A = 0.0, AY[3] = {0.0, 0.0, 0.0}, S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                    double dA[3] = {0.0, 0.0, 0.0}, dB = 0.0;  // dL/da_f, dL/db_f from the vertices
                    Vtx v0, v1, v2;
                    // the vertex part of one ring vertex: its share of plane f,
                    // and the direct term dx/dp_i = I once per vertex
                    auto vertex_part = [&](const Vtx& v, uint32_t u) {
                        if (!gvert || v.det == 0.0) return;
                        const double g[3] = {(double)gvert[3 * u], (double)gvert[3 * u + 1], (double)gvert[3 * u + 2]};
                        const double g0 = dot(v.c[0], g), g1 = dot(v.c[1], g), g2 = dot(v.c[2], g);
                        const double gk = (v.t[0] == (uint32_t)f ? g0 : (v.t[1] == (uint32_t)f ? g1 : g2)) / v.det;
                        dB += gk;
                        for (int q = 0; q < 3; ++q) dA[q] -= gk * v.y[q];
                        const uint32_t tmin = min(v.t[0], min(v.t[1], v.t[2]));
                        if (tmin == (uint32_t)f)
                            for (int q = 0; q < 3; ++q) self_p[q] += g[q];
                    };
                    vertex(a, s, r, r.FV[base], &v0);
                    vertex(a, s, r, r.FV[base + 1], &v1);
                    vertex_part(v0, r.FV[base]);
                    vertex_part(v1, r.FV[base + 1]);
                    for (uint32_t t = 2; t < sz; ++t) {
                        const uint32_t u = r.FV[base + t];
                        vertex(a, s, r, u, &v2);
                        vertex_part(v2, u);
                        double e1[3], e2[3], cr[3], sm[3];
                        for (int q = 0; q < 3; ++q) {
                            e1[q] = v1.y[q] - v0.y[q];
                            e2[q] = v2.y[q] - v0.y[q];
                            sm[q] = v0.y[q] + v1.y[q] + v2.y[q];
                        }
                        cross(e1, e2, cr);
                        const double at = 0.5 * dot(cr, nh);
                        A += at;
                        for (int q = 0; q < 3; ++q) AY[q] += at * sm[q] * (1.0 / 3.0);
                        // int over the triangle of y y^T = at/12 (sum_i v_i v_i^T + s s^T)
                        const double h = at * (1.0 / 12.0);
                        const double* P0 = v0.y;
                        const double* P1 = v1.y;
                        const double* P2 = v2.y;
                        S[0] += h * (P0[0] * P0[0] + P1[0] * P1[0] + P2[0] * P2[0] + sm[0] * sm[0]);
                        S[1] += h * (P0[0] * P0[1] + P1[0] * P1[1] + P2[0] * P2[1] + sm[0] * sm[1]);
                        S[2] += h * (P0[0] * P0[2] + P1[0] * P1[2] + P2[0] * P2[2] + sm[0] * sm[2]);
                        S[3] += h * (P0[1] * P0[1] + P1[1] * P1[1] + P2[1] * P2[1] + sm[1] * sm[1]);
                        S[4] += h * (P0[1] * P0[2] + P1[1] * P1[2] + P2[1] * P2[2] + sm[1] * sm[2]);
                        S[5] += h * (P0[2] * P0[2] + P1[2] * P1[2] + P2[2] * P2[2] + sm[2] * sm[2]);
                        v1 = v2;
                    }
                    // dL/db_f and dL/da_f from the cell integrals
                    dB += (alpha * A + dot(gam, AY)) / D;
                    const double Sg[3] = {S[0] * gam[0] + S[1] * gam[1] + S[2] * gam[2],
                                          S[1] * gam[0] + S[3] * gam[1] + S[4] * gam[2],
                                          S[2] * gam[0] + S[4] * gam[1] + S[5] * gam[2]};
                    for (int q = 0; q < 3; ++q) dA[q] -= (alpha * AY[q] + Sg[q]) / D;
                    if (code >= 0) {
                        // site plane: a = p_j - p_i, b = (|a|^2 + w_i - w_j) / 2
                        double gp[3];
                        for (int q = 0; q < 3; ++q) gp[q] = dA[q] + dB * n[q];
                        const double gwj = -0.5 * dB;
                        for (int q = 0; q < 3; ++q) self_p[q] -= gp[q];
                        self_w += 0.5 * dB;
                        const double4 out = make_double4(gp[0], gp[1], gp[2], gwj);
                        a.gf[a.off_f[i] + f] = out;
                        if (find_facet(a, (uint32_t)code, (int32_t)i) < 0) {
                            double* o = a.orphan + 4 * (int64_t)code;
                            atomicAdd(o, out.x);
                            atomicAdd(o + 1, out.y);
                            atomicAdd(o + 2, out.z);
                            atomicAdd(o + 3, out.w);
                        }
                    } else {
                        // box face: b = +-(B_k - p_i,k), a fixed
                        for (int q = 0; q < 3; ++q) self_p[q] -= dB * n[q];
                        const int face = -code - 1;
#pragma unroll
                        for (int c = 0; c < 6; ++c)
                            if (c == face) bx[c] += dB;
                    }
                }
                carry += (uint32_t)__shfl(x, 63);
            }
        }
        for (int q = 0; q < 3; ++q) self_p[q] = wsum(self_p[q]);
        self_w = wsum(self_w);
        if (ln == 0) a.gself[i] = make_double4(self_p[0] + gc[0], self_p[1] + gc[1], self_p[2] + gc[2], self_w);
    }
    if (a.moving_box) {
        for (int c = 0; c < 6; ++c) {
            const double t = wsum(bx[c]);
            if (ln == 0) a.box_part[wave * 6 + c] = t;
        }
    }
}

// Lowest original index of a site on each face of the sites' bounding box
// (the box is their FP32 minimum and maximum, so some site equals each face).
__global__ __launch_bounds__(256) void k_bwd_box_arg(BwdArgs a) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n) return;
    const float4 p = a.pts_orig[j];
    const float v[3] = {p.x, p.y, p.z};
#pragma unroll
    for (int c = 0; c < 6; ++c)
        if (v[c >> 1] == a.bbox[(c & 1) ? 3 + (c >> 1) : (c >> 1)]) atomicMin(&a.box_arg[c], (uint32_t)j);
}

// Sum of the per-wave box-face partials, in a fixed order (one block).
__global__ __launch_bounds__(256) void k_bwd_box_sum(BwdArgs a, int64_t nwaves) {
    __shared__ double red[6][256];
    double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t w = threadIdx.x; w < nwaves; w += 256)
        for (int c = 0; c < 6; ++c) s[c] += a.box_part[w * 6 + c];
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int c = 0; c < 6; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 6) a.box_sum[threadIdx.x] = red[threadIdx.x][0];
}

// Per site: its own cell's share, then what each neighbour's cell sent it
// (ascending neighbour order), then the asymmetric remainder.
__global__ __launch_bounds__(256) void k_bwd_gather(BwdArgs a) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n) return;
    const double4 g0 = a.gself[j];
    double g[4] = {g0.x, g0.y, g0.z, g0.w};
    const int F = (int)a.cnt_f[j], nn = (int)a.cnt_n[j];
    if (nn > 0) {
        const CellRec r = record_of(a, a.inv[j]);
        for (int t = F - nn; t < F; ++t) {
            const uint32_t i = (uint32_t)r.C[t];
            const int64_t f = find_facet(a, i, (int32_t)j);
            if (f >= 0) {
                const double4 c = a.gf[a.off_f[i] + f];
                g[0] += c.x;
                g[1] += c.y;
                g[2] += c.z;
                g[3] += c.w;
            }
        }
    }
    const double* o = a.orphan + 4 * j;
    for (int q = 0; q < 4; ++q) g[q] += o[q];
    if (a.moving_box)
        for (int c = 0; c < 6; ++c)
            if (a.box_arg[c] == (uint32_t)j) g[c >> 1] += (c & 1) ? a.box_sum[c] : -a.box_sum[c];
    a.g_xyz[3 * j] = (float)g[0];
    a.g_xyz[3 * j + 1] = (float)g[1];
    a.g_xyz[3 * j + 2] = (float)g[2];
    if (a.g_w) a.g_w[j] = (float)g[3];
}

// Fill of 64-bit words (clears the scratch of the allocation-free entry
// point with a kernel rather than a memset node, so that the call can be
// captured into a HIP graph).
__global__ __launch_bounds__(256) void k_fill_u64(uint64_t* dst, int64_t count, uint64_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = value;
}

// Device scratch of vd_backward_noalloc: the facet shares, the per-site
// shares, the asymmetric remainders and the box-face partials of one
// backward, in one fixed array per device (set up once per device by
// bwd_scratch_init; host code uses only the address it returns).
static __device__ __align__(256) unsigned char scratch[kBwdScratchBytes];

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

}  // namespace

hipError_t bwd_scratch_init(int device, void** ptr) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

hipError_t launch_fill_u64(uint64_t* dst, int64_t count, uint64_t value, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, s, dst, count, value);
    return hipGetLastError();
}

int64_t bwd_waves(int64_t n) {
    const int64_t waves = n < 65536 ? n : 65536;
    return (waves + 3) / 4 * 4;  // whole blocks of four waves
}

hipError_t launch_backward(const BwdArgs& a, hipStream_t s) {
    if (a.n < 1) return hipSuccess;
    const int64_t waves = bwd_waves(a.n);
    const int64_t blocks = waves / 4;
    hipLaunchKernelGGL(k_bwd_cells, dim3((unsigned)blocks), dim3(256), 0, s, a);
    if (a.moving_box) {
        hipLaunchKernelGGL(k_bwd_box_arg, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_bwd_box_sum, dim3(1), dim3(256), 0, s, a, waves);
    }
    hipLaunchKernelGGL(k_bwd_gather, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace vd
