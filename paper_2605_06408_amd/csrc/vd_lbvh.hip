// Input packing and the power-augmented BVH (paper Sec. 4.3, supplementary
// Sec. A "Input packing" and "Power-augmented BVH").
//
// The paper packs each site as one 16-byte (x, y, z, w) record and builds a
// binary BVH whose nodes also store the largest weight below them.  Here the
// BVH is a linear BVH: 63-bit Morton codes (21 bits per axis inside the clip
// box), an LSD radix sort, the Karras (2012) binary radix tree over the sorted
// codes, subtrees of at most `leaf_size` sites collapsed into leaves, and a
// bottom-up pass that fills every node's child boxes and max weights.
#include "vd_internal.h"

namespace vd {

// ------------------------------------------------------------------ packing

__global__ void k_pack(const float* __restrict__ xyz, const float* __restrict__ w, int64_t n, float4* __restrict__ pts,
                       uint32_t* err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
    float ww = w ? w[i] : 0.0f;
    if (!(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(ww))) atomicOr(err, 1u);
    pts[i] = make_float4(x, y, z, ww);
}

hipError_t launch_pack(const float* xyz, const float* w, int64_t n, float4* pts, uint32_t* err, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)blocks), dim3(256), 0, s, xyz, w, n, pts, err);
    return hipGetLastError();
}

// Bounding box of the sites: per-block partial min/max, then one block folds them.
__global__ __launch_bounds__(256) void k_bbox_partial(const float4* __restrict__ pts, int64_t n, float* partial) {
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float4 p = pts[i];
        mn[0] = fminf(mn[0], p.x); mn[1] = fminf(mn[1], p.y); mn[2] = fminf(mn[2], p.z);
        mx[0] = fmaxf(mx[0], p.x); mx[1] = fmaxf(mx[1], p.y); mx[2] = fmaxf(mx[2], p.z);
    }
    __shared__ float red[6][256];
    for (int c = 0; c < 3; ++c) {
        red[c][threadIdx.x] = mn[c];
        red[3 + c][threadIdx.x] = mx[c];
    }
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            for (int c = 0; c < 3; ++c) {
                red[c][threadIdx.x] = fminf(red[c][threadIdx.x], red[c][threadIdx.x + o]);
                red[3 + c][threadIdx.x] = fmaxf(red[3 + c][threadIdx.x], red[3 + c][threadIdx.x + o]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(64) void k_bbox_final(const float* partial, int nblk, float* bbox, uint32_t* err) {
    if (threadIdx.x != 0) return;
    float b[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int k = 0; k < nblk; ++k)
        for (int c = 0; c < 3; ++c) {
            b[c] = fminf(b[c], partial[6 * k + c]);
            b[3 + c] = fmaxf(b[3 + c], partial[6 * k + 3 + c]);
        }
    for (int c = 0; c < 6; ++c) bbox[c] = b[c];
    for (int c = 0; c < 3; ++c)
        if (!(b[3 + c] > b[c])) atomicOr(err, 2u);  // flat point set: no 3D box
}

hipError_t launch_bbox(const float4* pts, int64_t n, float* partial, int nblk_max, float* bbox, uint32_t* err,
                       hipStream_t s) {
    int64_t want = (n + 4095) / 4096;
    int nblk = (int)(want < nblk_max ? want : nblk_max);
    if (nblk < 1) nblk = 1;
    hipLaunchKernelGGL(k_bbox_partial, dim3(nblk), dim3(256), 0, s, pts, n, partial);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, s, partial, nblk, bbox, err);
    return hipGetLastError();
}

__global__ void k_check_bbox(const float* bbox, uint32_t* err) {
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c)
            if (!(bbox[3 + c] > bbox[c]) || !isfinite(bbox[c]) || !isfinite(bbox[3 + c])) atomicOr(err, 2u);
}

hipError_t launch_check_bbox(float* bbox, uint32_t* err, hipStream_t s) {
    hipLaunchKernelGGL(k_check_bbox, dim3(1), dim3(64), 0, s, bbox, err);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Morton

__device__ inline uint64_t spread21(uint32_t v) {
    uint64_t x = v & 0x1FFFFFu;
    x = (x | (x << 32)) & 0x001F00000000FFFFull;
    x = (x | (x << 16)) & 0x001F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ inline uint32_t quantize21(float x, float lo, float inv_ext) {
    float f = (x - lo) * inv_ext;
    f = fminf(fmaxf(f, 0.0f), 2097151.0f);
    return (uint32_t)f;
}

__global__ void k_morton(const float4* __restrict__ pts, int64_t n, const float* __restrict__ bbox,
                         uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float4 p = pts[i];
    const float scale = 2097152.0f;
    uint32_t qx = quantize21(p.x, bbox[0], scale / (bbox[3] - bbox[0]));
    uint32_t qy = quantize21(p.y, bbox[1], scale / (bbox[4] - bbox[1]));
    uint32_t qz = quantize21(p.z, bbox[2], scale / (bbox[5] - bbox[2]));
    keys[i] = (spread21(qx) << 2) | (spread21(qy) << 1) | spread21(qz);
    vals[i] = (uint32_t)i;
}

hipError_t launch_morton(const float4* pts, int64_t n, const float* bbox, uint64_t* keys, uint32_t* vals,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_morton, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pts, n, bbox, keys, vals);
    return hipGetLastError();
}

// ------------------------------------------------------------------ radix sort
// One 8-bit digit per pass: per-tile digit histograms (digit-major), an
// exclusive scan of them, and a stable scatter.  A tile is 4096 keys handled
// by 4 waves; each wave ranks its 1024 keys in 16 rounds of 64, finding the
// lanes that share a digit with 8 ballots (one per digit bit).

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;

size_t radix_hist_size(int64_t n) { return (size_t)256 * (size_t)((n + kSortTile - 1) / kSortTile); }

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                              uint32_t* __restrict__ hist, int nblk) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int it = 0; it < kSortItems; ++it) {
        int64_t i = base + it * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

__device__ inline void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint64_t* __restrict__ kin,
                                                                 const uint32_t* __restrict__ vin,
                                                                 uint64_t* __restrict__ kout,
                                                                 uint32_t* __restrict__ vout, int64_t n, int shift,
                                                                 const uint32_t* __restrict__ offs, int nblk) {
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t wbase[4][256];
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    for (int t = threadIdx.x; t < 1024; t += kSortThreads) (&wcnt[0][0])[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)wv * 64 * kSortItems;
    const uint64_t lt = (ln == 0) ? 0ull : (~0ull >> (64 - ln));
    uint64_t key[kSortItems];
    uint32_t val[kSortItems], rank[kSortItems];
    int dig[kSortItems];
    for (int it = 0; it < kSortItems; ++it) {
        int64_t i = base + it * 64 + ln;
        bool ok = i < n;
        key[it] = ok ? kin[i] : 0ull;
        val[it] = ok ? vin[i] : 0u;
        int d = ok ? (int)((key[it] >> shift) & 255u) : 0;
        dig[it] = ok ? d : -1;
        uint64_t peers = __ballot(ok);
        for (int b = 0; b < 8; ++b) {
            uint64_t bb = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bb : ~bb;
        }
        uint32_t before = ok ? wcnt[wv][d] : 0u;
        rank[it] = before + (uint32_t)__popcll(peers & lt);
        wave_fence();
        if (ok && (peers & lt) == 0) wcnt[wv][d] = before + (uint32_t)__popcll(peers);
        wave_fence();
    }
    __syncthreads();
    {
        int d = threadIdx.x;
        uint32_t s = 0;
        for (int w = 0; w < 4; ++w) {
            wbase[w][d] = s;
            s += wcnt[w][d];
        }
    }
    __syncthreads();
    for (int it = 0; it < kSortItems; ++it) {
        if (dig[it] < 0) continue;
        int d = dig[it];
        uint32_t pos = offs[(int64_t)d * nblk + blockIdx.x] + wbase[wv][d] + rank[it];
        kout[pos] = key[it];
        vout[pos] = val[it];
    }
}

hipError_t radix_sort(uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp, uint32_t* vals_tmp, int64_t n, int bits,
                      uint32_t* hist, uint32_t* scan_tmp, hipStream_t s, bool* result_in_tmp) {
    int nblk = (int)((n + kSortTile - 1) / kSortTile);
    uint64_t* ka = keys;
    uint32_t* va = vals;
    uint64_t* kb = keys_tmp;
    uint32_t* vb = vals_tmp;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kSortThreads), 0, s, ka, n, shift, hist, nblk);
        hipError_t e = scan_u32(hist, (int64_t)256 * nblk, hist, scan_tmp, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kSortThreads), 0, s, ka, va, kb, vb, n, shift, hist,
                           nblk);
        uint64_t* tk = ka; ka = kb; kb = tk;
        uint32_t* tv = va; va = vb; vb = tv;
    }
    *result_in_tmp = (ka != keys);
    return hipGetLastError();
}

// ------------------------------------------------------------------ gather

__global__ void k_gather(const float4* __restrict__ pts, const uint32_t* __restrict__ order, int64_t n,
                         float4* __restrict__ spts, uint32_t* __restrict__ inv) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t i = order[k];
    spts[k] = pts[i];
    inv[i] = (uint32_t)k;
}

hipError_t launch_gather(const float4* pts, const uint32_t* order, int64_t n, float4* spts, uint32_t* inv,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pts, order, n, spts, inv);
    return hipGetLastError();
}

// Coincident sites share a Morton code, so after the sort they sit in one run
// of equal codes.  Among sites with one position the heaviest keeps its cell
// (ties: lowest original index); the others are marked with weight -inf: their
// cells are empty and their planes, implied by the winner's, are skipped.
__global__ void k_loser_mark(const float4* __restrict__ spts, const uint64_t* __restrict__ keys,
                             const uint32_t* __restrict__ order, int64_t n, uint8_t* __restrict__ mark) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint64_t key = keys[k];
    const float4 p = spts[k];
    const uint32_t ok = order[k];
    bool lose = false;
    for (int dir = -1; dir <= 1; dir += 2) {
        for (int64_t j = k + dir; j >= 0 && j < n && keys[j] == key; j += dir) {
            float4 q = spts[j];
            if (q.x == p.x && q.y == p.y && q.z == p.z && (q.w > p.w || (q.w == p.w && order[j] < ok))) lose = true;
        }
    }
    mark[k] = lose ? 1 : 0;
}

__global__ void k_loser_apply(float4* __restrict__ spts, const uint8_t* __restrict__ mark, int64_t n) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n && mark[k]) spts[k].w = -INFINITY;
}

hipError_t launch_losers(float4* spts, const uint64_t* keys, const uint32_t* order, int64_t n, uint8_t* mark,
                         hipStream_t s) {
    unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_loser_mark, dim3(blocks), dim3(256), 0, s, spts, keys, order, n, mark);
    hipLaunchKernelGGL(k_loser_apply, dim3(blocks), dim3(256), 0, s, spts, mark, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Karras tree
// Internal node i of the binary radix tree over n sorted codes; equal codes
// are made distinct by their position (Karras 2012, Sec. 4).

__device__ inline int kdelta(const uint64_t* keys, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    uint64_t a = keys[i], b = keys[j];
    return a != b ? __clzll((long long)(a ^ b)) : 64 + __clz(i ^ j);
}

__global__ void k_karras(const uint64_t* __restrict__ keys, int n, int2* __restrict__ child, uint32_t* __restrict__ up,
                         int2* __restrict__ range) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int d = (kdelta(keys, n, i, i + 1) - kdelta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = kdelta(keys, n, i, i - d);
    int lmax = 2;
    while (kdelta(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (kdelta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = kdelta(keys, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (kdelta(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int gamma = i + s * d + (d < 0 ? -1 : 0);
    int first = i < j ? i : j, last = i < j ? j : i;
    int left = (first == gamma) ? ~gamma : gamma;
    int right = (last == gamma + 1) ? ~(gamma + 1) : gamma + 1;
    child[i] = make_int2(left, right);
    range[i] = make_int2(first, last);
    // parent link of each internal child: parent index and which child it is
    if (left >= 0) up[left] = (uint32_t)i << 1;
    if (right >= 0) up[right] = ((uint32_t)i << 1) | 1u;
    if (i == 0) up[0] = kNoParent;
}

hipError_t launch_karras(const uint64_t* keys, int64_t n, int2* child, uint32_t* up, int2* range, hipStream_t s) {
    if (n < 2) return hipSuccess;
    hipLaunchKernelGGL(k_karras, dim3((unsigned)((n - 1 + 255) / 256)), dim3(256), 0, s, keys, (int)n, child, up,
                       range);
    return hipGetLastError();
}

// ------------------------------------------------------------------ bounds
// Every node covers a contiguous range of sites in Morton order, so each
// child's box and max weight is a reduction over that range.  Boxes of
// aligned blocks of 64 sites are folded into a sparse table (level k holds
// the box of 2^k consecutive blocks), and a range is its partial head and tail
// blocks plus two overlapping table entries (min/max are idempotent).  No
// atomics, no fences, no climb.

struct BoxAcc {
    float lo[3], hi[3], w;
    __device__ void init() {
        lo[0] = lo[1] = lo[2] = INFINITY;
        hi[0] = hi[1] = hi[2] = -INFINITY;
        w = -INFINITY;
    }
    __device__ void add(float4 p) {
        lo[0] = fminf(lo[0], p.x); lo[1] = fminf(lo[1], p.y); lo[2] = fminf(lo[2], p.z);
        hi[0] = fmaxf(hi[0], p.x); hi[1] = fmaxf(hi[1], p.y); hi[2] = fmaxf(hi[2], p.z);
        w = fmaxf(w, p.w);
    }
    __device__ void add(const NodeChild& c) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], c.lo[k]);
            hi[k] = fmaxf(hi[k], c.hi[k]);
        }
        w = fmaxf(w, c.wmax);
    }
    __device__ NodeChild out(uint32_t ref) const {
        NodeChild c;
        for (int k = 0; k < 3; ++k) {
            c.lo[k] = lo[k];
            c.hi[k] = hi[k];
        }
        c.wmax = w;
        c.ref = ref;
        return c;
    }
};

__device__ inline float wave_min_f(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ inline float wave_max_f(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// level 0: one wave per block of 64 sites
__global__ __launch_bounds__(256) void k_block_boxes(const float4* __restrict__ spts, int64_t n,
                                                     NodeChild* __restrict__ lvl0, int64_t nb) {
    const int64_t b = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int ln = threadIdx.x & 63;
    if (b >= nb) return;
    const int64_t i = b * 64 + ln;
    float4 p = i < n ? spts[i] : make_float4(INFINITY, INFINITY, INFINITY, -INFINITY);
    float4 q = i < n ? p : make_float4(-INFINITY, -INFINITY, -INFINITY, -INFINITY);
    float l0 = wave_min_f(p.x), l1 = wave_min_f(p.y), l2 = wave_min_f(p.z);
    float h0 = wave_max_f(q.x), h1 = wave_max_f(q.y), h2 = wave_max_f(q.z), w = wave_max_f(q.w);
    if (ln == 0) {
        NodeChild c;
        c.lo[0] = l0; c.lo[1] = l1; c.lo[2] = l2;
        c.hi[0] = h0; c.hi[1] = h1; c.hi[2] = h2;
        c.wmax = w;
        c.ref = 0;
        lvl0[b] = c;
    }
}

// level k from level k-1: entry b covers blocks [b, b + 2^k)
__global__ void k_sparse_level(const NodeChild* __restrict__ prev, NodeChild* __restrict__ cur, int64_t nb,
                               int64_t half) {
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b + 2 * half > nb) return;
    BoxAcc a;
    a.init();
    a.add(prev[b]);
    a.add(prev[b + half]);
    cur[b] = a.out(0);
}

__device__ inline int floor_log2(int64_t x) { return 63 - __clzll((long long)x); }

__device__ NodeChild range_box(const float4* __restrict__ spts, const NodeChild* __restrict__ table, int64_t nb,
                               int f, int l, uint32_t ref) {
    BoxAcc a;
    a.init();
    const int64_t b0 = ((int64_t)f + 63) >> 6;      // first full block
    const int64_t b1 = ((int64_t)l + 1) >> 6;       // one past the last full block
    if (b1 <= b0 || l - f < 128) {
        for (int i = f; i <= l; ++i) a.add(spts[i]);
    } else {
        for (int64_t i = f; i < b0 * 64; ++i) a.add(spts[i]);
        for (int64_t i = b1 * 64; i <= l; ++i) a.add(spts[i]);
        const int64_t cnt = b1 - b0;
        const int k = floor_log2(cnt);
        const NodeChild* lv = table + (int64_t)k * nb;
        a.add(lv[b0]);
        a.add(lv[b1 - (int64_t(1) << k)]);
    }
    return a.out(ref);
}

__global__ void k_node_boxes(const float4* __restrict__ spts, int n, const int2* __restrict__ child,
                             const int2* __restrict__ range, const NodeChild* __restrict__ table, int64_t nb,
                             Node* __restrict__ nodes, int leaf_size) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int2 r = range[i];
    if (r.y - r.x + 1 <= leaf_size) return;  // a leaf itself: never visited as a node
    int2 ch = child[i];
    for (int s = 0; s < 2; ++s) {
        int c = s ? ch.y : ch.x;
        int f, l;
        if (c < 0) {
            f = l = ~c;
        } else {
            int2 cr = range[c];
            f = cr.x;
            l = cr.y;
        }
        uint32_t cnt = (uint32_t)(l - f + 1);
        uint32_t ref = cnt <= (uint32_t)leaf_size ? leaf_ref((uint32_t)f, cnt) : (uint32_t)c;
        nodes[i].c[s] = range_box(spts, table, nb, f, l, ref);
    }
}

// The leaf record of every site: the node whose child record is the leaf
// (a subtree of at most leaf_size sites under a node of more) and which child.
__global__ void k_leaf_of(const int2* __restrict__ child, const int2* __restrict__ range, int n, int leaf_size,
                          uint32_t* __restrict__ leaf_of) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int2 r = range[i];
    if (r.y - r.x + 1 <= leaf_size) return;
    int2 ch = child[i];
    for (int s = 0; s < 2; ++s) {
        int c = s ? ch.y : ch.x;
        int f = c < 0 ? ~c : range[c].x, l = c < 0 ? ~c : range[c].y;
        if (l - f + 1 > leaf_size) continue;
        for (int k = f; k <= l; ++k) leaf_of[k] = ((uint32_t)i << 1) | (uint32_t)s;
    }
}

size_t box_table_size(int64_t n) {
    int64_t nb = (n + 63) / 64;
    int levels = 1;
    while ((int64_t(1) << levels) <= nb) ++levels;
    return (size_t)levels * (size_t)nb;
}

hipError_t launch_bounds(const float4* spts, int64_t n, const int2* child, const int2* range, NodeChild* table,
                         Node* nodes, uint32_t* leaf_of, int leaf_size, hipStream_t s) {
    if (n < 2) return hipSuccess;
    const int64_t nb = (n + 63) / 64;
    hipLaunchKernelGGL(k_block_boxes, dim3((unsigned)((nb * 64 + 255) / 256)), dim3(256), 0, s, spts, n, table, nb);
    int k = 1;
    for (int64_t half = 1; 2 * half <= nb; half *= 2, ++k) {
        hipLaunchKernelGGL(k_sparse_level, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s,
                           table + (int64_t)(k - 1) * nb, table + (int64_t)k * nb, nb, half);
    }
    hipLaunchKernelGGL(k_node_boxes, dim3((unsigned)((n - 1 + 255) / 256)), dim3(256), 0, s, spts, (int)n, child,
                       range, table, nb, nodes, leaf_size);
    hipLaunchKernelGGL(k_leaf_of, dim3((unsigned)((n - 1 + 255) / 256)), dim3(256), 0, s, child, range, (int)n,
                       leaf_size, leaf_of);
    return hipGetLastError();
}

}  // namespace vd
