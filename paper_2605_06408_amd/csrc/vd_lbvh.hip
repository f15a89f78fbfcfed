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

__global__ void k_karras(const uint64_t* __restrict__ keys, int n, int2* __restrict__ child, int* __restrict__ parent_int,
                         int* __restrict__ parent_leaf, int2* __restrict__ range) {
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
    if (left >= 0) parent_int[left] = i; else parent_leaf[~left] = i;
    if (right >= 0) parent_int[right] = i; else parent_leaf[~right] = i;
    if (i == 0) parent_int[0] = -1;
}

hipError_t launch_karras(const uint64_t* keys, int64_t n, int2* child, int* parent_int, int* parent_leaf, int2* range,
                         hipStream_t s) {
    if (n < 2) return hipSuccess;
    hipLaunchKernelGGL(k_karras, dim3((unsigned)((n - 1 + 255) / 256)), dim3(256), 0, s, keys, (int)n, child,
                       parent_int, parent_leaf, range);
    return hipGetLastError();
}

// ------------------------------------------------------------------ bounds
// Bottom-up: one thread per site climbs towards the root; at each node the
// first arrival stores its child record and stops, the second merges both
// children and continues.  Children whose subtree holds <= leaf_size sites
// are referenced as leaves.

__device__ inline float ld_coherent(const float* p) {
    return __int_as_float(__hip_atomic_load((const int*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

__global__ void k_bounds(const float4* __restrict__ spts, int n, const int2* __restrict__ child,
                         const int* __restrict__ parent_int, const int* __restrict__ parent_leaf,
                         const int2* __restrict__ range, uint32_t* counters, Node* nodes, int leaf_size) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    float4 p = spts[k];
    float lo[3] = {p.x, p.y, p.z}, hi[3] = {p.x, p.y, p.z};
    float wm = p.w;
    uint32_t ref = leaf_ref((uint32_t)k, 1u);
    int cur = ~k;
    int par = parent_leaf[k];
    // a radix tree over 64-bit codes made unique by 32-bit positions is at
    // most 96 levels deep; the bound only guards against a malformed tree
    for (int depth = 0; par >= 0 && depth < 128; ++depth) {
        int2 ch = child[par];
        int slot = (ch.x == cur) ? 0 : 1;
        NodeChild* dst = &nodes[par].c[slot];
        float4* d4 = reinterpret_cast<float4*>(dst);
        d4[0] = make_float4(lo[0], lo[1], lo[2], wm);
        d4[1] = make_float4(hi[0], hi[1], hi[2], __uint_as_float(ref));
        __threadfence();
        uint32_t old = atomicAdd(&counters[par], 1u);
        if (old == 0) return;
        __threadfence();
        const float* sib = reinterpret_cast<const float*>(&nodes[par].c[1 - slot]);
        for (int c = 0; c < 3; ++c) {
            lo[c] = fminf(lo[c], ld_coherent(sib + c));
            hi[c] = fmaxf(hi[c], ld_coherent(sib + 4 + c));
        }
        wm = fmaxf(wm, ld_coherent(sib + 3));
        int2 r = range[par];
        uint32_t cnt = (uint32_t)(r.y - r.x + 1);
        ref = (cnt <= (uint32_t)leaf_size) ? leaf_ref((uint32_t)r.x, cnt) : (uint32_t)par;
        cur = par;
        par = parent_int[par];
    }
}

hipError_t launch_bounds(const float4* spts, int64_t n, const int2* child, const int* parent_int,
                         const int* parent_leaf, const int2* range, uint32_t* counters, Node* nodes, int leaf_size,
                         hipStream_t s) {
    if (n < 2) return hipSuccess;
    hipLaunchKernelGGL(k_bounds, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, spts, (int)n, child, parent_int,
                       parent_leaf, range, counters, nodes, leaf_size);
    return hipGetLastError();
}

}  // namespace vd
