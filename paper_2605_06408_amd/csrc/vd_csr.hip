// Prefix sums and the CSR write-out.
//
// Cells finish in any order and in Morton order, but the outputs are CSR rows
// in the caller's site order.  The clip kernels therefore stage each cell in a
// fixed-capacity slot and record its counts; an exclusive scan of the counts
// gives the row offsets, and one wave per cell copies its staged record into
// the rows (coalesced: lanes cover consecutive vertices, facets and indices).
#include "vd_internal.h"

namespace vd {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__device__ T block_exclusive_scan(T v, T* total) {
    __shared__ T wsum[kScanThreads / 64 + 1];
    const int ln = threadIdx.x & 63, wv = threadIdx.x >> 6;
    T x = v;
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o);
        if (ln >= o) x += y;
    }
    if (ln == 63) wsum[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        T s = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) {
            T t = wsum[w];
            wsum[w] = s;
            s += t;
        }
        wsum[kScanThreads / 64] = s;
    }
    __syncthreads();
    T excl = x - v + wsum[wv];
    *total = wsum[kScanThreads / 64];
    __syncthreads();
    return excl;
}

template <typename Tin, typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const Tin* __restrict__ in, int64_t n, T* partial) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T s = 0;
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += (T)in[base + k];
    T tot;
    block_exclusive_scan<T>(s, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Exclusive scan of the per-tile totals in place (one block); partial[nblk] = total.
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_mid(T* partial, int64_t nblk) {
    T carry = 0;
    for (int64_t base = 0; base < nblk; base += kScanTile) {
        int64_t b0 = base + (int64_t)threadIdx.x * kScanItems;
        T v[kScanItems];
        T s = 0;
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = (b0 + k < nblk) ? partial[b0 + k] : (T)0;
            s += v[k];
        }
        T tot;
        T e = block_exclusive_scan<T>(s, &tot) + carry;
        for (int k = 0; k < kScanItems; ++k) {
            if (b0 + k < nblk) partial[b0 + k] = e;
            e += v[k];
        }
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[nblk] = carry;
}

template <typename Tin, typename Tout, typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_final(const Tin* __restrict__ in, int64_t n,
                                                             const T* __restrict__ partial, Tout* out,
                                                             int write_total) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    Tin v[kScanItems];
    T s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : (Tin)0;
        s += (T)v[k];
    }
    T tot;
    T e = block_exclusive_scan<T>(s, &tot) + partial[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = (Tout)e;
        e += (T)v[k];
    }
    if (write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = (Tout)partial[gridDim.x];
}

size_t scan_tmp_size(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 2; }

hipError_t scan_counts(const uint32_t* in, int64_t n, int64_t* out, int64_t* tmp, hipStream_t s) {
    int64_t nblk = (n + kScanTile - 1) / kScanTile;
    if (nblk < 1) nblk = 1;
    hipLaunchKernelGGL((k_scan_reduce<uint32_t, int64_t>), dim3((unsigned)nblk), dim3(kScanThreads), 0, s, in, n, tmp);
    hipLaunchKernelGGL((k_scan_mid<int64_t>), dim3(1), dim3(kScanThreads), 0, s, tmp, nblk);
    hipLaunchKernelGGL((k_scan_final<uint32_t, int64_t, int64_t>), dim3((unsigned)nblk), dim3(kScanThreads), 0, s, in,
                       n, tmp, out, 1);
    return hipGetLastError();
}

hipError_t scan_u32(const uint32_t* in, int64_t n, uint32_t* out, uint32_t* tmp, hipStream_t s) {
    int64_t nblk = (n + kScanTile - 1) / kScanTile;
    if (nblk < 1) nblk = 1;
    hipLaunchKernelGGL((k_scan_reduce<uint32_t, uint32_t>), dim3((unsigned)nblk), dim3(kScanThreads), 0, s, in, n,
                       tmp);
    hipLaunchKernelGGL((k_scan_mid<uint32_t>), dim3(1), dim3(kScanThreads), 0, s, tmp, nblk);
    hipLaunchKernelGGL((k_scan_final<uint32_t, uint32_t, uint32_t>), dim3((unsigned)nblk), dim3(kScanThreads), 0, s,
                       in, n, tmp, out, 0);
    return hipGetLastError();
}

// ------------------------------------------------------------------ writer

// One group of kWriteLanes lanes per cell, several cells per wave: a cell has
// a few dozen vertices and facets, and each one waits on a short chain of
// dependent loads (its location, then its staged record), so more cells in
// flight per wave is what fills the memory system.
constexpr int kWriteLanes = 16;

__global__ __launch_bounds__(256) void k_write(WriteArgs a) {
    constexpr int LP = kWriteLanes;
    const int ln = threadIdx.x & (LP - 1);
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / LP;
    const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / LP;
    for (int64_t i = grp; i < a.n; i += ngrp) {
        const uint32_t k = a.inv[i];
        const uint32_t loc = a.loc[k];
        const uint32_t tier = loc >> 30;
        const Stage st = tier == 0 ? a.stage[0] : (tier == 1 ? a.stage[1] : (tier == 2 ? a.stage[2] : a.stage[3]));
        const int64_t slot = loc & 0x3FFFFFFFu;
        const int cap = st.cap;
        const float4* V = st.vert + slot * cap;
        const int32_t* C = st.code + slot * cap;
        const uint16_t* FS = st.fsize + slot * cap;
        const uint16_t* FV = st.fv + slot * 3 * cap;
        const int nv = (int)a.cnt_v[i], nf = (int)a.cnt_f[i], nn = (int)a.cnt_n[i];
        const int64_t vo = a.off_v[i], fo = a.off_f[i], no = a.off_n[i];
        for (int v = ln; v < nv; v += LP) {
            float4 q = V[v];
            uint32_t tri = __float_as_uint(q.w);
            if (a.vert) {
                a.vert[3 * (vo + v)] = q.x;
                a.vert[3 * (vo + v) + 1] = q.y;
                a.vert[3 * (vo + v) + 2] = q.z;
            }
            if (a.vert_planes) {
                uint32_t r0 = tri & 1023u, r1 = (tri >> 10) & 1023u, r2 = (tri >> 20) & 1023u;
                if (st.tri64) {
                    const uint64_t t = st.tri64[slot * cap + v];
                    r0 = (uint32_t)(t & 0x1FFFFFu);
                    r1 = (uint32_t)((t >> 21) & 0x1FFFFFu);
                    r2 = (uint32_t)((t >> 42) & 0x1FFFFFu);
                }
                a.vert_planes[3 * (vo + v)] = C[r0];
                a.vert_planes[3 * (vo + v) + 1] = C[r1];
                a.vert_planes[3 * (vo + v) + 2] = C[r2];
            }
        }
        const int nbox = nf - nn;
        int64_t carry = 3 * vo;
        for (int f0 = 0; f0 < nf; f0 += LP) {
            int f = f0 + ln;
            int32_t code = f < nf ? C[f] : 0;
            int64_t sz = f < nf ? (int64_t)FS[f] : 0;
            int64_t x = sz;
            for (int o = 1; o < LP; o <<= 1) {
                int64_t y = __shfl_up(x, o, LP);
                if (ln >= o) x += y;
            }
            if (f < nf) {
                if (a.facet_nbr) a.facet_nbr[fo + f] = code;
                if (a.fv_off) a.fv_off[fo + f] = carry + x - sz;
                if (a.nbr && f >= nbox) a.nbr[no + (f - nbox)] = code;
            }
            carry += __shfl(x, LP - 1, LP);
        }
        if (a.fv)
            for (int t = ln; t < 3 * nv; t += LP) a.fv[3 * vo + t] = (int32_t)(vo + FV[t]);
    }
}

hipError_t launch_write(const WriteArgs& a, hipStream_t s) {
    const int64_t groups = a.n < 4 * 65536 ? a.n : 4 * 65536;
    int64_t blocks = (groups * kWriteLanes + 255) / 256;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_write, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ dual
// The power diagram's dual is the regular triangulation of the weighted sites
// (Sec. 3): each diagram vertex inside the box, where the cell of site i
// meets three site facets j < k < l, is the centre of the tetrahedron
// (i, j, k, l).  It is a vertex of those four cells; the cell of the smallest
// of the four sites lists it.  One wave per cell, lanes over its vertices.
__device__ __forceinline__ bool tet_row(const Stage& st, int64_t slot, int v, int64_t i, int32_t* c) {
    const uint32_t tri = __float_as_uint(st.vert[slot * st.cap + v].w);
    uint32_t r0 = tri & 1023u, r1 = (tri >> 10) & 1023u, r2 = (tri >> 20) & 1023u;
    if (st.tri64) {
        const uint64_t t = st.tri64[slot * st.cap + v];
        r0 = (uint32_t)(t & 0x1FFFFFu);
        r1 = (uint32_t)((t >> 21) & 0x1FFFFFu);
        r2 = (uint32_t)((t >> 42) & 0x1FFFFFu);
    }
    const int32_t* C = st.code + slot * st.cap;
    c[0] = C[r0];
    c[1] = C[r1];
    c[2] = C[r2];
    return c[0] > i;  // codes ascend: the smallest is a site above i, so are all
}

template <bool kWrite>
__global__ __launch_bounds__(256) void k_tets(TetArgs a) {
    const int ln = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = wave; i < a.n; i += nwaves) {
        const uint32_t loc = a.loc[a.inv[i]];
        const uint32_t tier = loc >> 30;
        const Stage st = tier == 0 ? a.stage[0] : (tier == 1 ? a.stage[1] : (tier == 2 ? a.stage[2] : a.stage[3]));
        const int64_t slot = loc & 0x3FFFFFFFu;
        const int nv = (int)a.cnt_v[i];
        int64_t pos = kWrite ? a.off_t[i] : 0;
        for (int v0 = 0; v0 < nv; v0 += 64) {
            const int v = v0 + ln;
            int32_t c[3] = {0, 0, 0};
            const bool t = v < nv && tet_row(st, slot, v, i, c);
            const uint64_t m = __ballot(t);
            if (kWrite && t) {
                int32_t* row = a.tets + 4 * (pos + (int64_t)__builtin_amdgcn_mbcnt_hi(
                                                         (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u)));
                row[0] = (int32_t)i;
                row[1] = c[0];
                row[2] = c[1];
                row[3] = c[2];
            }
            pos += __popcll(m);
        }
        if (!kWrite && ln == 0) a.cnt_t[i] = (uint32_t)pos;
    }
}

static int64_t tet_blocks(int64_t n) {
    int64_t waves = n < 65536 ? n : 65536;
    int64_t blocks = (waves * 64 + 255) / 256;
    return blocks < 1 ? 1 : blocks;
}

hipError_t launch_tet_count(const TetArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_tets<false>, dim3((unsigned)tet_blocks(a.n)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tet_write(const TetArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_tets<true>, dim3((unsigned)tet_blocks(a.n)), dim3(256), 0, s, a);
    return hipGetLastError();
}

__global__ void k_set_i64(int64_t* dst, int64_t value) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = value;
}

hipError_t launch_set_i64(int64_t* dst, int64_t value, hipStream_t s) {
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, s, dst, value);
    return hipGetLastError();
}

}  // namespace vd
