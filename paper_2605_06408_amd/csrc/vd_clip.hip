// Per-site traversal and clipping: the hot loop of the method.
//
// What is computed (paper Sec. 4, Alg. 1, supplementary Sec. B): for every
// site p_i the cell starts as the clip box and is cut by the half-spaces
// a.y <= b (frame centred on p_i, a = p_j - p_i, b = (|a|^2 + w_i - w_j)/2)
// of candidate sites.  Candidates come from a best-first walk of the BVH:
// a node is skipped when the lower bound on the plane distance of any site
// in it (Sec. 4.2.2: d/2 + min(0, w_i - w_max)/(2d), d = distance from p_i
// to the node box) exceeds the directional radius of the cell toward the
// node (Sec. 4.2.1: distance from p_i to the far corner of the cell's AABB
// in each octant the node occupies); a site in a leaf is skipped when its
// plane distance b/|a| exceeds the directional radius of its own octant.
// Far children are queued with their bound as key, the minimum is popped and
// re-tested against the shrunken cell (Alg. 1).
//
// How it maps to CDNA4: one 64-wide wavefront owns one cell.  Vertex v lives
// in lane v % 64, slot v / 64: its position, the three planes meeting there,
// ordered so that their outward normals have a positive determinant, and the
// three vertices across its edges (edge k is the one that leaves plane k).
// Classifying all vertices against a plane is one ballot per slot; the hole
// left by removed vertices is closed by one new vertex per crossing edge
// (supplementary Sec. B): a kept vertex with a removed neighbour across edge
// k = (planes p_k+1, p_k+2) spawns the vertex (h, p_k+2, p_k+1), and new
// vertices find each other through two tables keyed by their old planes.  The
// node queue is spread one entry per lane (min-pop is a wave reduction), node
// children are tested by two lanes at once, and a leaf's sites by one lane
// each.
//
// Capacity tiers: 64 vertices (one slot; vertex state in registers, planes
// and tables in LDS), 128 (two slots, same layout), 1024 (16 slots; every
// per-cell array in LDS) and 16384 (256 slots; every per-cell array in an
// arena in global memory).  In the last two a workgroup of several waves
// builds one cell: the waves split every loop over vertex slots, combine
// their partial results through LDS (one barrier per exchange) and repeat
// the cell-wide control flow in step, so the few very large cells, which
// set the latency of the whole build, get many waves each; the node queue
// and the cell's final record belong to the first wave.  A cell that
// outgrows a tier is handed to the next.  The paper's own kernel keeps one cell per thread in
// global memory; that layout was made for its GPUs and is not used.
#include <type_traits>

#include "vd_internal.h"

// The slot loops are written once for every tier and marked for unrolling,
// which the register tiers need (their vertex state is indexed by slot); in
// the memory tiers their bounds are run-time values and they stay loops.
#pragma clang diagnostic ignored "-Wpass-failed"

namespace vd {
namespace {

// node queue of the 64-vertex pass: kQueue0 entries, the first 64 in
// registers (one per lane), the rest in LDS and touched only when the queue
// is that long.  With one entry per vertex slot (64), cells of far-reaching
// power cells and of sparse regions next to dense ones filled the queue long
// before their vertex slots and went to the slower second pass.
constexpr int kQueue0 = 256;

constexpr float kU = 5.9604645e-08f;  // FP32 unit roundoff 2^-24
constexpr double kU64 = 1.1102230246251565e-16;

// The launch arguments seen through a pointer the compiler cannot keep
// constant: the fields used once per cell (outputs, lists, counters) are then
// loaded where they are used instead of being held in scalar registers
// across the hot loops, which otherwise run out of them and spill.  Every
// clip kernel takes its ClipArgs as the first kernel argument.
using KArgs = const __attribute__((address_space(4))) ClipArgs;
__device__ __forceinline__ KArgs* cold_args() {
    KArgs* p = (KArgs*)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return p;
}

enum ClipResult { kNone = 0, kChanged = 1, kEmptied = 2, kOverflow = 3, kRestart = 4 };

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ int popc(uint64_t m) { return __popcll(m); }
__device__ __forceinline__ int lowest(uint64_t m) { return __builtin_ctzll(m); }
__device__ __forceinline__ float rdl(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ uint32_t rdl(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }
__device__ __forceinline__ int rdl(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
// Wave reductions by DPP lane moves (no LDS round trip): within quads
// (quad_perm [1,0,3,2] and [2,3,0,1]), across half-rows and rows
// (row_half_mirror, row_mirror), then row 0 into 1 and 2 into 3
// (row_bcast:15) and rows 0-1 into 2-3 (row_bcast:31); lane 63 holds the
// result, which is returned to every lane.  All 64 lanes must be active.
// dpp: lanes of rows the move does not write get `keep` (the identity of
// the sum it feeds).
template <int kCtrl, int kRows>
__device__ __forceinline__ int dpp(int keep, int v) {
    return __builtin_amdgcn_update_dpp(keep, v, kCtrl, kRows, 0xF, false);
}
// A move within rows (every lane reads a lane of its own row, so all reads
// are valid): the compiler can fold it into the operation that uses it.
template <int kCtrl>
__device__ __forceinline__ int dpp_row(int v) {
    return __builtin_amdgcn_mov_dpp(v, kCtrl, 0xF, 0xF, true);
}
// The two row broadcasts write only rows 1, 3 and then 2, 3; what the
// other rows then hold never reaches lane 63, so they need no defined value.
template <int kCtrl, int kRows>
__device__ __forceinline__ int dpp_bcast(int v) {
    return __builtin_amdgcn_mov_dpp(v, kCtrl, kRows, 0xF, false);
}
template <typename Op>
__device__ __forceinline__ int wave_reduce_i(int v, Op op) {
    v = op(v, dpp_row<0xB1>(v));
    v = op(v, dpp_row<0x4E>(v));
    v = op(v, dpp_row<0x141>(v));
    v = op(v, dpp_row<0x140>(v));
    v = op(v, dpp_bcast<0x142, 0xA>(v));
    v = op(v, dpp_bcast<0x143, 0xC>(v));
    return __builtin_amdgcn_readlane(v, 63);
}
// Float min and max reduce as integers: the bits of a float with the
// magnitude bits of negative values flipped order like the values (NaN is
// never reduced), so each step is one integer min or max on a lane move,
// with no float canonicalisation between the steps.
__device__ __forceinline__ int ford(float f) {
    const int i = __float_as_int(f);
    return i ^ ((i >> 31) & 0x7FFFFFFF);
}
__device__ __forceinline__ float unford(int k) { return __int_as_float(k ^ ((k >> 31) & 0x7FFFFFFF)); }
// Maximum of two non-negative floats (their bits order like integers).
__device__ __forceinline__ float pmax(float a, float b) {
    return __int_as_float(max(__float_as_int(a), __float_as_int(b)));
}
__device__ __forceinline__ float wmin(float v) {
    return unford(wave_reduce_i(ford(v), [](int a, int b) { return min(a, b); }));
}
__device__ __forceinline__ float wmax(float v) {
    return unford(wave_reduce_i(ford(v), [](int a, int b) { return max(a, b); }));
}
__device__ __forceinline__ uint64_t wor64(uint64_t v) {
    auto op = [](int a, int b) { return a | b; };
    const uint32_t lo = (uint32_t)wave_reduce_i((int)(uint32_t)v, op);
    const uint32_t hi = (uint32_t)wave_reduce_i((int)(uint32_t)(v >> 32), op);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}
__device__ __forceinline__ uint32_t wsum_u(uint32_t v) {
    return (uint32_t)wave_reduce_i((int)v, [](int a, int b) { return (int)((uint32_t)a + (uint32_t)b); });
}
template <int kCtrl, int kRows>
__device__ __forceinline__ double dpp64(double v) {
    const int lo = dpp<kCtrl, kRows>(0, __double2loint(v));
    const int hi = dpp<kCtrl, kRows>(0, __double2hiint(v));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wsum64(double v) {
    v += dpp64<0xB1, 0xF>(v);
    v += dpp64<0x4E, 0xF>(v);
    v += dpp64<0x141, 0xF>(v);
    v += dpp64<0x140, 0xF>(v);
    v += dpp64<0x142, 0xA>(v);
    v += dpp64<0x143, 0xC>(v);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Sizes and index packings of a tier.  Three vertex or plane indices are
// packed into one word: 10 bits each in 32-bit words up to 1024 vertices,
// 15 bits each in 64-bit words above.
template <int VPL>
struct Tier {
    static constexpr int CAP = 64 * VPL;
    static constexpr bool kReg = VPL <= 4;  // vertex state in registers, slot loops unrolled
    static constexpr bool kNarrow = CAP <= 1024;
    static constexpr int kB = kNarrow ? 10 : 15;
    using W = typename std::conditional<kNarrow, uint32_t, uint64_t>::type;
    static constexpr W kMask = (W(1) << kB) - 1;
    // new-vertex table entries: serial tag above the vertex index
    static constexpr int kTagShift = kNarrow ? 12 : 16;
    static constexpr uint32_t kTagMax = (1u << (32 - kTagShift)) - 2u;
    __device__ __forceinline__ static uint32_t fld(W w, int k) { return (uint32_t)((w >> (kB * k)) & kMask); }
    __device__ __forceinline__ static W setfld(W w, int k, uint32_t v) {
        return (w & ~(kMask << (kB * k))) | (W(v) << (kB * k));
    }
    __device__ __forceinline__ static W pack3(uint32_t a, uint32_t b, uint32_t c) {
        return W(a) | (W(b) << kB) | (W(c) << (2 * kB));
    }
};

// Orders this wave's accesses to its per-cell arrays, so that what one lane
// wrote before is seen by every lane after: LDS (one wave, no workgroup
// barrier needed) or, for the arena tier, global memory (one wave per
// workgroup).
template <bool kLds>
__device__ __forceinline__ void wave_sync() {
    if constexpr (kLds) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
}

// Per-slot values of one lane: a register array in the register tiers, a
// column of an arena array otherwise (element s at m[s * kStride]; stride 64
// for per-lane values, 1 for wave-uniform ones).
template <typename X, int N, bool kReg, int kStride>
struct Col {
    X r[kReg ? N : 1];
    X* m = nullptr;
    __device__ __forceinline__ X& operator[](int s) {
        if constexpr (kReg) return r[s];
        else return m[s * kStride];
    }
};

// Per-cell state that the register tiers keep in registers and the larger
// tiers in LDS or the arena (index slot * 64 + lane for per-lane values, slot
// for wave-uniform masks).
template <int VPL, bool kArena = !Tier<VPL>::kReg>
struct ArenaState {};
template <int VPL>
struct ArenaState<VPL, true> {
    using W = typename Tier<VPL>::W;
    static constexpr int CAP = Tier<VPL>::CAP;
    float y0[CAP], y1[CAP], y2[CAP], ev[CAP];  // vertex positions and error scales
    W vt[CAP], va[CAP];                         // vertex planes and neighbours
    uint32_t qe[CAP];                           // node queue
    float qk[CAP];
    uint32_t cross[CAP], pre[CAP], frank[CAP], nb1[CAP], nb2[CAP];  // clip temporaries
    W rec[CAP];
    uint8_t isnew[CAP], amb[CAP];
    uint64_t alive[VPL], R[VPL], fr[VPL];  // per-slot masks
};

// queue entries of the 64-vertex pass beyond the first 64
template <int VPL>
struct QueueExt {};
template <>
struct QueueExt<1> {
    uint32_t qxe[kQueue0 - 64];
    float qxk[kQueue0 - 64];
};
template <>
struct QueueExt<2> {
    uint32_t qxe[kQueue0 - 128];
    float qxk[kQueue0 - 128];
};
// queue capacity of the pass of vertex capacity cap
constexpr int queue_cap(int cap) { return cap < kQueue0 ? kQueue0 : cap; }

template <int VPL>
struct WaveMem : ArenaState<VPL>, QueueExt<VPL> {
    using W = typename Tier<VPL>::W;
    static constexpr int CAP = Tier<VPL>::CAP;
    float4 pl[CAP];        // planes: a.xyz, b (frame of the site)
    float psb[CAP];        // size of the terms b is formed from (error scale)
    float4 psite[CAP];     // the plane's site (x, y, z, w) for exact re-evaluation
    int32_t pcode[CAP];    // Morton index of the plane's site, or box code -1..-6
    uint32_t ta[CAP];      // clip: new vertex by first old plane | finalize: plane rank
    uint32_t tb[CAP];      // clip: new vertex by second old plane | finalize: facet size
    uint32_t sor[CAP];     // clip: free slot of rank | finalize: vertex renumbering
    uint32_t anchor[CAP];  // finalize: lowest vertex of each facet
    W edge[CAP];           // clip: crossing edges by rank
    W vtri[CAP];           // finalize: planes of each vertex
    W vadj[CAP];           // finalize: neighbours of each vertex
    double vpx[CAP], vpy[CAP], vpz[CAP];  // finalize: FP64 positions relative to vertex 0
    int32_t key[CAP];      // finalize and gc: output codes, used flags
    uint8_t outf[CAP];     // outside flags by vertex index (VPL > 1)
};

// A plane in FP64, recomputed from the input coordinates.
struct P64 {
    double a0, a1, a2, b;
};

// kLds: the per-cell arrays are in LDS (else in global memory).  kCount:
// count work units and cycles (a separate instantiation, so the timed
// kernels carry no counting code).  G: waves building the cell together
// (one in the register tiers).  kSoS: exact ties decided by the symbolic
// perturbation (its own instantiation: the checked exact evaluation would
// otherwise cost the default kernels registers).  kW: the sites carry
// weights; kOpt: the search options (culling, traversal order, warm start)
// are read at run time.  The 64- and 128-vertex passes of a build with the
// default options run instantiations with those options fixed, and for an
// unweighted build without the weight terms of the bounds and ball tests
// (every weight is zero there): the same results bit for bit, 4% less time
// for the fixed options (their checks and the scalar registers they held)
// and 2.5% for the weight terms.  Every wave of a group
// holds the same copy of the cell-wide scalars (site, bounds, plane and
// queue counts, flags) and changes it the same way, from values every wave
// has seen.
// Every member of Cell and the work loop are inlined into their kernel: as
// calls (the inliner's size limits give up on the larger instantiations)
// they cost a stack frame in scratch memory and spills around each call.
#pragma clang attribute push(__attribute__((always_inline)), apply_to = function)
template <int VPL, bool kLds, bool kCount, int G = 1, bool kSoS = false, bool kW = true, bool kOpt = true>
struct Cell {
    static_assert(G == 1 || !Tier<VPL>::kReg, "wave groups need the vertex state in memory");
    using T = Tier<VPL>;
    using W = typename T::W;
    static constexpr int CAP = T::CAP;
    static constexpr bool kReg = T::kReg;
    // hand-over: every pass but the last writes the state of the cells it
    // escalates; every pass but the first can take over such a state (from
    // the pass of capacity kPrevCap)
    static constexpr bool kSaves = CAP < kTierCap[kTiers - 1];
    static constexpr int kPrevCap = CAP == kTierCap[1] ? kTierCap[0]
                                    : (CAP == kTierCap[2] ? kTierCap[1] : (CAP == kTierCap[3] ? kTierCap[2] : 0));
    static constexpr bool kResumes = kPrevCap > 0;
    // queue capacity: one entry per vertex, but kQueue0 in the 64-vertex pass
    static constexpr bool kQExt = kReg && 64 * VPL < kQueue0;  // queue entries beyond the slots in LDS
    static constexpr int QCAP = queue_cap(CAP);
    static constexpr int kPrevQ = kPrevCap > 0 ? queue_cap(kPrevCap) : 64;
    using HIn = HandoffT<(kPrevCap > 0 ? kPrevCap : 64), (kPrevCap > 0 ? kPrevQ : 64)>;
    using HOut = HandoffT<(kSaves ? CAP : 64), (kSaves ? QCAP : 64)>;
    template <typename X>
    using Lane = Col<X, VPL, kReg, 64>;  // one value per slot of this lane
    template <typename X>
    using Wave = Col<X, VPL, kReg, 1>;   // one wave-uniform value per slot
    WaveMem<VPL>& M;
    const ClipArgs& A;
    const uint32_t ln;
    const uint32_t wid;  // wave of the group
    uint32_t* gx;        // group exchange tables in LDS: 2 x G x 8 words
    int gpar;            // table of the next exchange
    uint32_t serial;
    // site
    float px, py, pz, pw;
    // the site's weight where the arithmetic uses it (zero without weights)
    __device__ __forceinline__ float pwv() const { if constexpr (kW) return pw; else return 0.f; }
    // search options: the default instantiations fix them (directional plus
    // ball culling, best-first order, no warm start)
    __device__ __forceinline__ int culling() const { if constexpr (kOpt) return A.culling; else return 3; }
    __device__ __forceinline__ int traversal() const { if constexpr (kOpt) return A.traversal; else return 1; }
    __device__ __forceinline__ int warm_start() const { if constexpr (kOpt) return A.warm_start; else return 0; }
    uint32_t self;
    uint32_t flags;
    int robust;   // 0: FP32 signs; 1: doubtful signs in FP64; 2: every sign in FP64
    // vertices: slot s of this lane is vertex s*64 + lane
    Lane<float> y0, y1, y2, ev;
    Lane<W> vt, va;
    Wave<uint64_t> alive;
    int np;
    int vhi;  // one past the highest vertex index used since init
    // bounds of the current cell (uniform): AABB in the site's frame, the
    // squared far-corner coordinates, the directional and isotropic radii
    float blo0, blo1, blo2, bhi0, bhi1, bhi2;
    float hx2, hy2, hz2, lx2, ly2, lz2, rmax2, riso2;
    // 64-vertex pass: the vertex at each side of the AABB (min x, y, z, max
    // x, y, z) and the vertices the last effective clip removed; a clip that
    // removes none of the six leaves the AABB as it was (new vertices lie on
    // edges of the old cell)
    uint32_t ext[6];
    uint64_t cut_mask;
    // queue (entry q in lane q % 64, slot q / 64; in the 64-vertex pass entries
    // from 64 on are in LDS, M.qxe / M.qxk)
    Lane<uint32_t> qe;
    Lane<float> qk;
    int qn;
    // KNN warm start: the sites already clipped (Morton positions), lane t
    // holding the t-th; the leaves of the walk pass over them
    int nwarm;
    uint32_t wsite;
    // where the last capacity overflow struck: in leaf ov_leaf, with the
    // candidates ov_mask still to try (ov_ok), else somewhere not resumable
    bool ov_ok;
    uint32_t ov_leaf, ov_phase, ov_skip;
    uint64_t ov_mask;
    uint32_t leaf_phase = 1;  // 0 while clipping by the site's own leaf before any walk
    // work counters (uniform), accumulated over all cells of this wave
    uint64_t ctr[kCount ? kCtrCount : 1];
    static constexpr bool counting = kCount;

    // the first clip clears the new-vertex tables (the tag counter starts
    // at its wrap-around value)
    __device__ Cell(WaveMem<VPL>& m, const ClipArgs& a, uint32_t* gxch)
        : M(m), A(a), ln(lane_id()), wid(G > 1 ? (uint32_t)(threadIdx.x >> 6) : 0u), gx(gxch), gpar(0),
          serial(T::kTagMax - 1) {
#pragma unroll
        for (int c = 0; c < (kCount ? kCtrCount : 1); ++c) ctr[c] = 0;
        if constexpr (!kReg) {
            y0.m = M.y0 + ln; y1.m = M.y1 + ln; y2.m = M.y2 + ln; ev.m = M.ev + ln;
            vt.m = M.vt + ln; va.m = M.va + ln;
            alive.m = M.alive;
            qe.m = M.qe + ln; qk.m = M.qk + ln;
        }
        vhi = CAP;
    }
    __device__ __forceinline__ void count(int c, uint64_t v) {
        if constexpr (kCount) ctr[c] += v;
    }
    // elapsed shader clock of this wave, accumulated per phase when counting
    __device__ __forceinline__ uint64_t tic() const {
        if constexpr (kCount) return (uint64_t)clock64();
        else return 0ull;
    }
    __device__ __forceinline__ void toc(int c, uint64_t t0) {
        if constexpr (kCount) ctr[c] += (uint64_t)clock64() - t0;
    }
    // wsync orders this wave's accesses; sync those of the whole group
    __device__ __forceinline__ void wsync() { wave_sync<kLds>(); }
    __device__ __forceinline__ void sync() {
        if constexpr (G > 1) __syncthreads();
        else wave_sync<kLds>();
    }
    // the first wave of the group (the only one without groups)
    __device__ __forceinline__ bool lead() const { return G == 1 || wid == 0; }
    // Group exchange: every wave posts N uniform words; returns the table
    // (word k of wave w at [w * 8 + k]) once all have posted.  The two tables
    // alternate, so one barrier per exchange is enough: a wave writes a table
    // again only after the barrier of the exchange in between, which every
    // wave reaches after reading it.
    template <int N>
    __device__ __forceinline__ const uint32_t* exch(const uint32_t (&v)[N]) {
        static_assert(N <= 8, "eight words per wave");
        uint32_t* t = gx + gpar * (G * 8);
        gpar ^= 1;
        if (ln == 0) {
#pragma unroll
            for (int k = 0; k < N; ++k) t[wid * 8 + k] = v[k];
        }
        __syncthreads();
        return t;
    }
    __device__ __forceinline__ bool g_or(bool x) {
        if constexpr (G == 1) {
            return x;
        } else {
            const uint32_t v[1] = {x ? 1u : 0u};
            const uint32_t* t = exch(v);
            bool r = false;
#pragma unroll
            for (int w = 0; w < G; ++w) r |= t[w * 8] != 0;
            return r;
        }
    }
    // the first wave's value, for every wave of the group
    __device__ __forceinline__ uint32_t bcast(uint32_t x) {
        if constexpr (G == 1) {
            return uni(x);
        } else {
            const uint32_t v[1] = {x};
            return exch(v)[0];
        }
    }
    // Sum over the group of a per-wave count: the total, and in *below the
    // sum over the waves before this one.
    __device__ __forceinline__ uint32_t g_scan(uint32_t x, uint32_t* below) {
        if constexpr (G == 1) {
            *below = 0;
            return x;
        } else {
            const uint32_t v[1] = {x};
            const uint32_t* t = exch(v);
            uint32_t tot = 0, bl = 0;
#pragma unroll
            for (int w = 0; w < G; ++w) {
                const uint32_t c = t[w * 8];
                if (w < (int)wid) bl += c;
                tot += c;
            }
            *below = bl;
            return tot;
        }
    }
    // This wave's share [lo, hi) of n items dealt in runs of u (the last run
    // may reach past n, never past the next multiple of u).
    __device__ __forceinline__ void share(int n, int u, int* lo, int* hi) const {
        if constexpr (G == 1) {
            *lo = 0;
            *hi = n;
        } else {
            const int nu = (n + u - 1) / u;
            *lo = nu * (int)wid / G * u;
            *hi = nu * ((int)wid + 1) / G * u;
        }
    }
    // slots that may hold vertices (all of them in the register tiers)
    __device__ __forceinline__ int nsv() const { return kReg ? VPL : ((vhi + 63) >> 6); }
    __device__ __forceinline__ uint64_t nalive() {
        uint64_t c = 0;
        const int ns = nsv();
#pragma unroll
        for (int s = 0; s < (kReg ? VPL : ns); ++s) c += (uint64_t)popc(alive[s]);
        return c;
    }

    __device__ __forceinline__ bool is_alive(uint32_t u) {
        const int sl = (int)(u >> 6);
        uint64_t al = 0;
        if constexpr (kReg) {
#pragma unroll
            for (int s = 0; s < VPL; ++s)
                if (s == sl) al = alive[s];
        } else {
            if (sl < nsv()) al = alive[sl];
        }
        return (al >> (u & 63)) & 1;
    }

    // ------------------------------------------------------------ setup
    __device__ bool init(uint32_t k) {
        if constexpr (G > 1) sync();  // every wave is done with the previous cell
        self = k;
        float4 s = A.pts[k];
        px = s.x; py = s.y; pz = s.z; pw = s.w;
        flags = 0;
        qn = 0;
        nwarm = 0;
        if (pw == -INFINITY) return false;  // coincident with a heavier site
        const float lo[3] = {A.bbox[0] - px, A.bbox[1] - py, A.bbox[2] - pz};
        const float hi[3] = {A.bbox[3] - px, A.bbox[4] - py, A.bbox[5] - pz};
        if (ln < 6 && lead()) {
            int ax = ln >> 1, side = ln & 1;
            float a[3] = {0.f, 0.f, 0.f};
            a[ax] = side ? 1.f : -1.f;
            float b = side ? hi[ax] : -lo[ax];
            M.pl[ln] = make_float4(a[0], a[1], a[2], b);
            M.psb[ln] = fabsf(b);
            M.pcode[ln] = -(int)(ln + 1);
            M.psite[ln] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        if constexpr (kReg) {
#pragma unroll
            for (int s2 = 0; s2 < VPL; ++s2) alive[s2] = 0;
        }
        // slots above the first are written by a clip before they are read
        if (lead()) alive[0] = 0xFFull;
        vhi = 8;
        if (lead()) {
            uint32_t c = ln & 7;
            uint32_t sx = c & 1, sy = (c >> 1) & 1, sz = (c >> 2) & 1;
            uint32_t X = sx, Y = 2 + sy, Z = 4 + sz;
            bool pos = ((sx ^ sy ^ sz) & 1) == 1;  // product of the three normal signs > 0
            uint32_t p1 = pos ? Y : Z, p2 = pos ? Z : Y;
            uint32_t ax1 = p1 >> 1, ax2 = p2 >> 1;
            vt[0] = T::pack3(X, p1, p2);
            va[0] = T::pack3(c ^ 1u, c ^ (1u << ax1), c ^ (1u << ax2));
            y0[0] = sx ? hi[0] : lo[0];
            y1[0] = sy ? hi[1] : lo[1];
            y2[0] = sz ? hi[2] : lo[2];
            ev[0] = fabsf(y0[0]) + fabsf(y1[0]) + fabsf(y2[0]);
        }
        np = 6;
        sync();
        update_bounds();
        return true;
    }

    // Slots are visited kBatch at a time: in the LDS and arena tiers every
    // load of a batch is issued before any is used (one wait per batch, not
    // per slot); wave groups deal the slots out two at a time, so that a
    // cell of few slots still keeps every wave busy.  Slots at or above ns
    // read as dead (the loads stay in bounds: VPL is a multiple of kBatch).
    static constexpr int kBatch = kReg ? VPL : (G > 1 ? 2 : 4);
    struct VBatch {
        float a[kBatch], b[kBatch], c[kBatch];
        uint64_t al[kBatch];
    };
    __device__ __forceinline__ void load_batch(int s0, int ns, VBatch& v) {
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int s = s0 + k;
            v.a[k] = y0[s];
            v.b[k] = y1[s];
            v.c[k] = y2[s];
            const uint64_t al = alive[s];
            v.al[k] = s < ns ? al : 0ull;
        }
    }

    __device__ void update_bounds() {
        float mn0 = INFINITY, mn1 = INFINITY, mn2 = INFINITY, mx0 = -INFINITY, mx1 = -INFINITY, mx2 = -INFINITY,
              r2 = 0.f;
        const int ns = nsv();
        int lo, hi;
        share(ns, kBatch, &lo, &hi);
        for (int s0 = (kReg ? 0 : lo); s0 < (kReg ? VPL : hi); s0 += kBatch) {
            VBatch v;
            load_batch(s0, ns, v);
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                if ((v.al[k] >> ln) & 1) {
                    const float a = v.a[k], b = v.b[k], c = v.c[k];
                    mn0 = fminf(mn0, a); mn1 = fminf(mn1, b); mn2 = fminf(mn2, c);
                    mx0 = fmaxf(mx0, a); mx1 = fmaxf(mx1, b); mx2 = fmaxf(mx2, c);
                    if (culling() == 2) r2 = fmaxf(r2, fmaf(a, a, fmaf(b, b, c * c)));
                }
            }
        }
        float l0 = wmin(mn0), l1 = wmin(mn1), l2 = wmin(mn2);
        float h0 = wmax(mx0), h1 = wmax(mx1), h2 = wmax(mx2);
        riso2 = culling() == 2 ? wmax(r2) : 0.f;  // the isotropic radius only serves culling mode 2
        if constexpr (G > 1) {
            const uint32_t v[7] = {__float_as_uint(l0), __float_as_uint(l1), __float_as_uint(l2), __float_as_uint(h0),
                                   __float_as_uint(h1), __float_as_uint(h2), __float_as_uint(riso2)};
            const uint32_t* t = exch(v);
            l0 = l1 = l2 = INFINITY;
            h0 = h1 = h2 = -INFINITY;
            riso2 = 0.f;
#pragma unroll
            for (int w = 0; w < G; ++w) {
                const uint32_t* x = t + w * 8;
                l0 = fminf(l0, __uint_as_float(x[0])); l1 = fminf(l1, __uint_as_float(x[1]));
                l2 = fminf(l2, __uint_as_float(x[2]));
                h0 = fmaxf(h0, __uint_as_float(x[3])); h1 = fmaxf(h1, __uint_as_float(x[4]));
                h2 = fmaxf(h2, __uint_as_float(x[5]));
                riso2 = fmaxf(riso2, __uint_as_float(x[6]));
            }
        }
        blo0 = l0; blo1 = l1; blo2 = l2;
        bhi0 = h0; bhi1 = h1; bhi2 = h2;
        if constexpr (VPL == 1 && G == 1) {
            const bool al = (alive[0] >> ln) & 1;
            ext[0] = lowest(ballot(al && y0[0] == l0));
            ext[1] = lowest(ballot(al && y1[0] == l1));
            ext[2] = lowest(ballot(al && y2[0] == l2));
            ext[3] = lowest(ballot(al && y0[0] == h0));
            ext[4] = lowest(ballot(al && y1[0] == h1));
            ext[5] = lowest(ballot(al && y2[0] == h2));
        }
        derive_bounds();
    }
    __device__ __forceinline__ void derive_bounds() {
        hx2 = bhi0 * bhi0; hy2 = bhi1 * bhi1; hz2 = bhi2 * bhi2;
        lx2 = blo0 * blo0; ly2 = blo1 * blo1; lz2 = blo2 * blo2;
        rmax2 = fmaxf(hx2, lx2) + fmaxf(hy2, ly2) + fmaxf(hz2, lz2);
    }
    // After an effective clip: in the 64-vertex pass only the sides whose
    // vertex the clip removed are reduced again.
    __device__ void bounds_after_clip() {
        if constexpr (VPL == 1 && G == 1) {
            if (culling() != 2) {
                uint32_t lost = 0;
#pragma unroll
                for (int k = 0; k < 6; ++k) lost |= (uint32_t)((cut_mask >> ext[k]) & 1ull) << k;
                if (lost == 0) return;
                const bool al = (alive[0] >> ln) & 1;
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    if ((lost >> k) & 1u) {
                        const float v = (k % 3 == 0) ? y0[0] : ((k % 3 == 1) ? y1[0] : y2[0]);
                        const float m = k < 3 ? wmin(al ? v : INFINITY) : wmax(al ? v : -INFINITY);
                        ext[k] = lowest(ballot(al && v == m));
                        if (k == 0) blo0 = m; else if (k == 1) blo1 = m; else if (k == 2) blo2 = m;
                        else if (k == 3) bhi0 = m; else if (k == 4) bhi1 = m; else bhi2 = m;
                    }
                }
                derive_bounds();
                return;
            }
        }
        update_bounds();
    }

    // Squared radius of the cell toward direction a (far AABB corner of the
    // octant of a; zero components count as positive).
    __device__ __forceinline__ float radius2_toward(float ax, float ay, float az) const {
        if (culling() == 2) return riso2;
        return (ax >= 0.f ? hx2 : lx2) + (ay >= 0.f ? hy2 : ly2) + (az >= 0.f ? hz2 : lz2);
    }

    // Power-ball test of a node box (frame of the site): a site p_j in the box
    // with w_j <= wmax cuts the cell only if some vertex v has
    // |v - p_j|^2 - w_j < |v|^2 - w_i, and |v - p_j|^2 >= dist(v, box)^2.
    // Returns true if some vertex might be cut (the box cannot be skipped).
    __device__ bool ball_hit(float lx, float ly, float lz, float hx, float hy, float hz, float wm) {
        if constexpr (kCount) count(kCtrBall, nalive());
        bool hit = false;
        const int ns = nsv();
        int lo, hi;
        share(ns, kBatch, &lo, &hi);
        for (int s0 = (kReg ? 0 : lo); s0 < (kReg ? VPL : hi); s0 += kBatch) {
            VBatch v;
            load_batch(s0, ns, v);
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                if ((v.al[k] >> ln) & 1) {
                    const float a = v.a[k], b = v.b[k], c = v.c[k];
                    float dx = fmaxf(fmaxf(lx - a, a - hx), 0.f);
                    float dy = fmaxf(fmaxf(ly - b, b - hy), 0.f);
                    float dz = fmaxf(fmaxf(lz - c, c - hz), 0.f);
                    float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    float r2 = fmaf(a, a, fmaf(b, b, c * c));
                    float lhs = d2 - wm, rhs = r2 - pwv();
                    hit |= lhs - rhs <= 16.f * kU * (d2 + r2 + fabsf(wm) + fabsf(pwv()));
                }
            }
        }
        return g_or(ballot(hit) != 0);
    }

    // The ball test of both child records (lanes 0 and 1) in one pass over
    // the vertices (the vertex's own power is shared by the two boxes).
    __device__ void ball_hit_pair(const NodeChild& c, bool* hit0, bool* hit1) {
        if constexpr (kCount) count(kCtrBall, 2 * nalive());
        const float blx = c.lo[0] - px, bly = c.lo[1] - py, blz = c.lo[2] - pz;
        const float bhx = c.hi[0] - px, bhy = c.hi[1] - py, bhz = c.hi[2] - pz;
        const float l0x = rdl(blx, 0), l0y = rdl(bly, 0), l0z = rdl(blz, 0);
        const float h0x = rdl(bhx, 0), h0y = rdl(bhy, 0), h0z = rdl(bhz, 0), w0 = kW ? rdl(c.wmax, 0) : 0.f;
        const float l1x = rdl(blx, 1), l1y = rdl(bly, 1), l1z = rdl(blz, 1);
        const float h1x = rdl(bhx, 1), h1y = rdl(bhy, 1), h1z = rdl(bhz, 1), w1 = kW ? rdl(c.wmax, 1) : 0.f;
        bool a0 = false, a1 = false;
        const int ns = nsv();
        int lo, hi;
        share(ns, kBatch, &lo, &hi);
        for (int s0 = (kReg ? 0 : lo); s0 < (kReg ? VPL : hi); s0 += kBatch) {
            VBatch v;
            load_batch(s0, ns, v);
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                if ((v.al[k] >> ln) & 1) {
                    const float a = v.a[k], b = v.b[k], cc = v.c[k];
                    const float r2 = fmaf(a, a, fmaf(b, b, cc * cc)), rhs = r2 - pwv(), tol = r2 + fabsf(pwv());
                    float dx = fmaxf(fmaxf(l0x - a, a - h0x), 0.f);
                    float dy = fmaxf(fmaxf(l0y - b, b - h0y), 0.f);
                    float dz = fmaxf(fmaxf(l0z - cc, cc - h0z), 0.f);
                    float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    a0 |= (d2 - w0) - rhs <= 16.f * kU * (d2 + tol + fabsf(w0));
                    dx = fmaxf(fmaxf(l1x - a, a - h1x), 0.f);
                    dy = fmaxf(fmaxf(l1y - b, b - h1y), 0.f);
                    dz = fmaxf(fmaxf(l1z - cc, cc - h1z), 0.f);
                    d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    a1 |= (d2 - w1) - rhs <= 16.f * kU * (d2 + tol + fabsf(w1));
                }
            }
        }
        bool r0 = ballot(a0) != 0, r1 = ballot(a1) != 0;
        if constexpr (G > 1) {
            const uint32_t v2[2] = {r0 ? 1u : 0u, r1 ? 1u : 0u};
            const uint32_t* t = exch(v2);
            r0 = r1 = false;
#pragma unroll
            for (int w = 0; w < G; ++w) {
                r0 |= t[w * 8] != 0;
                r1 |= t[w * 8 + 1] != 0;
            }
        }
        *hit0 = r0;
        *hit1 = r1;
    }

    // Applies the ball test to the child record held by lane `l`.
    __device__ bool ball_hit_lane(const NodeChild& c, int l) {
        float lx = rdl(c.lo[0] - px, l), ly = rdl(c.lo[1] - py, l), lz = rdl(c.lo[2] - pz, l);
        float hx = rdl(c.hi[0] - px, l), hy = rdl(c.hi[1] - py, l), hz = rdl(c.hi[2] - pz, l);
        float wm = kW ? rdl(c.wmax, l) : 0.f;
        return ball_hit(lx, ly, lz, hx, hy, hz, wm);
    }

    // ------------------------------------------------------------ FP64 side test
    // Plane q in FP64, recomputed from the input coordinates: a = p_j - p_i
    // is exact in FP64, b = (|a|^2 + w_i - w_j) / 2 nearly so.
    __device__ P64 plane64(uint32_t q) const { return plane64(M.pcode[q], M.psite[q]); }

    __device__ P64 plane64(int32_t code, float4 site) const {
        P64 r;
        const double qx = px, qy = py, qz = pz, qw = pw;
        if (code < 0) {
            int c = -code - 1, ax = c >> 1, side = c & 1;
            double p[3] = {qx, qy, qz};
            r.a0 = r.a1 = r.a2 = 0.0;
            double sgn = side ? 1.0 : -1.0;
            if (ax == 0) r.a0 = sgn; else if (ax == 1) r.a1 = sgn; else r.a2 = sgn;
            r.b = side ? ((double)A.bbox[3 + ax] - p[ax]) : (p[ax] - (double)A.bbox[ax]);
        } else {
            r.a0 = (double)site.x - qx; r.a1 = (double)site.y - qy; r.a2 = (double)site.z - qz;
            r.b = 0.5 * (r.a0 * r.a0 + r.a1 * r.a1 + r.a2 * r.a2 + (qw - (double)site.w));
        }
        return r;
    }

    // Intersection of three FP64 planes: numerator n and determinant (y = n / det).
    __device__ static void cramer64(const P64& A0, const P64& B0, const P64& C0, double* n, double* det) {
        double bc0 = B0.a1 * C0.a2 - B0.a2 * C0.a1, bc1 = B0.a2 * C0.a0 - B0.a0 * C0.a2,
               bc2 = B0.a0 * C0.a1 - B0.a1 * C0.a0;
        double ca0 = C0.a1 * A0.a2 - C0.a2 * A0.a1, ca1 = C0.a2 * A0.a0 - C0.a0 * A0.a2,
               ca2 = C0.a0 * A0.a1 - C0.a1 * A0.a0;
        double ab0 = A0.a1 * B0.a2 - A0.a2 * B0.a1, ab1 = A0.a2 * B0.a0 - A0.a0 * B0.a2,
               ab2 = A0.a0 * B0.a1 - A0.a1 * B0.a0;
        *det = A0.a0 * bc0 + A0.a1 * bc1 + A0.a2 * bc2;
        n[0] = A0.b * bc0 + B0.b * ca0 + C0.b * ab0;
        n[1] = A0.b * bc1 + B0.b * ca1 + C0.b * ab1;
        n[2] = A0.b * bc2 + B0.b * ca2 + C0.b * ab2;
    }

    // Side of the vertex with planes t w.r.t. plane h, recomputed in FP64 from
    // the input coordinates.  Returns +1 outside, -1 inside, 0 undecided.
    __device__ int side64(W t, const P64& h) const {
        double n[3], det;
        cramer64(plane64(T::fld(t, 0)), plane64(T::fld(t, 1)), plane64(T::fld(t, 2)), n, &det);
        // s * det = a_h . n - b_h det, evaluated without dividing
        double s = h.a0 * n[0] + h.a1 * n[1] + h.a2 * n[2] - h.b * det;
        if (det < 0) s = -s;
        double scale = (fabs(h.a0) + fabs(h.a1) + fabs(h.a2)) * (fabs(n[0]) + fabs(n[1]) + fabs(n[2])) +
                       fabs(h.b * det);
        if (fabs(s) <= 64.0 * kU64 * scale) return 0;
        return s > 0 ? 1 : -1;
    }

    // ------------------------------------------------------------ exact ties
    // Side of the vertex with planes t w.r.t. the plane of site hsite (code
    // hcode) when the FP64 filter cannot decide it: the test is evaluated
    // again in FP64 with every operation checked to be exact (the error of
    // each product by a fused multiply-add, of each sum by the two-sum
    // identity).  That holds for inputs with short dyadic coordinates, such
    // as lattices, which is where exact ties occur.  If the value is exact
    // and non-zero its sign decides (+-1).  If it is exactly zero the weights
    // are perturbed symbolically, w_k -> w_k + d^(k+1) for infinitesimal d
    // and original index k (Simulation of Simplicity): the test S is linear
    // in the plane offsets b = (|a|^2 + w_i - w_x) / 2, hence in the weights,
    // and its sign is that of the weight derivative of lowest original index
    // among the non-zero ones (+-2).  Returns 0 if some operation was not
    // exact (the sign stays undecided).
    //   S = det (a_h . y - b_h) = b_A a_h.(B x C) + b_B a_h.(C x A) + b_C a_h.(A x B) - b_h det
    //   dS/dw_x = -a_h.cross_X / 2 (X the plane of site x), dS/dw_m = det / 2
    //   (m the site of h), dS/dw_i = (sum of a_h.cross_X over site planes - det) / 2;
    // the vertex is outside iff S det > 0.
    struct PX {
        double a[3], b;
        uint32_t orig;  // original index of the plane's site (box faces: none)
        bool site;
    };
    __device__ static double xmul(double a, double b, bool& ok) {
        const double p = a * b;
        ok &= fma(a, b, -p) == 0.0;
        return p;
    }
    __device__ static double xadd(double a, double b, bool& ok) {
        const double s = a + b;
        const double bv = s - a;
        ok &= ((a - (s - bv)) + (b - bv)) == 0.0;
        return s;
    }
    __device__ PX plane_exact(int32_t code, float4 site, bool& ok) const {
        PX r;
        const double q[3] = {(double)px, (double)py, (double)pz};
        if (code < 0) {
            const int c = -code - 1, ax = c >> 1, side = c & 1;
            r.a[0] = r.a[1] = r.a[2] = 0.0;
            r.a[ax] = side ? 1.0 : -1.0;
            r.b = side ? xadd((double)A.bbox[3 + ax], -q[ax], ok) : xadd(q[ax], -(double)A.bbox[ax], ok);
            r.orig = 0u;
            r.site = false;
        } else {
            r.a[0] = xadd((double)site.x, -q[0], ok);
            r.a[1] = xadd((double)site.y, -q[1], ok);
            r.a[2] = xadd((double)site.z, -q[2], ok);
            double s2 = xadd(xadd(xmul(r.a[0], r.a[0], ok), xmul(r.a[1], r.a[1], ok), ok),
                             xmul(r.a[2], r.a[2], ok), ok);
            r.b = 0.5 * xadd(s2, xadd((double)pw, -(double)site.w, ok), ok);
            r.orig = cold_args()->order[code];
            r.site = true;
        }
        return r;
    }
    __device__ static void xcross(const double* u, const double* v, double* o, bool& ok) {
        o[0] = xadd(xmul(u[1], v[2], ok), -xmul(u[2], v[1], ok), ok);
        o[1] = xadd(xmul(u[2], v[0], ok), -xmul(u[0], v[2], ok), ok);
        o[2] = xadd(xmul(u[0], v[1], ok), -xmul(u[1], v[0], ok), ok);
    }
    __device__ static double xdot(const double* u, const double* v, bool& ok) {
        return xadd(xadd(xmul(u[0], v[0], ok), xmul(u[1], v[1], ok), ok), xmul(u[2], v[2], ok), ok);
    }
    __device__ int side_exact(W t, int32_t hcode) const {
        const float4 hsite = A.pts[hcode];
        bool ok = true;
        const PX P0 = plane_exact(M.pcode[T::fld(t, 0)], M.psite[T::fld(t, 0)], ok);
        const PX P1 = plane_exact(M.pcode[T::fld(t, 1)], M.psite[T::fld(t, 1)], ok);
        const PX P2 = plane_exact(M.pcode[T::fld(t, 2)], M.psite[T::fld(t, 2)], ok);
        const PX H = plane_exact(hcode, hsite, ok);
        double cr[3][3];
        xcross(P1.a, P2.a, cr[0], ok);
        xcross(P2.a, P0.a, cr[1], ok);
        xcross(P0.a, P1.a, cr[2], ok);
        const double det = xdot(P0.a, cr[0], ok);
        const double hb[3] = {xdot(H.a, cr[0], ok), xdot(H.a, cr[1], ok), xdot(H.a, cr[2], ok)};
        double S = xadd(xadd(xmul(P0.b, hb[0], ok), xmul(P1.b, hb[1], ok), ok),
                        xadd(xmul(P2.b, hb[2], ok), -xmul(H.b, det, ok), ok), ok);
        if (!ok || det == 0.0) return 0;
        const int sd = det > 0.0 ? 1 : -1;
        if (S != 0.0) return (S > 0.0 ? 1 : -1) == sd ? 1 : -1;
        // exact tie: the lowest original index with a non-zero weight derivative
        uint32_t best = H.orig;
        int sgn = sd;  // dS/dw_m = det / 2
        double own = -det;
        const PX* X[3] = {&P0, &P1, &P2};
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            if (!X[r]->site) continue;
            own = xadd(own, hb[r], ok);
            if (hb[r] != 0.0 && X[r]->orig < best) {
                best = X[r]->orig;
                sgn = hb[r] > 0.0 ? -1 : 1;  // dS/dw_x = -a_h.cross_X / 2
            }
        }
        if (!ok) return 0;
        const uint32_t self_orig = cold_args()->order[self];
        if (own != 0.0 && self_orig < best) sgn = own > 0.0 ? 1 : -1;
        return sgn == sd ? 2 : -2;
    }

    // ------------------------------------------------------------ clip
    // mode 0: plain FP32 signs; 1: doubtful signs re-evaluated in FP64;
    // 2: doubtful signs taken as inside; 3: every sign evaluated in FP64.
    __device__ void classify(float ax, float ay, float az, float b, float sbh, int32_t hcode,
                             int mode, Wave<uint64_t>& R, bool* any_out, bool* all_out) {
        const float an1 = fabsf(ax) + fabsf(ay) + fabsf(az);
        if (kCount && mode != 2) count(kCtrClassify, nalive());
        const int ns = nsv();
        uint64_t amb_any = 0;
        bool anyo = false, allo = true;
        Lane<uint8_t> amb;
        if constexpr (!kReg) amb.m = M.amb + ln;
        int lo, hi;
        share(ns, kBatch, &lo, &hi);
        for (int s0 = (kReg ? 0 : lo); s0 < (kReg ? VPL : hi); s0 += kBatch) {
            VBatch v;
            load_batch(s0, ns, v);
            float e[kBatch];
            if (mode != 0) {
#pragma unroll
                for (int k = 0; k < kBatch; ++k) e[k] = ev[s0 + k];
            }
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const int s = s0 + k;
                const float sv = fmaf(ax, v.a[k], fmaf(ay, v.b[k], fmaf(az, v.c[k], -b)));
                const bool al = (v.al[k] >> ln) & 1;
                bool o = al && sv > 0.f;
                bool am = false;
                if (mode != 0) {
                    float beta = 64.f * kU * (an1 * e[k] + sbh);
                    am = al && (mode == 3 || fabsf(sv) <= beta);
                    if (am && mode == 2) o = false;
                }
                const uint64_t r = ballot(o);
                if (s < ns) {
                    amb[s] = am;
                    R[s] = r;
                }
                amb_any |= ballot(am);
                anyo |= r != 0;
                allo &= r == v.al[k];
            }
        }
        bool ambf = amb_any != 0;
        if constexpr (G > 1) {
            const uint32_t v[3] = {anyo ? 1u : 0u, allo ? 1u : 0u, ambf ? 1u : 0u};
            const uint32_t* t = exch(v);
            anyo = false;
            allo = true;
            ambf = false;
#pragma unroll
            for (int w = 0; w < G; ++w) {
                anyo |= t[w * 8] != 0;
                allo &= t[w * 8 + 1] != 0;
                ambf |= t[w * 8 + 2] != 0;
            }
        }
        if ((mode == 1 || mode == 3) && ambf) {
            flags |= kFlagFP64;
            if constexpr (kCount) {
                uint64_t na = 0;
#pragma unroll
                for (int s = 0; s < (kReg ? VPL : ns); ++s) na += (uint64_t)popc(ballot(amb[s] != 0));
                count(kCtrFP64, na);
            }
            P64 h = plane64(hcode, A.pts[hcode]);
            anyo = false;
            allo = true;
            bool uns = false, pert = false;
#pragma unroll
            for (int s = (kReg ? 0 : lo); s < (kReg ? VPL : min(hi, ns)); ++s) {
                bool o = (R[s] >> ln) & 1;
                bool unsure = false, tie = false;
                if (amb[s]) {
                    int sg = side64(vt[s], h);
                    if constexpr (kSoS) {
                        if (sg == 0) {
                            sg = side_exact(vt[s], hcode);
                            tie = sg == 2 || sg == -2;
                        }
                    }
                    o = sg > 0;
                    unsure = sg == 0;
                }
                const uint64_t r = ballot(o);
                R[s] = r;
                anyo |= r != 0;
                allo &= r == alive[s];
                uns |= ballot(unsure) != 0;
                pert |= ballot(tie) != 0;
            }
            if constexpr (G > 1) {
                const uint32_t v[4] = {anyo ? 1u : 0u, allo ? 1u : 0u, uns ? 1u : 0u, pert ? 1u : 0u};
                const uint32_t* t = exch(v);
                anyo = false;
                allo = true;
                uns = false;
                pert = false;
#pragma unroll
                for (int w = 0; w < G; ++w) {
                    anyo |= t[w * 8] != 0;
                    allo &= t[w * 8 + 1] != 0;
                    uns |= t[w * 8 + 2] != 0;
                    pert |= t[w * 8 + 3] != 0;
                }
            }
            if (uns) flags |= kFlagUncertain;
            if (pert) flags |= kFlagPerturbed;
        }
        *any_out = anyo;
        *all_out = allo;
    }

    // Tries the clip with the given outside masks; on an inconsistent
    // boundary sets *consistent = false and leaves the cell untouched.
    __device__ int apply(Wave<uint64_t>& R, bool any, bool all, float ax, float ay, float az, float b, float sbh,
                         int32_t hcode, bool* consistent) {
        *consistent = true;
        const int ns = nsv();
        if (!any) return kNone;
        if (all) return kEmptied;
        if (np >= CAP) {
            gc();
            if (np >= CAP) return kOverflow;
        }
        int sa, sb;  // this wave's share of the slots in use
        share(ns, 1, &sa, &sb);
        if constexpr (VPL > 1) {
#pragma unroll
            for (int s = (kReg ? 0 : sa); s < (kReg ? VPL : sb); ++s)
                M.outf[s * 64 + ln] = (uint8_t)((R[s] >> ln) & 1);
            sync();
        }
        auto is_out = [&](uint32_t v) -> bool {
            if constexpr (VPL == 1) return (R[0] >> v) & 1;
            else return M.outf[v] != 0;
        };
        Lane<uint32_t> cross, pre, frank, nb1, nb2;
        Lane<W> rec;
        Lane<uint8_t> isnew;
        Wave<uint64_t> fr;
        if constexpr (!kReg) {
            cross.m = M.cross + ln; pre.m = M.pre + ln; frank.m = M.frank + ln;
            nb1.m = M.nb1 + ln; nb2.m = M.nb2 + ln; rec.m = M.rec + ln; isnew.m = M.isnew + ln;
            fr.m = M.fr;
        }
        // crossing edges of kept vertices, ranked over the wave (over the
        // group: the counts of lower waves come first)
        uint32_t m = 0;
#pragma unroll
        for (int s = (kReg ? 0 : sa); s < (kReg ? VPL : sb); ++s) {
            bool kept = ((alive[s] & ~R[s]) >> ln) & 1;
            uint32_t c = 0, cnt = 0;
            if (kept) {
                const W nbr = va[s];
#pragma unroll
                for (int e = 0; e < 3; ++e)
                    if (is_out(T::fld(nbr, e))) {
                        c |= 1u << e;
                        ++cnt;
                    }
            }
            cross[s] = c;
            uint64_t b0 = ballot(cnt & 1), b1 = ballot(cnt & 2);
            pre[s] = m + mbcnt(b0) + 2 * mbcnt(b1);
            m += popc(b0) + 2 * popc(b1);
        }
        uint32_t pbase;
        m = g_scan(m, &pbase);
        // free slots (dead or removed), ranked; slots above the used ones are free
        const int nsf = kReg ? VPL : min(VPL, ns + (int)((m + 63) >> 6) + 1);
        int fa, fb;  // this wave's share of the slots new vertices may take
        share(nsf, 1, &fa, &fb);
        uint32_t nfree = 0;
#pragma unroll
        for (int s = (kReg ? 0 : fa); s < (kReg ? VPL : fb); ++s) {
            const uint64_t f = (s < ns) ? (~alive[s] | R[s]) : ~0ull;
            fr[s] = f;
            frank[s] = nfree + mbcnt(f);
            nfree += popc(f);
        }
        uint32_t fbase;
        nfree = g_scan(nfree, &fbase);
        if (m == 0) {  // some vertex is cut off but no edge crosses the plane
            *consistent = false;
            return kNone;
        }
        if (m > nfree) return kOverflow;
        const uint32_t h = (uint32_t)np;
        ++serial;
        if (serial >= T::kTagMax) {  // tag space exhausted: clear the tables
            for (int q = (int)(wid * 64 + ln); q < CAP; q += 64 * G) { M.ta[q] = 0; M.tb[q] = 0; }
            serial = 1;
        }
        const uint32_t tag = serial << T::kTagShift;
        const uint32_t vmask = (1u << T::kTagShift) - 1u;
#pragma unroll
        for (int s = (kReg ? 0 : fa); s < (kReg ? VPL : fb); ++s) {
            const uint32_t rk = frank[s] + fbase;
            const bool nw = ((fr[s] >> ln) & 1) && rk < m;
            isnew[s] = nw;
            if (nw) M.sor[rk] = s * 64 + ln;
        }
#pragma unroll
        for (int s = (kReg ? 0 : sa); s < (kReg ? VPL : sb); ++s) {
            const uint32_t c = cross[s];
            if (c) {
                uint32_t j = pre[s] + pbase;
                const W t = vt[s];
#pragma unroll
                for (int e = 0; e < 3; ++e)
                    if ((c >> e) & 1) {
                        uint32_t x = T::fld(t, (e + 2) % 3), y = T::fld(t, (e + 1) % 3);
                        M.edge[j++] = T::pack3((uint32_t)(s * 64 + ln), x, y);
                    }
            }
        }
        sync();
#pragma unroll
        for (int s = (kReg ? 0 : fa); s < (kReg ? VPL : fb); ++s) {
            W r = 0;
            if (isnew[s]) {
                r = M.edge[frank[s] + fbase];
                uint32_t me = tag | (uint32_t)(s * 64 + ln);
                M.ta[T::fld(r, 1)] = me;
                M.tb[T::fld(r, 2)] = me;
            }
            rec[s] = r;
        }
        sync();
        bool bad = false;
#pragma unroll
        for (int s = (kReg ? 0 : fa); s < (kReg ? VPL : fb); ++s) {
            uint32_t n1 = 0, n2 = 0;
            if (isnew[s]) {
                const W r = rec[s];
                uint32_t me = tag | (uint32_t)(s * 64 + ln);
                uint32_t x = T::fld(r, 1), y = T::fld(r, 2);
                uint32_t a1 = M.ta[y], a2 = M.tb[x];
                bad |= M.ta[x] != me || M.tb[y] != me;
                bad |= (a1 & ~vmask) != tag || (a2 & ~vmask) != tag;
                n1 = a1 & vmask;
                n2 = a2 & vmask;
            }
            nb1[s] = n1;
            nb2[s] = n2;
        }
        bad = g_or(ballot(bad) != 0);
        if (!bad) {
            // the new vertices must form one cycle around the new facet:
            // following "next around h" from the first one returns after m steps
            const uint32_t start = uni(M.sor[0]);
            uint32_t v = start, steps = 0;
            do {
                const int sl = (int)(v >> 6), lv = (int)(v & 63);
                uint32_t nxt = 0xFFFFFFFFu;
                if constexpr (kReg) {
#pragma unroll
                    for (int s = 0; s < VPL; ++s)
                        if (s == sl) nxt = rdl(nb1[s], lv);
                } else if constexpr (G == 1) {
                    if (sl < nsf) nxt = rdl(nb1[sl], lv);
                } else {
                    // written by other waves, before the exchange above
                    if (sl < nsf) nxt = uni(M.nb1[v]);
                }
                v = nxt;
                ++steps;
            } while (v != start && steps <= m);
            bad = steps != m;
        }
        if (ballot(bad)) {
            *consistent = false;
            return kNone;
        }
        // commit: kept vertices point at their new neighbours
#pragma unroll
        for (int s = (kReg ? 0 : sa); s < (kReg ? VPL : sb); ++s) {
            const uint32_t c = cross[s];
            if (c) {
                uint32_t j = pre[s] + pbase;
                W a = va[s];
#pragma unroll
                for (int e = 0; e < 3; ++e)
                    if ((c >> e) & 1) a = T::setfld(a, e, M.sor[j++]);
                va[s] = a;
            }
        }
        // new vertices: planes (h, x, y), position by Cramer's rule
#pragma unroll
        for (int s = (kReg ? 0 : fa); s < (kReg ? VPL : fb); ++s) {
            if (isnew[s]) {
                const W r = rec[s];
                uint32_t x = T::fld(r, 1), y = T::fld(r, 2);
                vt[s] = T::pack3(h, x, y);
                va[s] = T::pack3(T::fld(r, 0), nb1[s], nb2[s]);
                float4 P = M.pl[x], Q = M.pl[y];
                // n0 = a_x cross a_y, n1 = a_y cross a_h, n2 = a_h cross a_x
                float n00 = P.y * Q.z - P.z * Q.y, n01 = P.z * Q.x - P.x * Q.z, n02 = P.x * Q.y - P.y * Q.x;
                float n10 = Q.y * az - Q.z * ay, n11 = Q.z * ax - Q.x * az, n12 = Q.x * ay - Q.y * ax;
                float n20 = ay * P.z - az * P.y, n21 = az * P.x - ax * P.z, n22 = ax * P.y - ay * P.x;
                float det = fmaf(ax, n00, fmaf(ay, n01, az * n02));
                // hardware reciprocal (1 ulp): the FP32 position only decides
                // signs, within the error scale; outputs are recomputed in FP64
                float inv = __builtin_amdgcn_rcpf(det);
                const float q0 = (b * n00 + P.w * n10 + Q.w * n20) * inv;
                const float q1 = (b * n01 + P.w * n11 + Q.w * n21) * inv;
                const float q2 = (b * n02 + P.w * n12 + Q.w * n22) * inv;
                y0[s] = q0;
                y1[s] = q1;
                y2[s] = q2;
                // error scale of the vertex, for the doubtful-sign test (only
                // read when signs are checked: robust builds)
                if (robust != 0) {
                    const float sbx = M.psb[x], sby = M.psb[y];
                    float e = (sbh * (fabsf(n00) + fabsf(n01) + fabsf(n02)) +
                               sbx * (fabsf(n10) + fabsf(n11) + fabsf(n12)) +
                               sby * (fabsf(n20) + fabsf(n21) + fabsf(n22))) * fabsf(inv);
                    ev[s] = e + fabsf(q0) + fabsf(q1) + fabsf(q2);
                }
            }
        }
#pragma unroll
        for (int s = (kReg ? 0 : fa); s < (kReg ? VPL : fb); ++s) {
            const uint64_t keep = (s < ns) ? (alive[s] & ~R[s]) : 0ull;
            alive[s] = keep | ballot(isnew[s] != 0);
        }
        if constexpr (!kReg) {
            // free slots are taken in increasing order: the last rank's is the highest
            const int top = (int)uni(M.sor[m - 1]) + 1;
            if (top > vhi) vhi = top;
        }
        if (ln == 0 && lead()) {
            M.pl[h] = make_float4(ax, ay, az, b);
            M.psb[h] = sbh;
            M.pcode[h] = hcode;
            M.psite[h] = A.pts[hcode];
        }
        np = (int)h + 1;
        sync();
        count(kCtrNewVertex, m);
        count(kCtrEffective, 1);
        return kChanged;
    }

    // Plain FP32 signs unless the cell is being rebuilt robustly; an
    // inconsistent boundary in FP32 asks for that rebuild; in the robust modes
    // doubtful signs fall back to "inside" and, failing that, the plane is
    // skipped and the cell flagged.
    __device__ int clip(float ax, float ay, float az, float b, float sbh, int32_t hcode) {
        Wave<uint64_t> R;
        if constexpr (!kReg) R.m = M.R;
        count(kCtrClip, 1);
        bool any, all;
        classify(ax, ay, az, b, sbh, hcode, robust == 0 ? 0 : (robust == 1 ? 1 : 3), R, &any, &all);
        bool ok;
        int r = apply(R, any, all, ax, ay, az, b, sbh, hcode, &ok);
        if constexpr (VPL == 1 && G == 1) cut_mask = R[0];
        if (ok) return r;
        if (robust < 2) return kRestart;
        flags |= kFlagUncertain;
        classify(ax, ay, az, b, sbh, hcode, 2, R, &any, &all);
        r = apply(R, any, all, ax, ay, az, b, sbh, hcode, &ok);
        if constexpr (VPL == 1 && G == 1) cut_mask = R[0];
        return ok ? r : kNone;
    }

    // Drop planes no vertex uses (supplementary Sec. A, "Garbage collection").
    __device__ void gc() {
        const int ns = nsv();
        int sa, sb;
        share(ns, 1, &sa, &sb);
        for (int q = (int)(wid * 64 + ln); q < np; q += 64 * G) M.key[q] = 0;
        sync();
#pragma unroll
        for (int s = (kReg ? 0 : sa); s < (kReg ? VPL : sb); ++s)
            if ((alive[s] >> ln) & 1) {
                const W t = vt[s];
                M.key[T::fld(t, 0)] = 1;
                M.key[T::fld(t, 1)] = 1;
                M.key[T::fld(t, 2)] = 1;
            }
        sync();
        uint32_t cnt = 0;
        if constexpr (kReg) {
            float4 pl[VPL], ps[VPL];
            float sb[VPL];
            int32_t pc[VPL];
            uint32_t dst[VPL];
            bool used[VPL];
#pragma unroll
            for (int s = 0; s < VPL; ++s) {
                int q = s * 64 + ln;
                used[s] = q < np && M.key[q] != 0;
                uint64_t u = ballot(used[s]);
                dst[s] = cnt + mbcnt(u);
                cnt += popc(u);
                if (used[s]) {
                    pl[s] = M.pl[q];
                    ps[s] = M.psite[q];
                    sb[s] = M.psb[q];
                    pc[s] = M.pcode[q];
                }
            }
            sync();
#pragma unroll
            for (int s = 0; s < VPL; ++s) {
                int q = s * 64 + ln;
                if (used[s]) {
                    M.pl[dst[s]] = pl[s];
                    M.psite[dst[s]] = ps[s];
                    M.psb[dst[s]] = sb[s];
                    M.pcode[dst[s]] = pc[s];
                    M.key[q] = (int32_t)dst[s];
                }
            }
        } else {
            // in place, 64 planes at a time, by the first wave of the group:
            // a destination never lies above its source, and every source of
            // a chunk is read before any of its destinations is written
            for (int q0 = 0; q0 < (lead() ? np : 0); q0 += 64) {
                const int q = q0 + (int)ln;
                const bool used = q < np && M.key[q] != 0;
                const uint64_t u = ballot(used);
                const uint32_t dst = cnt + mbcnt(u);
                cnt += popc(u);
                float4 pl = make_float4(0.f, 0.f, 0.f, 0.f), ps = pl;
                float sb = 0.f;
                int32_t pc = 0;
                if (used) {
                    pl = M.pl[q];
                    ps = M.psite[q];
                    sb = M.psb[q];
                    pc = M.pcode[q];
                }
                wsync();
                if (used) {
                    M.pl[dst] = pl;
                    M.psite[dst] = ps;
                    M.psb[dst] = sb;
                    M.pcode[dst] = pc;
                    M.key[q] = (int32_t)dst;
                }
                wsync();
            }
            if constexpr (G > 1) cnt = bcast(cnt);
        }
        sync();
#pragma unroll
        for (int s = (kReg ? 0 : sa); s < (kReg ? VPL : sb); ++s)
            if ((alive[s] >> ln) & 1) {
                const W t = vt[s];
                vt[s] = T::pack3((uint32_t)M.key[T::fld(t, 0)], (uint32_t)M.key[T::fld(t, 1)],
                                 (uint32_t)M.key[T::fld(t, 2)]);
            }
        np = (int)cnt;
        sync();
    }

    // ------------------------------------------------------------ traversal
    // Tests one child record against the current cell (Sec. 4.2.2).
    __device__ void node_test(const NodeChild& c, float* key, bool* cull, float* delta) const {
        float blx = c.lo[0] - px, bly = c.lo[1] - py, blz = c.lo[2] - pz;
        float bhx = c.hi[0] - px, bhy = c.hi[1] - py, bhz = c.hi[2] - pz;
        float dx = fmaxf(fmaxf(blx, -bhx), 0.f), dy = fmaxf(fmaxf(bly, -bhy), 0.f), dz = fmaxf(fmaxf(blz, -bhz), 0.f);
        // hardware square roots (1 ulp), inside the bound's rounding margin
        float d = __builtin_amdgcn_sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
        float dw = kW ? pw - c.wmax : 0.f;
        float lb, err;
        if (dw > 0.f && culling() == 3) {
            // every site j in the box has b_j / |a_j| >= f(|a_j|) with
            // f(t) = t/2 + dw/(2t), and |a_j| lies between the box's nearest
            // and farthest distances: the bound is f at sqrt(dw) clamped to
            // that range (the paper's bound keeps only dw < 0 and is d/2 here)
            const float fx = pmax(fabsf(blx), fabsf(bhx)), fy = pmax(fabsf(bly), fabsf(bhy)),
                        fz = pmax(fabsf(blz), fabsf(bhz));
            const float dfar = __builtin_amdgcn_sqrtf(fmaf(fx, fx, fmaf(fy, fy, fz * fz)));
            const float dc = fminf(fmaxf(__builtin_amdgcn_sqrtf(dw), d), dfar);
            if (dc > 0.f) {
                lb = 0.5f * dc + 0.5f * dw * __builtin_amdgcn_rcpf(dc);
                err = lb;
            } else {
                lb = 0.5f * d;
                err = 0.5f * d;
            }
        } else if (dw >= 0.f) {
            lb = 0.5f * d;
            err = 0.5f * d;
        } else if (d > 0.f) {
            const float q = 0.5f * dw * __builtin_amdgcn_rcpf(d);
            lb = 0.5f * d + q;
            err = 0.5f * d - q;
        } else {
            lb = -INFINITY;
            err = 0.f;
        }
        float rb2;
        if (culling() == 2) {
            rb2 = riso2;
        } else {
            // per axis: the far-corner square of each side the box reaches
            const float tx = pmax(bhx >= 0.f ? hx2 : 0.f, blx < 0.f ? lx2 : 0.f);
            const float ty = pmax(bhy >= 0.f ? hy2 : 0.f, bly < 0.f ? ly2 : 0.f);
            const float tz = pmax(bhz >= 0.f ? hz2 : 0.f, blz < 0.f ? lz2 : 0.f);
            rb2 = tx + ty + tz;
        }
        float rb = __builtin_amdgcn_sqrtf(rb2);
        // lower bound made safe against FP32 rounding of its terms
        float lbs = lb - 16.f * kU * err;
        *key = lbs;
        *cull = lbs > rb * (1.f + 16.f * kU);
        *delta = lbs - rb;
    }

    __device__ void push(uint32_t e, float k) {
        const int slot = qn >> 6, l = qn & 63;
        if constexpr (kQExt) {
            if (slot >= VPL) {
                if (ln == 0) {
                    M.qxe[(slot - VPL) * 64 + l] = e;
                    M.qxk[(slot - VPL) * 64 + l] = k;
                }
                wsync();  // read back by every lane
                ++qn;
                return;
            }
        }
        if constexpr (kReg) {
#pragma unroll
            for (int s = 0; s < VPL; ++s)
                if (s == slot && (int)ln == l) {
                    qe[s] = e;
                    qk[s] = k;
                }
        } else {
            if ((int)ln == l && lead()) {
                qe[slot] = e;
                qk[slot] = k;
            }
        }
        ++qn;
    }

    // Removes and returns the entry with the smallest key (best-first), or
    // the last pushed one (depth-first).  The queue is kept by the first wave
    // of a group, which hands the entry to the others.
    __device__ void pop(uint32_t* e, float* k, bool least = false) {
        uint32_t ee = 0;
        float kk = 0.f;
        if (lead()) pop_lead(&ee, &kk, least || traversal() != 2);
        if constexpr (G > 1) {
            const uint32_t v[2] = {ee, __float_as_uint(kk)};
            const uint32_t* t = exch(v);
            ee = t[0];
            kk = __uint_as_float(t[1]);
        }
        --qn;
        *e = ee;
        *k = kk;
    }
    __device__ void pop_lead(uint32_t* e, float* k, bool least) {
        const int nq = (qn + 63) >> 6;
        int S, L;
        if (!least) {
            S = (qn - 1) >> 6;
            L = (qn - 1) & 63;
        } else {
            float bk = INFINITY;
            int bs = 0;
#pragma unroll
            for (int s = 0; s < (kReg ? VPL : nq); ++s) {
                int idx = s * 64 + (int)ln;
                if (idx < qn) {
                    const float kk = qk[s];
                    if (kk < bk) {
                        bk = kk;
                        bs = s;
                    }
                }
            }
            if constexpr (kQExt) {
                for (int s = VPL; s < (qn + 63) >> 6; ++s) {
                    const int idx = s * 64 + (int)ln;
                    if (idx < qn) {
                        const float kk = M.qxk[idx - 64 * VPL];
                        if (kk < bk) {
                            bk = kk;
                            bs = s;
                        }
                    }
                }
            }
            float m = wmin(bk);
            uint64_t msk = ballot(bk == m && (int)ln < qn);
            L = msk ? lowest(msk) : 0;
            S = rdl(bs, L);
        }
        uint32_t ee = 0, le = 0;
        float kk = 0.f, lk = 0.f;
        const int last = qn - 1, ls = last >> 6, ll = last & 63;
        if constexpr (kQExt) {
            if (ls >= VPL) {  // the last entry is beyond the register slots (LDS)
                if (S < VPL) {
#pragma unroll
                    for (int s = 0; s < VPL; ++s)
                        if (s == S) {
                            ee = rdl(qe[s], L);
                            kk = rdl(qk[s], L);
                        }
                } else {
                    ee = uni(M.qxe[(S - VPL) * 64 + L]);
                    kk = uni(M.qxk[(S - VPL) * 64 + L]);
                }
                le = uni(M.qxe[last - 64 * VPL]);
                lk = uni(M.qxk[last - 64 * VPL]);
                if (S < VPL) {
#pragma unroll
                    for (int s = 0; s < VPL; ++s)
                        if (s == S && (int)ln == L) {
                            qe[s] = le;
                            qk[s] = lk;
                        }
                } else {
                    if (ln == 0) {
                        M.qxe[(S - VPL) * 64 + L] = le;
                        M.qxk[(S - VPL) * 64 + L] = lk;
                    }
                    wsync();
                }
                *e = ee;
                *k = kk;
                return;
            }
        }
        if constexpr (kReg) {
#pragma unroll
            for (int s = 0; s < VPL; ++s)
                if (s == S) {
                    ee = rdl(qe[s], L);
                    kk = rdl(qk[s], L);
                }
#pragma unroll
            for (int s = 0; s < VPL; ++s)
                if (s == ls) {
                    le = rdl(qe[s], ll);
                    lk = rdl(qk[s], ll);
                }
#pragma unroll
            for (int s = 0; s < VPL; ++s)
                if (s == S && (int)ln == L) {
                    qe[s] = le;
                    qk[s] = lk;
                }
        } else {
            ee = rdl(qe[S], L);
            kk = rdl(qk[S], L);
            le = rdl(qe[ls], ll);
            lk = rdl(qk[ls], ll);
            if ((int)ln == L) {
                qe[S] = le;
                qk[S] = lk;
            }
        }
        *e = ee;
        *k = kk;
    }

    // The candidates of `mask` (plane of lane L: a, b, size sb) that have
    // some vertex of the cell outside, or, when doubtful signs are
    // re-evaluated, within rounding of it.  A plane that misses the cell
    // misses every cell it is later clipped to, so the others need no clip:
    // one pass over the vertices for the whole leaf (and for a wave group one
    // exchange) instead of a selection and a clip each.  The test is the FP32
    // side test of classify.
    __device__ uint64_t cutting(uint64_t mask, float ax, float ay, float az, float b, float sb) {
        const int ns = nsv();
        int lo, hi;
        share(ns, kBatch, &lo, &hi);
        const bool tol = robust != 0;
        if constexpr (kCount) count(kCtrClassify, nalive() * (uint64_t)popc(mask));
        uint64_t cb = 0;  // candidates this lane's vertices put outside
        for (int s0 = (kReg ? 0 : lo); s0 < (kReg ? VPL : hi); s0 += kBatch) {
            VBatch v;
            load_batch(s0, ns, v);
            float e[kBatch];
            if (tol) {
#pragma unroll
                for (int k = 0; k < kBatch; ++k) e[k] = ev[s0 + k];
            }
            for (uint64_t m = mask; m; m &= m - 1) {
                const int L = lowest(m);
                const float hx = rdl(ax, L), hy = rdl(ay, L), hz = rdl(az, L), hb = rdl(b, L);
                const float an1 = fabsf(hx) + fabsf(hy) + fabsf(hz), hs = rdl(sb, L);
                bool o = false;
#pragma unroll
                for (int k = 0; k < kBatch; ++k) {
                    const float sv = fmaf(hx, v.a[k], fmaf(hy, v.b[k], fmaf(hz, v.c[k], -hb)));
                    const bool al = (v.al[k] >> ln) & 1;
                    o |= al && (tol ? sv >= -64.f * kU * (an1 * e[k] + hs) : sv > 0.f);
                }
                if (o) cb |= 1ull << L;
            }
        }
        uint64_t cut = wor64(cb);
        if constexpr (G > 1) {
            const uint32_t v2[2] = {(uint32_t)cut, (uint32_t)(cut >> 32)};
            const uint32_t* t = exch(v2);
            cut = 0;
#pragma unroll
            for (int w = 0; w < G; ++w) cut |= (uint64_t)t[w * 8] | ((uint64_t)t[w * 8 + 1] << 32);
        }
        return mask & cut;
    }

    // Clips by the candidate sites of one leaf (those of lanes in `allow`);
    // nearest plane first.
    __device__ int leaf(uint32_t ref, uint64_t allow) {
        const uint32_t first = leaf_first(ref), nsite = leaf_count(ref);
        count(kCtrLeaf, 1);
        count(kCtrSite, nsite);
        float ax = 0.f, ay = 0.f, az = 0.f, a2 = 0.f, b = 0.f, dw = 0.f, key = INFINITY;
        float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
        bool cand = false;
        {
            // every lane loads (lanes past the leaf repeat its last site) so
            // that the arithmetic runs without a divergent branch
            const uint32_t j = first + ((uint32_t)ln < nsite ? (uint32_t)ln : nsite - 1u);
            q = A.pts[j];
            ax = q.x - px; ay = q.y - py; az = q.z - pz;
            a2 = fmaf(ax, ax, fmaf(ay, ay, az * az));
            dw = kW ? pw - q.w : 0.f;
            b = 0.5f * (a2 + dw);
            cand = (uint32_t)ln < nsite && j != self && q.w != -INFINITY && a2 > 0.f;
            for (int t = 0; t < nwarm; ++t) cand = cand && j != rdl(wsite, t);
            key = cand ? b * __builtin_amdgcn_rsqf(a2) : INFINITY;  // orders candidates only
        }
        const float sbl = 0.5f * (a2 + fabsf(dw));  // size of the terms of b (error scale)
        auto keep = [&](bool c) -> bool {
            if (!c) return false;
            if (culling() == 3) {
                // the plane misses the cell's AABB: max over the box of a.y <= b
                float cx = ax >= 0.f ? bhi0 : blo0, cy = ay >= 0.f ? bhi1 : blo1, cz = az >= 0.f ? bhi2 : blo2;
                float mm = fmaf(ax, cx, fmaf(ay, cy, az * cz));
                float slack = 8.f * kU * (fabsf(ax * cx) + fabsf(ay * cy) + fabsf(az * cz) + a2 + fabsf(dw));
                return mm > b - slack;
            }
            float r2 = radius2_toward(ax, ay, az);
            float t = b - 4.f * kU * (2.f * a2 + fabsf(dw) + r2);
            return !(t > 0.f && t * t > a2 * r2);
        };
        uint64_t mask = ballot(keep(cand));
        if constexpr (kResumes) mask &= allow;
        // from 128 vertices up, the candidates that miss the cell are dropped
        // all at once (not when every sign is taken in FP64)
        if constexpr (G > 1 || VPL >= 2) {
            if (mask && robust < 2) mask = cutting(mask, ax, ay, az, b, 0.5f * (a2 + fabsf(dw)));
        }
        while (mask) {
            // nearest plane first (both traversal orders)
            int L;
            {
                float kk = ((mask >> ln) & 1) ? key : INFINITY;
                float m = wmin(kk);
                uint64_t mm = ballot(kk == m) & mask;
                L = lowest(mm ? mm : mask);
            }
            mask &= ~(1ull << L);
            float hx = rdl(ax, L), hy = rdl(ay, L), hz = rdl(az, L), hb = rdl(b, L);
            const float sb = rdl(sbl, L);
            const uint64_t t0 = tic();
            int r = clip(hx, hy, hz, hb, sb, (int32_t)(first + (uint32_t)L));
            toc(kCtrCycClip, t0);
            if constexpr (kSaves) {
                if (r == kOverflow) {  // the cell is as before this candidate
                    ov_ok = true;
                    ov_leaf = ref;
                    ov_mask = mask | (1ull << L);
                    ov_phase = leaf_phase;
                }
            }
            if (r == kEmptied || r == kOverflow || r == kRestart) return r;
            if (r == kChanged) {
                bounds_after_clip();
                mask &= ballot(keep(true));
            }
        }
        return kNone;
    }

    __device__ void load_child(uint32_t node, int s, NodeChild* c) const {
        const float4* src = reinterpret_cast<const float4*>(&A.nodes[node].c[s]);
        float4 u = src[0], v = src[1];
        c->lo[0] = u.x; c->lo[1] = u.y; c->lo[2] = u.z; c->wmax = u.w;
        c->hi[0] = v.x; c->hi[1] = v.y; c->hi[2] = v.z; c->ref = __float_as_uint(v.w);
    }

    // KNN warm start (supplementary Sec. A): before the walk, the K sites
    // nearest to p_i are found by a best-first walk of the same BVH (queue
    // keyed by squared distance to the child boxes), and the cell is clipped
    // by their planes, nearest first.  Lanes 0..K-1 keep the K best squared
    // distances (best) and sites (bsite); `worst` is the K-th best (infinite
    // until K are found).  The walk that follows passes over these sites.
    // Returns kNone or what a clip returned (kEmptied, kOverflow, kRestart).
    __device__ int knn_warm(int K) {
        float best = INFINITY;
        uint32_t bsite = 0u;
        float worst = INFINITY;
        qn = 0;
        auto box_d2 = [&](const NodeChild& c) {
            const float dx = fmaxf(fmaxf(c.lo[0] - px, px - c.hi[0]), 0.f);
            const float dy = fmaxf(fmaxf(c.lo[1] - py, py - c.hi[1]), 0.f);
            const float dz = fmaxf(fmaxf(c.lo[2] - pz, pz - c.hi[2]), 0.f);
            return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        };
        auto take_leaf = [&](uint32_t ref) {
            const uint32_t first = leaf_first(ref), cnt = leaf_count(ref);
            const uint32_t j = first + ((uint32_t)ln < cnt ? (uint32_t)ln : cnt - 1u);
            const float4 q = A.pts[j];
            const float dx = q.x - px, dy = q.y - py, dz = q.z - pz;
            const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            const bool ok = (uint32_t)ln < cnt && j != self && q.w != -INFINITY && d2 > 0.f;
            count(kCtrSite, cnt);
            uint64_t m = ballot(ok && d2 < worst);
            while (m) {
                const float c = wmin(((m >> ln) & 1) ? d2 : INFINITY);
                if (!(c < worst)) break;
                const uint64_t mm = ballot(((m >> ln) & 1) && d2 == c) & m;
                const int L = lowest(mm);
                m &= ~(1ull << L);
                const uint32_t js = rdl(j, L);
                // it replaces the worst of the K kept
                const float wv = wmax((int)ln < K ? best : -INFINITY);
                const int W = lowest(ballot((int)ln < K && best == wv));
                if ((int)ln == W) {
                    best = c;
                    bsite = js;
                }
                worst = wmax((int)ln < K ? best : -INFINITY);
            }
        };
        bool ok = true;
        {
            NodeChild c;
            load_child(A.root, (int)(ln & 1), &c);
            const float d = box_d2(c);
            count(kCtrNode, 2);
            push(A.root << 1, rdl(d, 0));
            push((A.root << 1) | 1u, rdl(d, 1));
        }
        int64_t budget = 4 * A.n + 1024;
        while (qn > 0 && ok) {
            if (--budget < 0) break;
            uint32_t e;
            float k;
            pop(&e, &k, true);
            if (!(k < worst)) break;
            NodeChild c;
            load_child(e >> 1, (int)(e & 1), &c);
            const uint32_t ref = uni(c.ref);
            if (ref_is_leaf(ref)) {
                take_leaf(ref);
                continue;
            }
            NodeChild cc;
            load_child(ref, (int)(ln & 1), &cc);
            const float d = box_d2(cc);
            count(kCtrNode, 2);
            for (int sd = 0; sd < 2; ++sd) {
                const float dd = rdl(d, sd);
                if (!(dd < worst)) continue;
                if (qn >= QCAP) {
                    ok = false;  // queue full: go on with the nearest found so far
                    break;
                }
                push((ref << 1) | (uint32_t)sd, dd);
            }
        }
        qn = 0;
        // clip by the found sites, nearest first
        float dd = (int)ln < K ? best : INFINITY;
        for (int t = 0; t < K; ++t) {
            const float c = wmin(dd);
            if (c == INFINITY) break;
            const int L = lowest(ballot(dd == c));
            if ((int)ln == L) dd = INFINITY;
            const uint32_t j = rdl(bsite, L);
            if ((int)ln == nwarm) wsite = j;
            ++nwarm;
            const float4 q = A.pts[j];
            const float ax = q.x - px, ay = q.y - py, az = q.z - pz;
            const float a2 = fmaf(ax, ax, fmaf(ay, ay, az * az));
            const float dw = kW ? pw - q.w : 0.f;
            const uint64_t t0 = tic();
            const int r = clip(ax, ay, az, 0.5f * (a2 + dw), 0.5f * (a2 + fabsf(dw)), (int32_t)j);
            toc(kCtrCycClip, t0);
            if (r == kEmptied || r == kOverflow || r == kRestart) return r;
            if (r == kChanged) update_bounds();
        }
        return kNone;
    }

    // The start of Alg. 1.  From the root, the walk first reaches the site's
    // own leaf (its bound is 0 there) and on the way down queues the sibling
    // of every node on that path, tested against the still uncut box.  Here
    // the own leaf (found through the site's leaf record) is clipped first;
    // then the siblings of its path are gathered by one scalar climb over the
    // parent links, one per lane, and tested together against the cut cell.
    // Only those that may still cut it are queued, with the keys Alg. 1 gives
    // them (a sibling culled here would be culled when popped: the cell only
    // shrinks), top of the path first so that the nearest is queued last.
    // Returns kNone, or what the leaf returned (kEmptied, kOverflow,
    // kRestart); *deep if the path has more than 64 siblings (the walk then
    // starts at the root and passes over the own leaf).
    __device__ int own_leaf_start(uint32_t* own, bool* deep) {
        KArgs* ka = cold_args();
        const uint32_t rec = uni(ka->leaf_of[self]);
        const uint32_t oref = uni(A.nodes[rec >> 1].c[rec & 1].ref);
        *own = oref;
        *deep = false;
        uint32_t e = rec ^ 1u;  // this lane's sibling record: (node << 1) | which child
        int ns = 1;
        for (uint32_t cur = rec;;) {
            const uint32_t u = uni(ka->up[cur >> 1]);
            if (u == kNoParent) break;
            if (ns == 64) {
                *deep = true;
                return kNone;
            }
            if ((int)ln == ns) e = u ^ 1u;
            ++ns;
            cur = u;
        }
        count(kCtrNode, (uint64_t)ns);
        // lanes past the path test the first sibling again (no divergent load)
        const uint32_t me = (int)ln < ns ? e : rdl(e, 0);
        NodeChild c;
        load_child(me >> 1, (int)(me & 1), &c);
        float key = 0.f, delta = 0.f;
        bool cull = true;
        const uint64_t t0 = tic();
        leaf_phase = 0;
        int r = leaf(oref, ~0ull);
        leaf_phase = 1;
        toc(kCtrCycLeaf, t0);
        if (r != kNone) return r;
        node_test(c, &key, &cull, &delta);
        uint64_t live = ballot(!cull && (int)ln < ns);
        while (live) {
            const int L = 63 - __builtin_clzll(live);
            live &= ~(1ull << L);
            if (culling() == 3 && !ball_hit_lane(c, L)) continue;
            if (qn >= QCAP) return kOverflow;
            push(rdl(me, L), rdl(key, L));
        }
        return kNone;
    }

    // Alg. 1.  Returns kNone when done, kEmptied, kOverflow or kRestart.
    // A cell taken over from the previous pass (resume) first finishes the
    // leaf it stopped in, then goes on with the queue it brought.
    __device__ int traverse(bool resume = false, uint32_t rleaf = 0, uint64_t rmask = 0, uint32_t rphase = 1,
                            uint32_t rskip = kNoParent) {
        uint32_t cur = A.root;
        bool have = true;
        uint64_t allow = ~0ull;  // candidates of the first leaf
        if constexpr (kSaves) ov_ok = false;
        uint32_t done_leaf = 0;
        bool skip_done = false;
        bool own_first = false;  // the first leaf is the site's own, then the walk starts at the root
        if constexpr (kResumes) {
            if (resume) {
                // the rest of the leaf it stopped in (one call site of leaf():
                // through the loop below)
                cur = rleaf;
                allow = rmask;
                own_first = rphase == 0;
                if (rphase != 0 && rskip != kNoParent) {  // the own leaf, clipped before this walk
                    done_leaf = rskip;
                    skip_done = true;
                }
            }
        }
        // own leaf first, then the siblings of its path (not for a cell taken
        // over), in the 64-vertex pass only: for the cells that outgrew it
        // the walk from the root is faster (starting them at their own leaf
        // made the larger passes 40-60% slower on the power and surface
        // workloads)
        if (!resume && A.leaf_of != nullptr) {
            if (warm_start() > 0) {
                const int rw = knn_warm(warm_start());
                if constexpr (kSaves) ov_ok = false;  // an overflow in the warm start starts over
                if (rw != kNone) return rw;
            }
            if constexpr (VPL == 1) {
                bool deep;
                const int r = own_leaf_start(&done_leaf, &deep);
                if (r != kNone) return r;
                have = deep;
                skip_done = deep;
            }
        }
        // every node is visited at most once in a valid tree; the bound only
        // guarantees termination if the tree were ever malformed
        int64_t budget = 4 * A.n + 1024;
        for (;;) {
            while (have && !ref_is_leaf(cur)) {
                if (--budget < 0) return kOverflow;
                count(kCtrNode, 2);
                const uint32_t node = cur;
                float key = 0.f, delta = 0.f;
                bool cull = true;
                uint32_t ref = 0;
                NodeChild cc;
                load_child(node, (int)(ln & 1), &cc);
                node_test(cc, &key, &cull, &delta);
                ref = cc.ref;
                const uint64_t cm = ballot(cull);
                bool c0 = (cm & 1ull) != 0, c1 = (cm & 2ull) != 0;
                if (culling() == 3) {
                    if (!c0 && !c1) {
                        bool h0, h1;
                        ball_hit_pair(cc, &h0, &h1);
                        c0 = !h0;
                        c1 = !h1;
                    } else {
                        if (!c0 && !ball_hit_lane(cc, 0)) c0 = true;
                        if (!c1 && !ball_hit_lane(cc, 1)) c1 = true;
                    }
                }
                if (c0 && c1) {
                    have = false;
                    break;
                }
                // descend into the nearer child (smaller bound minus radius),
                // queue the other: the same in both traversal orders, which
                // differ only in what they pop next (Alg. 1: the least key;
                // depth-first: the last pushed)
                const float d0 = rdl(delta, 0), d1 = rdl(delta, 1);
                const int near = c1 ? 0 : (c0 ? 1 : (d0 <= d1 ? 0 : 1));
                const int far = 1 - near;
                if (!(far ? c1 : c0)) {
                    if (qn >= QCAP) return kOverflow;
                    push((node << 1) | (uint32_t)far, rdl(key, far));
                }
                cur = rdl(ref, near);
            }
            if (have && !(skip_done && cur == done_leaf)) {
                const uint64_t t0 = tic();
                if constexpr (kResumes) leaf_phase = own_first ? 0u : 1u;
                int r = leaf(cur, allow);
                if constexpr (kResumes) leaf_phase = 1;
                if constexpr (kSaves) ov_skip = skip_done ? done_leaf : kNoParent;
                if constexpr (kResumes) allow = ~0ull;
                toc(kCtrCycLeaf, t0);
                if (r != kNone) return r;
            }
            if constexpr (kResumes) {
                if (own_first) {  // the own leaf is done: from the root, passing over it
                    own_first = false;
                    done_leaf = cur;
                    skip_done = true;
                    cur = A.root;
                    continue;
                }
            }
            have = false;
            while (qn > 0) {
                if (--budget < 0) return kOverflow;
                uint32_t e;
                float k;
                pop(&e, &k);
                count(kCtrNode, 1);
                if (traversal() != 2 && k > __builtin_amdgcn_sqrtf(rmax2) * (1.f + 16.f * kU)) {
                    qn = 0;  // every key left is at least k: nothing can cut the cell
                    break;
                }
                float key = 0.f, delta = 0.f;
                bool cull = true;
                uint32_t ref = 0;
                NodeChild c;
                load_child(e >> 1, (int)(e & 1), &c);
                node_test(c, &key, &cull, &delta);
                ref = c.ref;
                bool culled = rdl((int)cull, 0) != 0;
                if (!culled && culling() == 3 && !ball_hit_lane(c, 0)) culled = true;
                if (!culled) {
                    cur = rdl(ref, 0);
                    have = true;
                    break;
                }
            }
            if (!have) return kNone;
        }
    }

    // ------------------------------------------------------------ hand-over
    // Writes the state of a cell that overflowed for the next pass; only the
    // header when the overflow is not resumable.
    __device__ void save(HOut& H) {
        if constexpr (kSaves) {
            sync();
            const int tid = (int)(wid * 64 + ln), step = 64 * G;
            if (ov_ok) {
                for (int q = tid; q < np; q += step) {
                    H.pl[q] = M.pl[q];
                    H.psite[q] = M.psite[q];
                    H.psb[q] = M.psb[q];
                    H.pcode[q] = M.pcode[q];
                }
                if constexpr (kReg) {
#pragma unroll
                    for (int s = 0; s < VPL; ++s) {
                        const int q = s * 64 + (int)ln;
                        H.y0[q] = y0[s];
                        H.y1[q] = y1[s];
                        H.y2[q] = y2[s];
                        H.ev[q] = ev[s];
                        H.vt[q] = vt[s];
                        H.va[q] = va[s];
                        H.qe[q] = qe[s];
                        H.qk[q] = qk[s];
                        if (ln == 0) H.alive[s] = alive[s];
                    }
                    if constexpr (kQExt) {
                        for (int q = 64 * VPL + (int)ln; q < qn; q += 64) {
                            H.qe[q] = M.qxe[q - 64 * VPL];
                            H.qk[q] = M.qxk[q - 64 * VPL];
                        }
                    }
                } else {
                    for (int q = tid; q < vhi; q += step) {
                        H.y0[q] = M.y0[q];
                        H.y1[q] = M.y1[q];
                        H.y2[q] = M.y2[q];
                        H.ev[q] = M.ev[q];
                        H.vt[q] = M.vt[q];
                        H.va[q] = M.va[q];
                    }
                    for (int q = tid; q < qn; q += step) {
                        H.qe[q] = M.qe[q];
                        H.qk[q] = M.qk[q];
                    }
                    if (tid < nsv()) H.alive[tid] = M.alive[tid];
                }
            }
            if (tid < kMaxWarm) H.wsite[tid] = tid < nwarm ? wsite : 0u;  // lane t of wave 0 holds site t
            if (tid == 0) {
                H.nwarm = (uint32_t)nwarm;
                H.np = (uint32_t)np;
                H.vhi = (uint32_t)(kReg ? CAP : vhi);
                H.qn = (uint32_t)qn;
                H.flags = flags;
                H.robust = (uint32_t)robust;
                H.leaf = ov_leaf;
                H.mask = ov_mask;
                H.phase = ov_phase;
                H.skip = ov_phase == 0 ? kNoParent : ov_skip;
                H.valid = ov_ok ? 1u : 0u;
            }
        }
    }

    // Takes over a cell saved by the previous pass (instead of init): the
    // traversal then goes on with resume = true, H.leaf, H.mask, H.phase.
    // Vertex, plane and queue numbers are the same in every pass.
    __device__ void resume(uint32_t k, const HIn& H) {
        if constexpr (kResumes) {
            sync();  // every wave is done with the previous cell
            self = k;
            float4 s = A.pts[k];
            px = s.x; py = s.y; pz = s.z; pw = s.w;
            flags = H.flags;
            robust = (int)H.robust;
            nwarm = (int)H.nwarm;
            wsite = (int)ln < kMaxWarm ? H.wsite[ln] : 0u;
            np = (int)H.np;
            vhi = (int)H.vhi;
            qn = (int)H.qn;
            const int tid = (int)(wid * 64 + ln), step = 64 * G;
            for (int q = tid; q < np; q += step) {
                M.pl[q] = H.pl[q];
                M.psite[q] = H.psite[q];
                M.psb[q] = H.psb[q];
                M.pcode[q] = H.pcode[q];
            }
            if constexpr (kReg) {
#pragma unroll
                for (int s2 = 0; s2 < VPL; ++s2) {
                    const int q = s2 * 64 + (int)ln;
                    if (s2 < kPrevCap / 64) {
                        y0[s2] = H.y0[q];
                        y1[s2] = H.y1[q];
                        y2[s2] = H.y2[q];
                        ev[s2] = H.ev[q];
                        vt[s2] = H.vt[q];
                        va[s2] = H.va[q];
                        alive[s2] = H.alive[s2];
                    } else {
                        alive[s2] = 0ull;
                    }
                    if (s2 < kPrevQ / 64) {
                        qe[s2] = H.qe[q];
                        qk[s2] = H.qk[q];
                    }
                }
                if constexpr (kQExt) {
                    for (int q = 64 * VPL + (int)ln; q < qn; q += 64) {
                        M.qxe[q - 64 * VPL] = H.qe[q];
                        M.qxk[q - 64 * VPL] = H.qk[q];
                    }
                }
                vhi = CAP;
            } else {
                // vertex and plane indices: ten bits each there, wider here
                // above 1024 vertices
                auto wide = [](uint32_t x) -> W {
                    if constexpr (T::kNarrow) return (W)x;
                    else return T::pack3(x & 1023u, (x >> 10) & 1023u, (x >> 20) & 1023u);
                };
                for (int q = tid; q < vhi; q += step) {
                    M.y0[q] = H.y0[q];
                    M.y1[q] = H.y1[q];
                    M.y2[q] = H.y2[q];
                    M.ev[q] = H.ev[q];
                    M.vt[q] = wide(H.vt[q]);
                    M.va[q] = wide(H.va[q]);
                }
                for (int q = tid; q < qn; q += step) {
                    M.qe[q] = H.qe[q];
                    M.qk[q] = H.qk[q];
                }
                if (tid < nsv()) M.alive[tid] = H.alive[tid];
            }
            sync();
            update_bounds();
        }
    }

    // ------------------------------------------------------------ output
    // FP64 position of a vertex (relative to the site) from its three planes.
    __device__ void pos64(W t, float fx, float fy, float fz, double* y) const {
        double n[3], det;
        cramer64(plane64(T::fld(t, 0)), plane64(T::fld(t, 1)), plane64(T::fld(t, 2)), n, &det);
        if (det != 0.0) {
            double inv = 1.0 / det;
            y[0] = n[0] * inv; y[1] = n[1] * inv; y[2] = n[2] * inv;
        } else {
            y[0] = fx; y[1] = fy; y[2] = fz;
        }
    }

    // Writes the cell's record.  Returns false if the vertex/facet structure
    // is not a closed simple polytope (the caller then rebuilds the cell).
    // The planes are compacted by the group, the record written by its first
    // wave.
    __device__ bool finalize(uint32_t slot, uint32_t orig) {
        gc();
        bool ok = true;
        if (lead()) ok = finalize_lead(slot, orig);
        if constexpr (G > 1) ok = bcast(ok ? 1u : 0u) != 0;
        return ok;
    }
    __device__ bool finalize_lead(uint32_t slot, uint32_t orig) {
        const int F = np;
        const int ns = nsv();
        // facet order: ascending output code (box faces -6..-1, then original site ids)
        const uint32_t* order = cold_args()->order;
        for (int q = ln; q < F; q += 64) {
            int32_t c = M.pcode[q];
            M.key[q] = c >= 0 ? (int32_t)order[c] : c;
        }
        wsync();
        for (int q = ln; q < F; q += 64) {
            int32_t mine = M.key[q];
            uint32_t r = 0;
            for (int t = 0; t < F; ++t) r += M.key[t] < mine ? 1u : 0u;
            M.ta[q] = r;
            M.tb[q] = 0;
            M.anchor[q] = 0xFFFFFFFFu;
        }
        Stage st;
        {
            KArgs* ka = cold_args();
            st.cap = ka->stage.cap;
            st.vert = ka->stage.vert;
            st.tri64 = ka->stage.tri64;
            st.code = ka->stage.code;
            st.fsize = ka->stage.fsize;
            st.fv = ka->stage.fv;
        }
        int32_t* codes = st.code + (int64_t)slot * st.cap;
        for (int q = ln; q < F; q += 64) codes[M.ta[q]] = M.key[q];
        // vertex renumbering 0..nv-1 (slot-major)
        uint32_t nv = 0;
        int s0 = -1;
#pragma unroll
        for (int s = 0; s < (kReg ? VPL : ns); ++s) {
            const uint64_t al = alive[s];
            if (s0 < 0 && al) s0 = s;
            if ((al >> ln) & 1) M.sor[s * 64 + ln] = nv + mbcnt(al);
            nv += popc(al);
        }
        wsync();
        if (s0 < 0) return false;
        // reference point of the tetrahedral fan: vertex 0, in FP64
        double ref[3] = {0.0, 0.0, 0.0};
        {
            const int l0 = lowest(alive[s0]);
            double y[3] = {0.0, 0.0, 0.0};
            if constexpr (kReg) {
#pragma unroll
                for (int s = 0; s < VPL; ++s)
                    if (s == s0 && (int)ln == l0) pos64(vt[s], y0[s], y1[s], y2[s], y);
            } else {
                if ((int)ln == l0) pos64(vt[s0], y0[s0], y1[s0], y2[s0], y);
            }
            for (int c = 0; c < 3; ++c) ref[c] = __shfl(y[c], l0);
        }
        // every neighbour must be a live vertex (its new number is then < nv;
        // numbers left from dead vertices are not trusted)
        bool bad = false;
#pragma unroll
        for (int s = 0; s < (kReg ? VPL : ns); ++s) {
            if ((alive[s] >> ln) & 1) {
                const W a = va[s];
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    const uint32_t u = T::fld(a, e);
                    bad |= !is_alive(u);
                }
            }
        }
        if (ballot(bad)) return false;
        float4* vout = st.vert + (int64_t)slot * st.cap;
        uint64_t* tri64 = st.tri64 ? st.tri64 + (int64_t)slot * st.cap : nullptr;
        const double p64[3] = {(double)px, (double)py, (double)pz};
#pragma unroll
        for (int s = 0; s < (kReg ? VPL : ns); ++s) {
            if ((alive[s] >> ln) & 1) {
                const W t = vt[s], a = va[s];
                uint32_t t0 = M.ta[T::fld(t, 0)], t1 = M.ta[T::fld(t, 1)], t2 = M.ta[T::fld(t, 2)];
                uint32_t a0 = M.sor[T::fld(a, 0)], a1 = M.sor[T::fld(a, 1)], a2 = M.sor[T::fld(a, 2)];
                const uint32_t v = M.sor[s * 64 + ln];
                M.vtri[v] = T::pack3(t0, t1, t2);
                M.vadj[v] = T::pack3(a0, a1, a2);
                double y[3];
                pos64(t, y0[s], y1[s], y2[s], y);
                M.vpx[v] = y[0] - ref[0];
                M.vpy[v] = y[1] - ref[1];
                M.vpz[v] = y[2] - ref[2];
                uint32_t u0 = t0, u1 = t1, u2 = t2, tmp;
                if (u0 > u1) { tmp = u0; u0 = u1; u1 = tmp; }
                if (u1 > u2) { tmp = u1; u1 = u2; u2 = tmp; }
                if (u0 > u1) { tmp = u0; u0 = u1; u1 = tmp; }
                const uint32_t packed = tri64 ? 0u : (u0 | (u1 << 10) | (u2 << 20));
                vout[v] = make_float4((float)(p64[0] + y[0]), (float)(p64[1] + y[1]), (float)(p64[2] + y[2]),
                                      __uint_as_float(packed));
                if (tri64) tri64[v] = (uint64_t)u0 | ((uint64_t)u1 << 21) | ((uint64_t)u2 << 42);
                atomicAdd(&M.tb[t0], 1u);
                atomicAdd(&M.tb[t1], 1u);
                atomicAdd(&M.tb[t2], 1u);
                atomicMin(&M.anchor[t0], v);
                atomicMin(&M.anchor[t1], v);
                atomicMin(&M.anchor[t2], v);
            }
        }
        wsync();
        // facet rings in output (rank) order, counter-clockwise seen from outside;
        // sizes and anchors (lowest vertex) are indexed by facet rank
        uint16_t* fs = st.fsize + (int64_t)slot * st.cap;
        uint16_t* fvp = st.fv + (int64_t)slot * 3 * st.cap;
        uint32_t carry = 0;
        for (int r0 = 0; r0 < F; r0 += 64) {
            const uint32_t r = (uint32_t)(r0 + (int)ln);
            uint32_t sz = r < (uint32_t)F ? M.tb[r] : 0u;
            uint32_t x = sz;
            for (int o = 1; o < 64; o <<= 1) {
                uint32_t y = __shfl_up(x, o);
                if ((int)ln >= o) x += y;
            }
            if (r < (uint32_t)F) {
                fs[r] = (uint16_t)sz;
                const uint32_t base = carry + x - sz, start = M.anchor[r];
                if (sz < 3 || start >= nv) {
                    bad = true;
                } else {
                    uint32_t v = start, t = 0;
                    do {
                        fvp[base + t] = (uint16_t)v;
                        ++t;
                        W tri = M.vtri[v], adj = M.vadj[v];
                        uint32_t k = T::fld(tri, 0) == r ? 0u : (T::fld(tri, 1) == r ? 1u : 2u);
                        v = T::fld(adj, (k + 1) % 3);
                    } while (v != start && t < sz && v < nv);
                    bad |= (v != start) || (t != sz);
                }
            }
            carry += (uint32_t)__shfl(x, 63);
        }
        if (ballot(bad)) return false;
        // volume and centroid from the tetrahedra (ref, anchor_f, v, next_f(v)),
        // accumulated in FP64 (thin cells cancel badly in FP32)
        double vol6 = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
        for (uint32_t v = ln; v < nv; v += 64) {
            const double Px = M.vpx[v], Py = M.vpy[v], Pz = M.vpz[v];
            W tri = M.vtri[v], adj = M.vadj[v];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                uint32_t an = M.anchor[T::fld(tri, k)];
                uint32_t nx = T::fld(adj, (k + 1) % 3);
                if (an == v || nx == an) continue;
                const double Qx = M.vpx[an], Qy = M.vpy[an], Qz = M.vpz[an];
                const double Nx = M.vpx[nx], Ny = M.vpy[nx], Nz = M.vpz[nx];
                // det(anchor, v, next) relative to the reference vertex
                double cx = Py * Nz - Pz * Ny, cy = Pz * Nx - Px * Nz, cz = Px * Ny - Py * Nx;
                double det = Qx * cx + Qy * cy + Qz * cz;
                vol6 += det;
                mx += det * (Qx + Px + Nx);
                my += det * (Qy + Py + Ny);
                mz += det * (Qz + Pz + Nz);
            }
        }
        vol6 = wsum64(vol6);
        mx = wsum64(mx);
        my = wsum64(my);
        mz = wsum64(mz);
        uint32_t nbox = 0;
        for (int q = ln; q < F; q += 64) nbox += M.key[q] < 0 ? 1u : 0u;
        nbox = wsum_u(nbox);
        count(kCtrFinal, nv);
        if (ln == 0) {
            KArgs* ka = cold_args();
            ka->cnt_v[orig] = nv;
            ka->cnt_f[orig] = (uint32_t)F;
            ka->cnt_n[orig] = (uint32_t)F - nbox;
            ka->vol[orig] = (float)(vol6 / 6.0);
            double inv = vol6 != 0.0 ? 0.25 / vol6 : 0.0;
            ka->cen[3 * orig] = (float)(p64[0] + ref[0] + mx * inv);
            ka->cen[3 * orig + 1] = (float)(p64[1] + ref[1] + my * inv);
            ka->cen[3 * orig + 2] = (float)(p64[2] + ref[2] + mz * inv);
            ka->flags[orig] = (uint8_t)flags;
            ka->loc[self] = make_loc((uint32_t)A.tier, slot);
        }
        return true;
    }

    __device__ void write_empty(uint32_t orig, uint32_t extra) {
        if (ln == 0 && lead()) {
            KArgs* ka = cold_args();
            ka->cnt_v[orig] = 0;
            ka->cnt_f[orig] = 0;
            ka->cnt_n[orig] = 0;
            ka->vol[orig] = 0.f;
            ka->cen[3 * orig] = px;
            ka->cen[3 * orig + 1] = py;
            ka->cen[3 * orig + 2] = pz;
            ka->flags[orig] = (uint8_t)(flags | kFlagEmpty | extra);
            ka->loc[self] = make_loc((uint32_t)A.tier, 0);
        }
    }
};

// The work loop shared by every tier (per wave, or per wave group with gx
// its exchange tables).
template <int VPL, bool kLds, bool kCount, int G = 1, bool kSoS = false, bool kW = true, bool kOpt = true>
__device__ void run_cells(WaveMem<VPL>& M, const ClipArgs& A, uint32_t* gx) {
    KArgs* ka = cold_args();
    // the input checks (non-finite values, a flat box) ran before this pass:
    // on such input no cell is built
    if (*ka->err != 0u) return;
    const uint32_t count = ka->list ? *ka->list_count : (uint32_t)A.n;
    if (count == 0) return;  // a larger pass with no cell
    Cell<VPL, kLds, kCount, G, kSoS, kW, kOpt> C(M, A, gx);
    unsigned long long st_empty = 0, st_large = 0, st_unc = 0, st_fail = 0, st_fp64 = 0, st_res = 0, st_pert = 0;
    // Cells are split into kWorkRanges contiguous (Morton-ordered) ranges, one
    // per XCD: the waves of workgroup b take chunks of their own range b % 8
    // first, so neighbouring cells (which walk the same nodes and sites) share
    // one L2, then help the other ranges.  A worker claims one cell at a time:
    // in the later passes, which get the few cells that overflowed, claiming
    // several made one worker build several large cells in a row while others
    // idled, and in the first pass single claims also end the pass sooner.
    uint32_t r = blockIdx.x % kWorkRanges;
    int tried = 0;
    uint32_t cur = 0, end = 0;
    for (;;) {
        if (cur >= end) {
            bool got = false;
            while (tried < kWorkRanges) {
                const uint32_t lo = (uint32_t)((uint64_t)count * r / kWorkRanges);
                const uint32_t hi = (uint32_t)((uint64_t)count * (r + 1) / kWorkRanges);
                uint32_t c0 = 0;
                if (C.ln == 0 && C.lead()) c0 = atomicAdd(&cold_args()->work_counter[r], 1u);
                c0 = C.bcast(c0);
                if (c0 < hi - lo) {
                    cur = lo + c0;
                    end = cur + 1;
                    got = true;
                    break;
                }
                r = (r + 1) % kWorkRanges;
                ++tried;
            }
            if (!got) break;
        }
        const uint32_t c = cur++;
        KArgs* kc = cold_args();
        if (kc->list && c >= kc->slots) {
            // no staging slot: left undone and counted (the build runs the
            // passes again with more slots)
            if (C.ln == 0 && C.lead()) atomicAdd(kc->deferred, 1u);
            continue;
        }
        const uint32_t k = kc->list ? kc->list[c] : c;
        const uint32_t slot = kc->list ? c : k;
        const uint32_t orig = kc->order[k];
        // a cell the previous pass handed over goes on from where it stopped
        using CellT = Cell<VPL, kLds, kCount, G, kSoS, kW, kOpt>;
        const typename CellT::HIn* hin = nullptr;
        if constexpr (CellT::kResumes) {
            if (kc->hand_in && c < kc->hand_in_cap) {
                const auto* h = static_cast<const typename CellT::HIn*>(kc->hand_in) + c;
                if (h->valid) hin = h;
            }
        }
        // a cell is built with plain FP32 signs first (mixed mode: with FP64
        // re-evaluation of doubtful ones); if that meets an inconsistent
        // configuration it is rebuilt with the FP64 re-evaluation, then with
        // every sign in FP64
        C.robust = A.precision == 2 ? 1 : 0;
        bool done = false, escalated = false, loser = false;
        for (int attempt = 0; attempt < 3 && !done; ++attempt) {
            const bool res = attempt == 0 && hin != nullptr;
            if (res) {
                C.resume(k, *hin);
                ++st_res;
            } else if (!C.init(k)) {
                loser = true;
                break;
            }
            if (attempt > 0) C.flags |= kFlagFP64;
            if (A.tier > 0) C.flags |= kFlagLarge;
            const uint64_t t0 = C.tic();
            int r = C.traverse(res, res ? hin->leaf : 0u, res ? hin->mask : 0ull, res ? hin->phase : 1u,
                               res ? hin->skip : kNoParent);
            C.toc(kCtrCycTraverse, t0);
            if (r == kRestart) {
                C.robust = C.robust + 1;
                continue;
            }
            if (r == kOverflow) {
                KArgs* kn = cold_args();
                if (kn->next_list) {
                    uint32_t pos = 0;
                    if (C.ln == 0 && C.lead()) {
                        pos = atomicAdd(kn->next_count, 1u);
                        kn->next_list[pos] = k;
                    }
                    if constexpr (CellT::kSaves) {
                        pos = C.bcast(pos);
                        if (kn->hand_out && pos < kn->hand_out_cap)
                            C.save(static_cast<typename CellT::HOut*>(kn->hand_out)[pos]);
                    }
                    escalated = true;
                } else {
                    C.write_empty(orig, kFlagFailed);
                    ++st_fail;
                    ++st_empty;
                }
                done = true;
                break;
            }
            if (r == kEmptied) {
                C.write_empty(orig, 0);
                ++st_empty;
                done = true;
            } else if ([&] {
                           const uint64_t t1 = C.tic();
                           const bool ok = C.finalize(slot, orig);
                           C.toc(kCtrCycFinal, t1);
                           return ok;
                       }()) {
                done = true;
            } else if (C.robust < 2) {
                C.robust = C.robust + 1;
            } else {
                break;
            }
        }
        if (loser) {
            C.write_empty(orig, 0);
            ++st_empty;
            continue;
        }
        if (escalated) continue;
        if (!done) {
            // still inconsistent after the robust rebuilds: report an empty cell
            C.write_empty(orig, kFlagFailed | kFlagUncertain);
            ++st_fail;
            ++st_empty;
        }
        st_large += (C.flags & kFlagLarge) ? 1 : 0;
        st_unc += (C.flags & kFlagUncertain) ? 1 : 0;
        st_fp64 += (C.flags & kFlagFP64) ? 1 : 0;
        st_pert += (C.flags & kFlagPerturbed) ? 1 : 0;
    }
    if (C.ln == 0 && C.lead()) {
        ka = cold_args();
        if constexpr (kCount)
            for (int c = 0; c < kCtrCount; ++c)
                if (C.ctr[c]) atomicAdd(&ka->ctr[c], (unsigned long long)C.ctr[c]);
        if (st_empty) atomicAdd(&ka->stats[kStatEmpty], st_empty);
        if (st_large) atomicAdd(&ka->stats[kStatLarge], st_large);
        if (st_unc) atomicAdd(&ka->stats[kStatUncertain], st_unc);
        if (st_fail) atomicAdd(&ka->stats[kStatFailed], st_fail);
        if (st_fp64) atomicAdd(&ka->stats[kStatFP64], st_fp64);
        if (st_res) atomicAdd(&ka->stats[kStatResumed], st_res);
        if (st_pert) atomicAdd(&ka->stats[kStatPerturbed], st_pert);
    }
}

#pragma clang attribute pop

// Register tiers: per-cell arrays in LDS, WAVES independent waves per
// block.  Register budgets: the 64-vertex pass is held to 128 registers for
// 4 waves per SIMD (a few spills cost less than the lost occupancy: the pass
// issues VALU work back to back), the 128-vertex pass to 256 for 2 (its
// cells are fewer and longer: at 3 waves per SIMD the spills of its two
// slots made each cell slower than the occupancy gained).
template <int VPL, int WAVES, bool kCount, bool kSoS = false, bool kW = true, bool kOpt = true>
__global__ __launch_bounds__(64 * WAVES, VPL == 1 ? 4 : 2) void k_clip(ClipArgs A) {
    __shared__ WaveMem<VPL> mem[WAVES];
    run_cells<VPL, true, kCount, 1, kSoS, kW, kOpt>(mem[threadIdx.x >> 6], A, nullptr);
}

// Waves per cell in the 1024-vertex (LDS) and 16384-vertex (arena) tiers.
constexpr int kGroupLds = 4;
constexpr int kGroupArena = 8;

// 1024-vertex tier: the kGroupLds waves of a block build one cell, its
// arrays in LDS (one block per CU).
template <bool kCount, bool kSoS = false>
__global__ __launch_bounds__(64 * kGroupLds, 1) void k_clip_lds(ClipArgs A) {
    __shared__ WaveMem<16> mem;
    __shared__ uint32_t gx[2 * kGroupLds * 8];
    run_cells<16, true, kCount, kGroupLds, kSoS>(mem, A, gx);
}

// 16384-vertex tier: the kGroupArena waves of a block build one cell, its
// arrays in arena[blockIdx.x].
constexpr int kArenaVPL = kTierCap[3] / 64;
template <bool kCount, bool kSoS = false>
__global__ __launch_bounds__(64 * kGroupArena) void k_clip_arena(ClipArgs A, WaveMem<kArenaVPL>* arena) {
    __shared__ uint32_t gx[2 * kGroupArena * 8];
    run_cells<kArenaVPL, false, kCount, kGroupArena, kSoS>(arena[blockIdx.x], A, gx);
}

static_assert(kTierCap[0] == 64 && kTierCap[1] == 128 && kTierCap[2] == 1024,
              "the LDS tiers are instantiated for 64, 256 and 1024 vertices");
static_assert(sizeof(WaveMem<16>) + 2 * kGroupLds * 8 * sizeof(uint32_t) <= 160 * 1024,
              "the 1024-vertex tier must fit the LDS of one CU");
static_assert(Tier<kArenaVPL>::CAP <= (1 << Tier<kArenaVPL>::kB) && Tier<kArenaVPL>::CAP <= (1 << 16),
              "arena-tier indices must fit their packings and the 16-bit staged facet lists");

}  // namespace

size_t arena_bytes_per_worker() { return sizeof(WaveMem<kArenaVPL>); }

size_t handoff_bytes(int tier) {
    switch (tier) {
        case 0: return sizeof(HandoffT<kTierCap[0], kQueue0>);
        case 1: return sizeof(HandoffT<kTierCap[1], kQueue0>);
        case 2: return sizeof(HandoffT<kTierCap[2]>);
        default: return 0;
    }
}

int clip_grid_workers(int tier, int num_cu) {
    int per_cu = 0;
    hipError_t e = hipSuccess;
    if (tier == 0) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_clip<1, 4, false>, 256, 0);
        per_cu *= 4;
    } else if (tier == 1) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_clip<2, 2, false>, 128, 0);
        per_cu *= 2;
    } else if (tier == 2) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_clip_lds<false>, 64 * kGroupLds, 0);
        if (e == hipSuccess && per_cu > 0) return per_cu * num_cu;
        return num_cu;
    } else {
        return num_cu;  // arena groups: one per CU, bounded by arena memory
    }
    if (e != hipSuccess || per_cu < 1) per_cu = 4;
    return per_cu * num_cu;
}

template <bool kCount, bool kSoS>
void launch_tier(const ClipArgs& a, int workers, void* arena, hipStream_t s) {
    // the register passes have instantiations with the default search options fixed
    const bool def = a.culling == 3 && a.traversal == 1 && a.warm_start == 0;
    switch (a.tier) {
        case 0:
            if (kSoS || !def)
                hipLaunchKernelGGL((k_clip<1, 4, kCount, kSoS>), dim3((workers + 3) / 4), dim3(256), 0, s, a);
            else if (a.weighted)
                hipLaunchKernelGGL((k_clip<1, 4, kCount, false, true, false>), dim3((workers + 3) / 4), dim3(256), 0, s, a);
            else
                hipLaunchKernelGGL((k_clip<1, 4, kCount, false, false, false>), dim3((workers + 3) / 4), dim3(256), 0, s, a);
            break;
        case 1:
            if (kSoS || !def)
                hipLaunchKernelGGL((k_clip<2, 2, kCount, kSoS>), dim3((workers + 1) / 2), dim3(128), 0, s, a);
            else if (a.weighted)
                hipLaunchKernelGGL((k_clip<2, 2, kCount, false, true, false>), dim3((workers + 1) / 2), dim3(128), 0, s, a);
            else
                hipLaunchKernelGGL((k_clip<2, 2, kCount, false, false, false>), dim3((workers + 1) / 2), dim3(128), 0, s, a);
            break;
        case 2:
            hipLaunchKernelGGL((k_clip_lds<kCount, kSoS>), dim3(workers), dim3(64 * kGroupLds), 0, s, a);
            break;
        default:
            hipLaunchKernelGGL((k_clip_arena<kCount, kSoS>), dim3(workers), dim3(64 * kGroupArena), 0, s, a,
                               static_cast<WaveMem<kArenaVPL>*>(arena));
            break;
    }
}

hipError_t launch_clip(const ClipArgs& a, int workers, void* arena, hipStream_t s) {
    if (a.tier >= 3 && !arena) return hipErrorInvalidValue;
    if (workers < 1) return hipErrorInvalidValue;
    // the perturbed build has no counting instantiation (counters stay zero)
    if (a.perturb) launch_tier<false, true>(a, workers, arena, s);
    else if (a.ctr) launch_tier<true, false>(a, workers, arena, s);
    else launch_tier<false, false>(a, workers, arena, s);
    return hipGetLastError();
}

}  // namespace vd
