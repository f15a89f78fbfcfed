// Internal declarations shared by the libvd translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vd {

// ---------------------------------------------------------------- limits

constexpr int kMaxLeaf = 64;                 // leaf refs store count-1 in 6 bits
constexpr int64_t kMaxSites = int64_t(1) << 25;  // leaf refs store `first` in 25 bits
constexpr int kDefaultLeaf = 32;
// Work distribution of the clip kernels: one contiguous range of cells per
// XCD (workgroup b runs on XCD b % 8), claimed one cell at a time.
constexpr int kWorkRanges = 8;
// Vertex (= plane) capacity of a cell in each clipping pass.
constexpr int kTiers = 4;
constexpr int kTierCap[kTiers] = {64, 128, 1024, 16384};

// ---------------------------------------------------------------- BVH

// One child of a binary BVH node: its box, the largest weight of the sites
// below it (the power-diagram augmentation of paper Sec. 4.3) and a
// reference.  A reference with bit 31 set is a leaf: bits 0..24 hold the
// first site (Morton order) and bits 25..30 the site count minus one;
// otherwise it is the index of an internal node.  Each internal node holds
// both children's records side by side (64 bytes) so one visit reads one
// contiguous block.
struct __align__(16) NodeChild {
    float lo[3];
    float wmax;
    float hi[3];
    uint32_t ref;
};
struct __align__(16) Node {
    NodeChild c[2];
};

constexpr uint32_t kLeafBit = 0x80000000u;
constexpr uint32_t kNoParent = 0xFFFFFFFFu;  // parent link of the root
__host__ __device__ inline uint32_t leaf_ref(uint32_t first, uint32_t count) {
    return kLeafBit | ((count - 1u) << 25) | first;
}
__host__ __device__ inline bool ref_is_leaf(uint32_t r) { return (r & kLeafBit) != 0; }
__host__ __device__ inline uint32_t leaf_first(uint32_t r) { return r & 0x1FFFFFFu; }
__host__ __device__ inline uint32_t leaf_count(uint32_t r) { return ((r >> 25) & 63u) + 1u; }

// ---------------------------------------------------------------- staging

// Finished cells are written to fixed-capacity slots before the CSR pass.
// Capacity `cap` = vertices = planes per cell; facet-vertex lists hold 3 cap.
//   vert[slot*cap + v]   : global position xyz, .w = the vertex's three facet
//                          ranks (ascending, 10 bits each) as raw bits, unless
//                          tri64 is set (cap > 1024)
//   tri64[slot*cap + v]  : the three facet ranks, 21 bits each (or null)
//   code[slot*cap + f]   : facet codes in ascending order (site ids, box -1..-6)
//   fsize[slot*cap + f]  : vertices of facet f
//   fv[slot*3cap + t]    : cell-local vertex indices of all facets, concatenated
struct Stage {
    int cap;
    float4* vert;
    uint64_t* tri64;
    int32_t* code;
    uint16_t* fsize;
    uint16_t* fv;
};

// Location of a cell's staged record: tier in bits 30..31, slot below.
__host__ __device__ inline uint32_t make_loc(uint32_t tier, uint32_t slot) { return (tier << 30) | slot; }

// Per-cell flag bits (mirror vd.h)
constexpr uint32_t kFlagEmpty = 1u, kFlagFP64 = 2u, kFlagLarge = 4u, kFlagUncertain = 8u, kFlagFailed = 16u,
                   kFlagPerturbed = 32u;

// Build statistics accumulated by the clip kernels (device, uint64 each).
enum StatIndex { kStatEmpty = 0, kStatLarge, kStatUncertain, kStatFailed, kStatFP64, kStatResumed, kStatPerturbed,
                 kStatCount };
// Work counters (mirror VD_CTR_* in vd.h).
enum CtrIndex { kCtrClassify = 0, kCtrNewVertex, kCtrNode, kCtrSite, kCtrFinal, kCtrClip, kCtrEffective, kCtrLeaf,
                kCtrBall, kCtrFP64, kCtrCycTraverse, kCtrCycLeaf, kCtrCycClip, kCtrCycFinal, kCtrCount };

// State of a cell that outgrew a clipping pass while clipping by the sites
// of a leaf, handed to the next pass so that the cell goes on from there
// instead of starting over: vertices (same numbering; indices packed ten bits
// each, as in every pass up to 1024 vertices), planes, node queue, and the
// leaf with its candidates not yet tried.  phase 0: the leaf was the site's
// own leaf, clipped before any walk (the next pass finishes it, then walks
// from the root passing over it); 1: a leaf of the walk (the next pass
// finishes it, then goes on with the queue).  HC: vertex capacity of the
// pass that writes the record, QC: its queue capacity (larger than HC in the
// 64-vertex pass).
constexpr int kMaxWarm = 16;       // largest K of the KNN warm start
template <int HC, int QC = HC>
struct HandoffT {
    float4 pl[HC];            // planes: a.xyz, b
    float4 psite[HC];         // the plane's site
    unsigned long long alive[HC / 64];
    unsigned long long mask;  // candidates of the leaf still to try (lanes)
    float y0[HC], y1[HC], y2[HC], ev[HC];
    uint32_t vt[HC], va[HC];
    float psb[HC];
    int32_t pcode[HC];
    uint32_t qe[QC];          // node queue (QC: the writer's queue capacity)
    float qk[QC];
    uint32_t valid;           // 1: the state above can be resumed
    uint32_t np, vhi, qn, flags, robust, leaf, phase;
    uint32_t skip;            // a leaf the walk must pass over (already clipped), or kNoParent
    uint32_t nwarm;           // sites of the KNN warm start (passed over by the leaves)
    uint32_t wsite[kMaxWarm];
};
// Bytes of the hand-over record that the pass of tier t writes (t < kTiers - 1).
size_t handoff_bytes(int tier);

struct ClipArgs {
    const float4* pts;        // sites in Morton order: x, y, z, w (w = -inf: coincident loser)
    const uint32_t* order;    // Morton position -> original index
    const Node* nodes;        // internal nodes (n-1)
    uint32_t root;            // root reference
    const uint32_t* up;       // [n-1] parent link of each internal node: (parent << 1) | which child
    const uint32_t* leaf_of;  // [n] by Morton position: (node << 1) | which child holds the site's leaf
                              // (null when the root is a leaf)
    const float* bbox;        // device [6]: lo.xyz, hi.xyz
    int64_t n;
    int leaf_size;
    int culling;              // 1 directional, 2 isotropic
    int traversal;            // 1 best-first, 2 depth-first
    int warm_start;           // K of the KNN warm start (0: none)
    int precision;            // 1 fp32, 2 mixed
    int perturb;              // 1: exact ties decided by symbolic perturbation of the weights
    int weighted;             // 0: no weights were given (every weight is zero)
    int tier;                 // 0..3 (capacity kTierCap[tier])
    // work: cells c in [0, count) are list[c] (or c itself when list == null),
    // split into kWorkRanges contiguous ranges with one counter each (zeroed)
    uint32_t* work_counter;
    const uint32_t* list;
    const uint32_t* list_count;   // device count (list != null), else count = n
    uint32_t slots;           // staging slots of this pass (list tiers: cells at
                              // list positions from slots on are left undone)
    uint32_t* deferred;       // counts the cells left undone
    uint32_t* next_list;      // escalation list for the next tier (null: last tier)
    uint32_t* next_count;
    // hand-over records (HandoffT of this pass's capacity) written for the
    // cells this pass escalates, at their position in next_list, for
    // positions below hand_out_cap (null: none); and those the previous pass
    // wrote, read for the cells of this pass's list below hand_in_cap
    void* hand_out;
    uint32_t hand_out_cap;
    const void* hand_in;
    uint32_t hand_in_cap;
    Stage stage;
    uint32_t* loc;            // [n] by Morton position
    uint32_t* cnt_v;          // [n] by original index
    uint32_t* cnt_f;
    uint32_t* cnt_n;
    float* vol;               // [n] by original index
    float* cen;               // [3n]
    uint8_t* flags;           // [n]
    unsigned long long* stats;  // [kStatCount]
    unsigned long long* ctr;    // [kCtrCount] work counters, or null
    const uint32_t* err;      // input error bits of this build (non-zero: do nothing)
};

struct WriteArgs {
    int64_t n;
    const uint32_t* inv;      // original index -> Morton position
    const uint32_t* loc;
    Stage stage[kTiers];
    const uint32_t* cnt_v;
    const uint32_t* cnt_f;
    const uint32_t* cnt_n;
    const int64_t* off_v;
    const int64_t* off_f;
    const int64_t* off_n;
    int32_t* nbr;
    int32_t* facet_nbr;
    int64_t* fv_off;
    int32_t* fv;
    float* vert;
    int32_t* vert_planes;
};

// Inputs and outputs of the backward pass over the last build.
struct BwdArgs {
    int64_t n;
    const float4* pts;        // sites in Morton order: x, y, z, w
    const uint32_t* inv;      // original index -> Morton position
    const uint32_t* loc;      // staged record of each cell, by Morton position
    Stage stage[kTiers];
    const uint32_t* cnt_v;    // by original index
    const uint32_t* cnt_f;
    const uint32_t* cnt_n;
    const int64_t* off_v;     // vertex and facet CSR offsets of the build
    const int64_t* off_f;
    const float* bbox;        // device [6]
    const float* g_vol;       // [n] or null
    const float* g_cen;       // [3n] or null
    const float* g_vert;      // [3 n_vert] or null
    // FP64 scratch: shares of neighbouring cells cancel to a much smaller
    // site gradient wherever cells are thin, so they are kept and summed in FP64
    double4* gf;              // [n_facet]: what a cell sends to its facet's site (dp xyz, dw)
    double4* gself;           // [n]: each cell's share for its own site
    double* orphan;           // [4n], zeroed: shares of facets not listed back
    float* g_xyz;             // [3n] out
    float* g_w;               // [n] out, or null
    // Box of the sites (the build was given no box): its faces move with the
    // extreme sites.  Each wave of the cell pass sums dL/db of the box faces
    // of its cells into box_part[wave * 6 + face]; box_sum[face] is their
    // total and box_arg[face] (preset to 0xFFFFFFFF) the lowest original
    // index of a site on that face.  moving_box = 0: faces held fixed.
    int moving_box;
    const float4* pts_orig;   // [n] sites in the caller's order
    double* box_part;         // [bwd_waves(n) * 6]
    double* box_sum;          // [6]
    uint32_t* box_arg;        // [6]
};

// Waves of the backward cell pass (the size of BwdArgs.box_part is six
// doubles per wave).
int64_t bwd_waves(int64_t n);

// ---------------------------------------------------------------- launches
// (host wrappers; each returns the hipError_t of its launch)

hipError_t launch_pack(const float* xyz, const float* w, int64_t n, float4* pts, uint32_t* err, hipStream_t s);
hipError_t launch_bbox(const float4* pts, int64_t n, float* partial, int nblk_max, float* bbox, uint32_t* err,
                       hipStream_t s);
hipError_t launch_check_bbox(float* bbox, uint32_t* err, hipStream_t s);
hipError_t launch_morton(const float4* pts, int64_t n, const float* bbox, uint64_t* keys, uint32_t* vals,
                         hipStream_t s);
// LSD radix sort of 64-bit keys with 32-bit values over `bits` low bits.
// tmp buffers: same sizes; hist: radix_hist_size(n) uint32.
size_t radix_hist_size(int64_t n);
hipError_t radix_sort(uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp, uint32_t* vals_tmp, int64_t n, int bits,
                      uint32_t* hist, uint32_t* scan_tmp, hipStream_t s, bool* result_in_tmp);
hipError_t launch_gather(const float4* pts, const uint32_t* order, int64_t n, float4* spts, uint32_t* inv,
                         hipStream_t s);
hipError_t launch_losers(float4* spts, const uint64_t* keys, const uint32_t* order, int64_t n, uint8_t* mark,
                         hipStream_t s);
// Binary radix tree over the sorted codes: children, ranges, and the parent
// link of every internal node ((parent << 1) | which child; kNoParent at the
// root).
hipError_t launch_karras(const uint64_t* keys, int64_t n, int2* child, uint32_t* up, int2* range, hipStream_t s);
// Child boxes and max weights of every internal node (range reductions over a
// sparse table of 64-site block boxes; table: box_table_size(n) entries), and
// the leaf record of every site ((node << 1) | which child, by Morton position).
size_t box_table_size(int64_t n);
hipError_t launch_bounds(const float4* spts, int64_t n, const int2* child, const int2* range, NodeChild* table,
                         Node* nodes, uint32_t* leaf_of, int leaf_size, hipStream_t s);

// Exclusive scan of uint32 counts into int64 offsets [n+1] (out[n] = total).
size_t scan_tmp_size(int64_t n);
hipError_t scan_counts(const uint32_t* in, int64_t n, int64_t* out, int64_t* tmp, hipStream_t s);
// Exclusive scan of uint32 -> uint32 (for radix histograms).
hipError_t scan_u32(const uint32_t* in, int64_t n, uint32_t* out, uint32_t* tmp, hipStream_t s);

// Cell workers to launch for a clipping pass (a wave in the two register
// tiers, a workgroup of waves sharing one cell in the two larger ones), and
// the per-worker arena the last pass (tier 3) needs: launch_clip(tier 3)
// takes workers * arena_bytes_per_worker().
int clip_grid_workers(int tier, int num_cu);
size_t arena_bytes_per_worker();
hipError_t launch_clip(const ClipArgs& a, int workers, void* arena, hipStream_t s);
hipError_t launch_set_i64(int64_t* dst, int64_t value, hipStream_t s);
hipError_t launch_write(const WriteArgs& a, hipStream_t s);

// Dual tetrahedra of the staged cells (see vd_tetrahedra): count per cell,
// then write rows at the scanned offsets.
struct TetArgs {
    int64_t n;
    const uint32_t* inv;      // original index -> Morton position
    const uint32_t* loc;
    Stage stage[kTiers];
    const uint32_t* cnt_v;
    uint32_t* cnt_t;          // [n] tetrahedra per cell (count pass)
    const int64_t* off_t;     // [n+1] their offsets (write pass)
    int32_t* tets;            // [4 * total] out
};
hipError_t launch_tet_count(const TetArgs& a, hipStream_t s);
hipError_t launch_tet_write(const TetArgs& a, hipStream_t s);
hipError_t launch_backward(const BwdArgs& a, hipStream_t s);

// Fixed device scratch of the allocation-free backward (vd_backward_noalloc):
// kBwdScratchBytes per device, its address looked up once per device with
// that device current (bwd_scratch_init) and kept.  dst[0, count) = value.
constexpr size_t kBwdScratchBytes = size_t(64) << 20;
hipError_t bwd_scratch_init(int device, void** ptr);
hipError_t launch_fill_u64(uint64_t* dst, int64_t count, uint64_t value, hipStream_t s);

}  // namespace vd
