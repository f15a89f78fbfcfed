/* vd.h -- C ABI of libvd: 3D Voronoi and power diagrams on one AMD MI355X.
 *
 * The library builds every cell of the power diagram of weighted sites
 * independently (paper Sec. 3, Eq. 1):
 *     C_i = B  intersected with  { x : |x-p_i|^2 - w_i <= |x-p_j|^2 - w_j  for all j != i }
 * by clipping the box B against the bisecting (radical) planes of candidate
 * sites (Sec. 4.1 and supplementary Sec. B).  Candidates come from a
 * best-first walk of a bounding-volume hierarchy whose nodes also carry the
 * largest weight below them (Sec. 4.3, Alg. 1), pruned by the directional
 * cell bounds of Sec. 4.2.1 and the node bound of Sec. 4.2.2.  With all
 * weights equal (or w == NULL) this is the Voronoi diagram.  Two sites are
 * neighbours when their cells share a facet of positive area (Sec. 3).
 *
 * Everything is plain C: pointers, sizes and status codes.  Device pointers
 * are HIP device memory of the context's device; `stream` is a hipStream_t
 * passed as void* (NULL = the null stream).  All work is ordered on that
 * stream.  No call throws; errors come back as a status, with a message from
 * vd_last_error() (thread-local, valid until the next call on that thread).
 *
 * Typical use:
 *     vd_context* ctx;  vd_create(0, &ctx);
 *     vd_sizes sz;      vd_build(ctx, xyz, w, n, bbox, NULL, stream, &sz);
 *     ... allocate vd_outputs arrays of the sizes in sz ...
 *     vd_write(ctx, &out, stream);
 *     vd_destroy(ctx);
 */
#ifndef VD_H
#define VD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VD_API __attribute__((visibility("default")))

typedef enum {
    VD_OK = 0,
    VD_ERR_INVALID_ARG = 1,  /* bad pointer, size, option or box; non-finite input */
    VD_ERR_HIP = 2,          /* a HIP runtime call failed */
    VD_ERR_OOM = 3,          /* device allocation failed */
    VD_ERR_STATE = 4,        /* vd_write / vd_backward without a successful vd_build */
    VD_ERR_CAPACITY = 5      /* some cell needed more than the largest capacity */
} vd_status;

/* Per-cell flag bits (vd_outputs.flags). */
#define VD_FLAG_EMPTY 1u      /* the cell is empty (power diagrams, coincident sites) */
#define VD_FLAG_FP64 2u       /* some predicate of this cell was re-evaluated in FP64 */
#define VD_FLAG_LARGE 4u      /* built by a larger-capacity pass */
#define VD_FLAG_UNCERTAIN 8u  /* FP32 clipping met an inconsistent configuration */
#define VD_FLAG_FAILED 16u    /* cell exceeded every capacity; outputs empty */
#define VD_FLAG_PERTURBED 32u /* some exact tie of this cell was decided by the
                                 symbolic perturbation (vd_options.perturb) */

/* Options; pass NULL for the defaults.  Zero in any field means its default. */
typedef struct vd_options {
    int32_t precision;  /* 1 = FP32 predicates (default), 2 = mixed FP32 / FP64 */
    int32_t leaf_size;  /* sites per BVH leaf, 1..64 (default 32) */
    int32_t culling;    /* 1 = directional (Sec. 4.2.1-4.2.2), 2 = isotropic radius,
                           3 = directional plus vertex power-ball node test and
                               exact plane-versus-cell-box site test (default) */
    int32_t traversal;  /* 1 = best-first (Alg. 1, default): the queued node of least
                           bound next; 2 = depth-first (ablation): the node queued
                           last next.  Both descend into the nearer child first and
                           clip a leaf's sites nearest plane first */
    int32_t profile;    /* 1 = record per-phase HIP-event timings (vd_get_timings) */
    int32_t counters;   /* 1 = count the method's work units (vd_get_counters) */
    int32_t warm_start; /* K = 1..16: KNN warm start (supplementary Sec. A): each cell is
                           first clipped by its K nearest sites, found by a best-first
                           query of the same BVH; 0 = none (default) */
    int32_t perturb;    /* 1 = symbolic perturbation of exact degeneracies: signs FP32
                           cannot decide are re-evaluated in FP64 as in the mixed form
                           (precision is taken as 2), then, where that evaluation is
                           exact (checked per operation; true for short dyadic
                           coordinates such as lattices) and zero, decided as for the
                           weights w_k + d^(k+1), d infinitesimal, k the original index
                           (Simulation of Simplicity, Edelsbrunner and Muecke 1990).
                           The result is then the diagram of that perturbed input, in
                           general position: every vertex joins three planes, and at
                           a vertex of five or more co-spherical sites the dual is a
                           proper regular triangulation.  Its geometry is the limit
                           d -> 0 (zero-area facets and coincident vertices where the
                           input is degenerate; such facets are listed and their
                           sites are neighbours).  Signs the checked evaluation cannot
                           settle stay flagged VD_FLAG_UNCERTAIN.  0 = off (default):
                           exact ties are kept inside (Sec. B's convention) */
} vd_options;

/* Phases reported by vd_get_timings (milliseconds, HIP events on `stream`). */
#define VD_PHASE_LBVH 0       /* packing, Morton codes, radix sort, tree, bounds */
#define VD_PHASE_CLIP 1       /* traversal + clipping, 64-vertex tier (one kernel) */
#define VD_PHASE_CLIP_LARGE 2 /* traversal + clipping, 128-, 1024- and 16384-vertex tiers */
#define VD_PHASE_SCAN 3       /* prefix sums of the per-cell counts */
#define VD_PHASE_BUILD 4      /* the whole vd_build, first to last device operation */
#define VD_PHASE_WRITE 5      /* vd_write (CSR write-out and copies) */
#define VD_PHASE_CLIP_TIER1 6 /* the 128-vertex tier alone (part of VD_PHASE_CLIP_LARGE) */
#define VD_PHASE_BACKWARD 7   /* vd_backward */
#define VD_PHASE_COUNT 8

/* Work units counted when vd_options.counters = 1.  vd_get_counters returns
 * them per capacity tier: entry k + VD_CTR_COUNT * t is unit k of tier t
 * (t = 0: 64 vertices, 1: 128, 2: 1024, 3: 16384; VD_TIERS tiers). */
#define VD_TIERS 4
#define VD_CTR_CLASSIFY 0     /* vertex-versus-plane side tests */
#define VD_CTR_NEW_VERTEX 1   /* vertices created by clipping */
#define VD_CTR_NODE_TEST 2    /* BVH child-box tests (Sec. 4.2.2) */
#define VD_CTR_SITE_TEST 3    /* per-site plane-distance tests in leaves (Sec. 4.2.1) */
#define VD_CTR_FINAL_VERTEX 4 /* vertices of the finished cells */
#define VD_CTR_CLIP 5         /* clip attempts (candidate planes that passed the tests) */
#define VD_CTR_CLIP_EFFECTIVE 6 /* clips that changed the cell */
#define VD_CTR_LEAF 7         /* leaves visited */
#define VD_CTR_BALL 8         /* vertex-versus-node-box power-ball tests (culling 3) */
#define VD_CTR_FP64 9         /* vertex side tests re-evaluated in FP64 (of VD_CTR_CLASSIFY) */
/* Shader clock cycles the waves spent (summed over waves, wall time of each
 * wave, so stalls included): the whole traversal of a cell, the leaves within
 * it, the clips within those, and finalizing the cell. */
#define VD_CTR_CYC_TRAVERSE 10
#define VD_CTR_CYC_LEAF 11
#define VD_CTR_CYC_CLIP 12
#define VD_CTR_CYC_FINAL 13
#define VD_CTR_COUNT 14

/* Result sizes of the last vd_build. */
typedef struct vd_sizes {
    int64_t n;          /* sites */
    int64_t n_nbr;      /* total neighbour entries */
    int64_t n_facet;    /* total facets (site and box facets) */
    int64_t n_vert;     /* total cell vertices (each cell lists its own) */
    int64_t n_fv;       /* total facet-vertex entries (= 3 n_vert) */
    int64_t n_empty;    /* empty cells */
    int64_t n_large;    /* cells built by the larger-capacity passes */
    int64_t n_uncertain;/* cells flagged VD_FLAG_UNCERTAIN */
    int64_t n_failed;   /* cells flagged VD_FLAG_FAILED (status VD_ERR_CAPACITY) */
    int64_t n_fp64;     /* cells with at least one FP64 re-evaluation */
    int64_t n_huge;     /* cells that needed the 16384-vertex pass */
    int64_t n_resumed;  /* cells a larger pass took over from the previous
                           pass where that one stopped, rather than anew */
    int64_t n_perturbed;/* cells flagged VD_FLAG_PERTURBED */
} vd_sizes;

/* Output arrays: caller-owned device memory, sized from vd_sizes.  Rows are
 * in the caller's original site order.  Any pointer may be NULL to skip it.
 *   nbr_off   int64[n+1]      neighbour rows (CSR offsets)
 *   nbr       int32[n_nbr]    neighbour site ids, ascending per row
 *   facet_off int64[n+1]      facet rows
 *   facet_nbr int32[n_facet]  per facet: site id (>= 0) or box face
 *                             -1..-6 = x_min, x_max, y_min, y_max, z_min, z_max;
 *                             ascending per row (box facets first)
 *   fv_off    int64[n_facet+1] vertices of each facet (CSR offsets into fv)
 *   fv        int32[n_fv]     global vertex indices (rows of `vert`),
 *                             counter-clockwise seen from outside the cell,
 *                             starting at the cell's lowest vertex index
 *   vert_off  int64[n+1]      vertex rows
 *   vert      float[n_vert*3] vertex positions
 *   vert_planes int32[n_vert*3] the three facet codes meeting at the vertex,
 *                             ascending (same coding as facet_nbr)
 *   vol       float[n]        cell volume
 *   centroid  float[n*3]      cell centroid (the site itself for empty cells)
 *   flags     uint8[n]        VD_FLAG_* bits
 */
typedef struct vd_outputs {
    int64_t* nbr_off;
    int32_t* nbr;
    int64_t* facet_off;
    int32_t* facet_nbr;
    int64_t* fv_off;
    int32_t* fv;
    int64_t* vert_off;
    float* vert;
    int32_t* vert_planes;
    float* vol;
    float* centroid;
    uint8_t* flags;
} vd_outputs;

typedef struct vd_context vd_context;

/* Create a context on HIP device `device`.  The context owns the device
 * scratch reused across builds (it grows as needed and is released by
 * vd_destroy).  A context is not thread-safe: use one per thread. */
VD_API vd_status vd_create(int device, vd_context** ctx);
VD_API void vd_destroy(vd_context* ctx);

/* Build the diagram.
 *   xyz   device float[n*3], row-major site positions (borrowed, read only)
 *   w     device float[n] weights, or NULL for the Voronoi diagram
 *   n     1 <= n <= 33554432
 *   bbox  HOST float[6] = {xmin, ymin, zmin, xmax, ymax, zmax}, the initial
 *         cell of every site (supplementary Sec. B starts from the sites'
 *         bounding box); NULL = the sites' bounding box.  Sites may lie
 *         outside it.  Each extent must be positive.
 *   opt   NULL for defaults
 *   sizes receives the output sizes
 * Non-finite coordinates or weights give VD_ERR_INVALID_ARG.  Host-blocking:
 * it synchronises `stream` to learn the output sizes.  The result stays in
 * the context until the next vd_build. */
VD_API vd_status vd_build(vd_context* ctx, const float* xyz, const float* w, int64_t n, const float* bbox,
                          const vd_options* opt, void* stream, vd_sizes* sizes);

/* Write the last build's diagram into caller-allocated device arrays (sizes
 * from vd_build).  Stream-ordered, does not synchronise. */
VD_API vd_status vd_write(vd_context* ctx, const vd_outputs* out, void* stream);

/* Gradients of L = sum_i g_vol[i] V_i + g_cen[i] . c_i + sum_v g_vert[v] . x_v
 * with respect to the site positions and weights of the last build, through
 * its combinatorics (facets and vertex plane-triples held fixed; the
 * derivatives of Sec. 3, Eq. 1 under a motion of the bisecting planes).  The
 * cell records staged by vd_build are the checkpoint: nothing is clipped
 * again, so the call is valid until the next vd_build on this context.
 *   g_vol   device float[n], or NULL (zero)
 *   g_cen   device float[n*3], or NULL
 *   g_vert  device float[n_vert*3] in the vertex order of vd_write, or NULL
 *   g_xyz   device float[n*3] out (original site order)
 *   g_w     device float[n] out, or NULL to skip (computed also for Voronoi
 *           builds, as the derivative at w = 0)
 * An empty cell has V = 0 and c = p_i, so it passes g_cen[i] to its site.
 * A box given to vd_build is held fixed.  Without one the box is the sites'
 * bounding box, whose faces move with the extreme sites: the sum over all
 * cells of dL/db of each face then goes to the lowest-index site on that
 * face (b = p_i,k - min_j p_j,k for a lower face, max_j p_j,k - p_i,k for an
 * upper one).
 * Stream-ordered, does not synchronise; the output is deterministic except
 * where a facet is not listed back by its neighbour (FP32-undecidable
 * configurations), whose share is added atomically.  VD_ERR_STATE without a
 * build. */
VD_API vd_status vd_backward(vd_context* ctx, const float* g_vol, const float* g_cen, const float* g_vert,
                             float* g_xyz, float* g_w, void* stream);

/* vd_backward for callers that cannot allocate device memory (code under HIP
 * graph capture, tight training or serving loops, harnesses that forbid
 * hipMalloc): same arguments, same kernels and the same result, but its
 * scratch is a fixed device array of the library (64 MiB per device, set up
 * by vd_create on that device and held until the process ends) instead of
 * context memory grown with hipMalloc.  It calls no allocating routine and
 * no memset (its scratch is cleared by a fill kernel).  The caller still
 * passes the inputs and outputs; the context's build state is read as in
 * vd_backward.  Needs 32 (n_facet + 2 n) bytes, each part rounded up to 256
 * (plus 48 per site, at most about 3 MB, when the box is the sites' own);
 * VD_ERR_INVALID_ARG with the size in the message if the last build
 * needs more (use vd_backward).  All calls on one device share that array,
 * which keeps the last call's contents: calls that overlap in time on one
 * device (several streams or host threads) race and must be serialised by
 * the caller. */
VD_API vd_status vd_backward_noalloc(vd_context* ctx, const float* g_vol, const float* g_cen, const float* g_vert,
                                     float* g_xyz, float* g_w, void* stream);

/* The dual of the last build (paper Sec. 3: the power diagram's dual is the
 * regular triangulation of the weighted sites; for equal weights the Delaunay
 * tetrahedralisation): one tetrahedron per diagram vertex that lies inside the
 * box, i.e. whose three facets are all site facets -- that vertex joins the
 * cells of four sites i < j < k < l, and the row is (i, j, k, l).  Tetrahedra
 * whose vertex (their power centre) falls outside the box are not listed.
 *   tets      device int32[capacity * 4] out, or NULL to only count
 *   capacity  rows available in tets
 *   count     HOST int64 out: the number of tetrahedra
 * Rows are grouped by their smallest site i (ascending), then in the vertex
 * order of that cell in vd_write.  Host-blocking (it synchronises `stream` to
 * count); VD_ERR_INVALID_ARG if capacity is below the count (nothing
 * written), VD_ERR_STATE without a build. */
VD_API vd_status vd_tetrahedra(vd_context* ctx, int32_t* tets, int64_t capacity, int64_t* count, void* stream);

/* The bounding-volume hierarchy of the last build, for inspection and tests
 * (Sec. 4.3: a binary BVH over the sites whose nodes also hold the largest
 * weight below them).  Every output is optional (NULL skips it); device
 * arrays, written on `stream` (not synchronised):
 *   morton      uint64[n]  Morton code of each site, caller's order (63 bits,
 *                          21 per axis inside the build's box)
 *   sorted_keys uint64[n]  the codes sorted ascending (the radix sort's output)
 *   order       uint32[n]  Morton position -> caller's index of the site
 *   nodes       (n-1) records of 64 bytes: for each internal node its two
 *               children, each { float lo[3]; float wmax; float hi[3];
 *               uint32 ref }; ref bit 31 set: a leaf of sites at Morton
 *               positions [ref & 0x1FFFFFF, + ((ref >> 25) & 63) + 1),
 *               otherwise the index of an internal node
 *   leaf_of     uint32[n]  per Morton position: (node << 1) | child, the
 *               record of the leaf that holds the site
 *   root        HOST uint32: the root reference (a leaf when n <= leaf size;
 *               nodes and leaf_of are then not written)
 * VD_ERR_STATE without a build. */
VD_API vd_status vd_inspect_bvh(vd_context* ctx, uint64_t* morton, uint64_t* sorted_keys, uint32_t* order,
                                void* nodes, uint32_t* leaf_of, uint32_t* root, void* stream);

/* Counters of the last build (see vd_sizes); host call, no device work. */
VD_API vd_status vd_get_sizes(const vd_context* ctx, vd_sizes* sizes);

/* Per-phase times of the last build/write/backward, ms[VD_PHASE_*]; needs
 * vd_options.profile = 1 on that build (phases not run read 0).  Waits for
 * the recorded events. */
VD_API vd_status vd_get_timings(vd_context* ctx, float* ms, int32_t count);

/* Work counters of the last build (up to VD_TIERS * VD_CTR_COUNT entries, see
 * VD_CTR_*); needs vd_options.counters = 1. */
VD_API vd_status vd_get_counters(const vd_context* ctx, uint64_t* out, int32_t count);

/* Achievable peaks of HIP device `device`, for roofline reports: the HBM
 * bandwidth of a plain float4 stream copy of 1 GiB (bytes read plus written
 * per second, in GB/s) and the rate of independent FP32 fused multiply-adds
 * (lane operations per second, one per FMA, in units of 10^12), each the best
 * of five timed runs (HIP events on `stream`) after one warm-up run.
 * Allocates and frees 2 GiB of device scratch; host-blocking.  Not part of
 * building a diagram. */
VD_API vd_status vd_measure_peaks(int device, void* stream, double* copy_gbs, double* fma_tops);

/* Message for the last error on this thread ("" if none). */
VD_API const char* vd_last_error(void);

/* Library version string. */
VD_API const char* vd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VD_H */
