// Host side of the C ABI declared in include/vd.h.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "vd.h"
#include "vd_internal.h"

namespace {

thread_local std::string g_err;


vd_status fail(vd_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define VD_HIP(x)                                                                                   \
    do {                                                                                            \
        hipError_t e_ = (x);                                                                        \
        if (e_ != hipSuccess) return fail(VD_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
};

}  // namespace

struct vd_context {
    int device = 0;
    int num_cu = 0;
    // grow-only device scratch
    // pint: parent links of the internal nodes; pleaf: leaf record of each site
    DevBuf pts, spts, keys[2], vals[2], inv, mark, child, pint, pleaf, range, counters, nodes, hist, stmp, bbox,
        bpart, misc, loc, cnt_v, cnt_f, cnt_n, vol, cen, flags, offv, offf, offn, scan_tmp, stats, ctr;
    DevBuf lists[vd::kTiers];  // lists[t]: cells handed on to tier t (t >= 1)
    DevBuf st_vert[vd::kTiers], st_tri64[vd::kTiers], st_code[vd::kTiers], st_fsize[vd::kTiers], st_fv[vd::kTiers];
    DevBuf arena;  // per-worker cell arrays of the last (16384-vertex) pass
    DevBuf hand[vd::kTiers - 1];  // hand[t]: states of the cells the pass of tier t hands to the next
    uint32_t seen[vd::kTiers] = {};  // largest cell count of each pass met so far (sizes its buffers)
    DevBuf tet_cnt, tet_off;  // dual tetrahedra per cell and their offsets
    DevBuf bwd_facet, bwd_self, bwd_orphan, bwd_box;  // backward scratch
    DevBuf inspect;  // scratch of vd_inspect_bvh
    void* fixed_scratch = nullptr;  // this device's fixed scratch of vd_backward_noalloc
    // last build
    bool valid = false;
    int64_t n = 0;
    vd_sizes sizes{};
    const uint32_t* order = nullptr;
    const uint64_t* skeys = nullptr;  // sorted Morton codes of the last build
    uint32_t root = 0;
    int leaf_size = 0;
    int tier_slots[vd::kTiers] = {};
    // profiling: events e[0..6] bracket the build phases, e[7..8] the write,
    // e[9..10] the backward
    hipEvent_t ev[11] = {};
    bool ev_ready = false;
    bool profiled = false, write_profiled = false, bwd_profiled = false;
    bool counted = false;
    bool box_given = false;  // false: the box of the last build is the sites' bounding box
};

namespace {

using vd::kTierCap;
constexpr int kMiscWords = 16 + vd::kWorkRanges * vd::kTiers;
static_assert(vd::kTiers <= 4 && vd::kWorkRanges == 8, "misc layout");

vd_status ensure(DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (b.cap >= bytes) return VD_OK;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
        if (e != hipSuccess) return fail(VD_ERR_HIP, std::string("hipFree: ") + hipGetErrorString(e));
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return fail(VD_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    b.cap = bytes;
    return VD_OK;
}

void release(DevBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

template <typename T>
T* as(DevBuf& b) {
    return static_cast<T*>(b.p);
}

#define VD_TRY(x)                     \
    do {                              \
        vd_status s_ = (x);           \
        if (s_ != VD_OK) return s_;   \
    } while (0)

vd_status ensure_stage(vd_context* c, int tier, int64_t slots) {
    const size_t cap = (size_t)kTierCap[tier];
    const size_t sl = (size_t)(slots > 0 ? slots : 1);
    VD_TRY(ensure(c->st_vert[tier], sl * cap * sizeof(float4)));
    if (cap > 1024) VD_TRY(ensure(c->st_tri64[tier], sl * cap * sizeof(uint64_t)));
    VD_TRY(ensure(c->st_code[tier], sl * cap * sizeof(int32_t)));
    VD_TRY(ensure(c->st_fsize[tier], sl * cap * sizeof(uint16_t)));
    VD_TRY(ensure(c->st_fv[tier], sl * 3 * cap * sizeof(uint16_t)));
    return VD_OK;
}

vd_status ensure_events(vd_context* c) {
    if (c->ev_ready) return VD_OK;
    for (hipEvent_t& e : c->ev) VD_HIP(hipEventCreate(&e));
    c->ev_ready = true;
    return VD_OK;
}

vd::Stage stage_of(vd_context* c, int tier) {
    vd::Stage s;
    s.cap = kTierCap[tier];
    s.vert = as<float4>(c->st_vert[tier]);
    s.tri64 = kTierCap[tier] > 1024 ? as<uint64_t>(c->st_tri64[tier]) : nullptr;
    s.code = as<int32_t>(c->st_code[tier]);
    s.fsize = as<uint16_t>(c->st_fsize[tier]);
    s.fv = as<uint16_t>(c->st_fv[tier]);
    return s;
}

}  // namespace

extern "C" {

VD_API const char* vd_last_error(void) { return g_err.c_str(); }

VD_API const char* vd_version(void) { return "libvd 0.1 (gfx950)"; }

VD_API vd_status vd_create(int device, vd_context** out) {
    g_err.clear();
    if (!out) return fail(VD_ERR_INVALID_ARG, "vd_create: null output pointer");
    *out = nullptr;
    int count = 0;
    VD_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(VD_ERR_INVALID_ARG, "vd_create: no such device");
    VD_HIP(hipSetDevice(device));
    vd_context* c = new vd_context;
    c->device = device;
    hipError_t e = hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess || c->num_cu < 1) c->num_cu = 256;
    // address of this device's fixed backward scratch (looked up once per device)
    e = vd::bwd_scratch_init(device, &c->fixed_scratch);
    if (e != hipSuccess) {
        delete c;
        return fail(VD_ERR_HIP, std::string("vd_create: scratch symbol lookup: ") + hipGetErrorString(e));
    }
    *out = c;
    return VD_OK;
}

VD_API void vd_destroy(vd_context* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    DevBuf* all[] = {&c->pts, &c->spts, &c->keys[0], &c->keys[1], &c->vals[0], &c->vals[1], &c->inv, &c->mark,
                     &c->child, &c->pint, &c->pleaf, &c->range, &c->counters, &c->nodes, &c->hist, &c->stmp,
                     &c->bbox, &c->bpart, &c->misc, &c->loc, &c->cnt_v, &c->cnt_f, &c->cnt_n, &c->vol, &c->cen,
                     &c->flags, &c->offv, &c->offf, &c->offn, &c->scan_tmp, &c->stats,
                     &c->ctr, &c->arena, &c->tet_cnt, &c->tet_off, &c->bwd_facet, &c->bwd_self,
                     &c->bwd_orphan, &c->bwd_box, &c->inspect};
    for (DevBuf* b : all) release(*b);
    if (c->ev_ready)
        for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    for (int t = 0; t + 1 < vd::kTiers; ++t) release(c->hand[t]);
    for (int t = 0; t < vd::kTiers; ++t) {
        release(c->lists[t]);
        release(c->st_vert[t]);
        release(c->st_tri64[t]);
        release(c->st_code[t]);
        release(c->st_fsize[t]);
        release(c->st_fv[t]);
    }
    delete c;
}

VD_API vd_status vd_get_sizes(const vd_context* c, vd_sizes* sizes) {
    if (!c || !sizes) return fail(VD_ERR_INVALID_ARG, "vd_get_sizes: null argument");
    if (!c->valid) return fail(VD_ERR_STATE, "vd_get_sizes: no successful build");
    *sizes = c->sizes;
    return VD_OK;
}

VD_API vd_status vd_build(vd_context* c, const float* xyz, const float* w, int64_t n, const float* bbox,
                          const vd_options* opt, void* stream, vd_sizes* sizes) {
    g_err.clear();
    if (!c || !xyz || !sizes) return fail(VD_ERR_INVALID_ARG, "vd_build: null argument");
    c->valid = false;
    if (n < 1 || n > vd::kMaxSites)
        return fail(VD_ERR_INVALID_ARG, "vd_build: n must be in [1, " + std::to_string(vd::kMaxSites) + "]");
    vd_options o{};
    if (opt) o = *opt;
    if (o.perturb < 0 || o.perturb > 1) return fail(VD_ERR_INVALID_ARG, "vd_build: perturb must be 0 or 1");
    if (o.perturb) o.precision = 2;  // ties reach the exact test through the FP64 re-evaluation
    if (o.precision == 0) o.precision = 1;
    if (o.leaf_size == 0) o.leaf_size = vd::kDefaultLeaf;
    if (o.culling == 0) o.culling = 3;
    if (o.traversal == 0) o.traversal = 1;
    if (o.precision < 1 || o.precision > 2) return fail(VD_ERR_INVALID_ARG, "vd_build: precision must be 1 or 2");
    if (o.leaf_size < 1 || o.leaf_size > vd::kMaxLeaf)
        return fail(VD_ERR_INVALID_ARG, "vd_build: leaf_size must be in [1, 64]");
    if (o.culling < 1 || o.culling > 3) return fail(VD_ERR_INVALID_ARG, "vd_build: culling must be 1, 2 or 3");
    if (o.traversal < 1 || o.traversal > 2) return fail(VD_ERR_INVALID_ARG, "vd_build: traversal must be 1 or 2");
    if (o.warm_start < 0 || o.warm_start > vd::kMaxWarm)
        return fail(VD_ERR_INVALID_ARG, "vd_build: warm_start must be in [0, " + std::to_string(vd::kMaxWarm) + "]");
    if (bbox) {
        for (int k = 0; k < 6; ++k)
            if (!std::isfinite(bbox[k])) return fail(VD_ERR_INVALID_ARG, "vd_build: non-finite bbox");
        for (int k = 0; k < 3; ++k)
            if (!(bbox[3 + k] > bbox[k])) return fail(VD_ERR_INVALID_ARG, "vd_build: bbox extent must be positive");
    }
    VD_HIP(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t N = (size_t)n;
    const bool prof = o.profile != 0;
    c->profiled = false;
    c->write_profiled = false;
    c->bwd_profiled = false;
    c->counted = false;
    if (prof) VD_TRY(ensure_events(c));

    VD_TRY(ensure(c->pts, N * sizeof(float4)));
    VD_TRY(ensure(c->spts, N * sizeof(float4)));
    for (int k = 0; k < 2; ++k) {
        VD_TRY(ensure(c->keys[k], N * sizeof(uint64_t)));
        VD_TRY(ensure(c->vals[k], N * sizeof(uint32_t)));
    }
    VD_TRY(ensure(c->inv, N * sizeof(uint32_t)));
    VD_TRY(ensure(c->mark, N));
    VD_TRY(ensure(c->child, N * sizeof(int2)));
    VD_TRY(ensure(c->pint, N * sizeof(int)));
    VD_TRY(ensure(c->pleaf, N * sizeof(int)));
    VD_TRY(ensure(c->range, N * sizeof(int2)));
    VD_TRY(ensure(c->counters, vd::box_table_size(n) * sizeof(vd::NodeChild)));
    VD_TRY(ensure(c->nodes, N * sizeof(vd::Node)));
    VD_TRY(ensure(c->hist, vd::radix_hist_size(n) * sizeof(uint32_t)));
    VD_TRY(ensure(c->stmp, vd::scan_tmp_size((int64_t)vd::radix_hist_size(n)) * sizeof(uint64_t)));
    VD_TRY(ensure(c->bbox, 8 * sizeof(float)));
    VD_TRY(ensure(c->bpart, 1024 * 6 * sizeof(float)));
    VD_TRY(ensure(c->misc, kMiscWords * sizeof(uint32_t)));
    VD_TRY(ensure(c->loc, N * sizeof(uint32_t)));
    VD_TRY(ensure(c->cnt_v, N * sizeof(uint32_t)));
    VD_TRY(ensure(c->cnt_f, N * sizeof(uint32_t)));
    VD_TRY(ensure(c->cnt_n, N * sizeof(uint32_t)));
    VD_TRY(ensure(c->vol, N * sizeof(float)));
    VD_TRY(ensure(c->cen, 3 * N * sizeof(float)));
    VD_TRY(ensure(c->flags, N));
    VD_TRY(ensure(c->offv, (N + 1) * sizeof(int64_t)));
    VD_TRY(ensure(c->offf, (N + 1) * sizeof(int64_t)));
    VD_TRY(ensure(c->offn, (N + 1) * sizeof(int64_t)));
    VD_TRY(ensure(c->scan_tmp, vd::scan_tmp_size(n) * sizeof(int64_t)));
    for (int t = 1; t < vd::kTiers; ++t) VD_TRY(ensure(c->lists[t], N * sizeof(uint32_t)));
    VD_TRY(ensure(c->stats, vd::kStatCount * sizeof(unsigned long long)));
    VD_TRY(ensure(c->ctr, vd::kTiers * vd::kCtrCount * sizeof(unsigned long long)));
    VD_TRY(ensure_stage(c, 0, n));

    // misc: [0] error bits, [1] cells left undone for want of slots, [4 + t]
    // list count of tier t >= 1, [16 + 8 t ..] the kWorkRanges work counters
    // of tier t
    uint32_t* misc = as<uint32_t>(c->misc);
    if (prof) VD_HIP(hipEventRecord(c->ev[0], s));
    VD_HIP(hipMemsetAsync(misc, 0, kMiscWords * sizeof(uint32_t), s));
    if (o.counters) VD_HIP(hipMemsetAsync(c->ctr.p, 0, vd::kTiers * vd::kCtrCount * sizeof(unsigned long long), s));
    VD_HIP(hipMemsetAsync(c->stats.p, 0, vd::kStatCount * sizeof(unsigned long long), s));
    float4* pts = as<float4>(c->pts);
    float* dbbox = as<float>(c->bbox);
    VD_HIP(vd::launch_pack(xyz, w, n, pts, misc, s));
    if (bbox) {
        VD_HIP(hipMemcpyAsync(dbbox, bbox, 6 * sizeof(float), hipMemcpyHostToDevice, s));
        VD_HIP(vd::launch_check_bbox(dbbox, misc, s));
    } else {
        VD_HIP(vd::launch_bbox(pts, n, as<float>(c->bpart), 1024, dbbox, misc, s));
    }
    VD_HIP(vd::launch_morton(pts, n, dbbox, as<uint64_t>(c->keys[0]), as<uint32_t>(c->vals[0]), s));
    bool in_tmp = false;
    VD_HIP(vd::radix_sort(as<uint64_t>(c->keys[0]), as<uint32_t>(c->vals[0]), as<uint64_t>(c->keys[1]),
                          as<uint32_t>(c->vals[1]), n, 63, as<uint32_t>(c->hist), as<uint32_t>(c->stmp), s,
                          &in_tmp));
    const uint64_t* skeys = as<uint64_t>(c->keys[in_tmp ? 1 : 0]);
    const uint32_t* order = as<uint32_t>(c->vals[in_tmp ? 1 : 0]);
    float4* spts = as<float4>(c->spts);
    VD_HIP(vd::launch_gather(pts, order, n, spts, as<uint32_t>(c->inv), s));
    VD_HIP(vd::launch_losers(spts, skeys, order, n, as<uint8_t>(c->mark), s));
    uint32_t root;
    if (n > o.leaf_size) {
        VD_HIP(vd::launch_karras(skeys, n, as<int2>(c->child), as<uint32_t>(c->pint), as<int2>(c->range), s));
        VD_HIP(vd::launch_bounds(spts, n, as<int2>(c->child), as<int2>(c->range), as<vd::NodeChild>(c->counters),
                                 as<vd::Node>(c->nodes), as<uint32_t>(c->pleaf), o.leaf_size, s));
        root = 0;
    } else {
        root = vd::leaf_ref(0u, (uint32_t)n);
    }

    vd::ClipArgs a{};
    a.pts = spts;
    a.order = order;
    a.nodes = as<vd::Node>(c->nodes);
    a.root = root;
    a.up = as<uint32_t>(c->pint);
    a.leaf_of = vd::ref_is_leaf(root) ? nullptr : as<uint32_t>(c->pleaf);
    a.bbox = dbbox;
    a.n = n;
    a.leaf_size = o.leaf_size;
    a.culling = o.culling;
    a.traversal = o.traversal;
    a.warm_start = o.warm_start;
    a.precision = o.precision;
    a.perturb = o.perturb;
    a.weighted = w != nullptr ? 1 : 0;
    a.loc = as<uint32_t>(c->loc);
    a.cnt_v = as<uint32_t>(c->cnt_v);
    a.cnt_f = as<uint32_t>(c->cnt_f);
    a.cnt_n = as<uint32_t>(c->cnt_n);
    a.vol = as<float>(c->vol);
    a.cen = as<float>(c->cen);
    a.flags = as<uint8_t>(c->flags);
    a.stats = as<unsigned long long>(c->stats);
    a.ctr = o.counters ? as<unsigned long long>(c->ctr) : nullptr;
    a.err = misc;

    // The clipping passes run back to back with no host synchronisation: the
    // larger passes are launched with persistent grids that read their cell
    // counts from device memory, on buffers sized beforehand for at least a
    // floor of cells (n/64 and n/1024, at least 1024 each, and 16 for the
    // 128-, 1024- and 16384-vertex passes) and at least as many as earlier
    // builds on this context needed.  A pass with more cells than slots leaves the extra ones
    // undone and counts them; the one synchronisation at the end then sees the
    // counts, the buffers grow, and the passes run again (a first build of a
    // larger workload; the LBVH is kept).
    uint32_t hmisc[16];
    int64_t tot[3];
    unsigned long long st[vd::kStatCount];
    for (int attempt = 0;; ++attempt) {
        if (attempt > 0) {
            VD_HIP(hipMemsetAsync(misc + 1, 0, (kMiscWords - 1) * sizeof(uint32_t), s));
            VD_HIP(hipMemsetAsync(c->stats.p, 0, vd::kStatCount * sizeof(unsigned long long), s));
            if (o.counters)
                VD_HIP(hipMemsetAsync(c->ctr.p, 0, vd::kTiers * vd::kCtrCount * sizeof(unsigned long long), s));
        }
        uint32_t slots[vd::kTiers];
        slots[0] = (uint32_t)n;
        for (int t = 1; t < vd::kTiers; ++t) {
            static constexpr uint32_t kDiv[vd::kTiers] = {1u, 64u, 1024u, 0u};
            static constexpr uint32_t kFloor[vd::kTiers] = {0u, 1024u, 1024u, 16u};
            uint64_t cap = kDiv[t] ? (uint64_t)n / kDiv[t] : 0;
            if (cap < kFloor[t]) cap = kFloor[t];
            if (cap < c->seen[t]) cap = c->seen[t];
            if (cap > (uint64_t)n) cap = (uint64_t)n;
            slots[t] = (uint32_t)cap;
            VD_TRY(ensure_stage(c, t, cap));
        }
        // hand-over records: every cell the 64-vertex pass may escalate, at
        // most 8192 from the 128-vertex pass and 256 from the 1024-vertex pass
        static constexpr uint32_t kHandMax[vd::kTiers - 1] = {0xFFFFFFFFu, 8192u, 256u};
        uint32_t hand_cap[vd::kTiers - 1];
        for (int t = 0; t + 1 < vd::kTiers; ++t) {
            hand_cap[t] = slots[t + 1] < kHandMax[t] ? slots[t + 1] : kHandMax[t];
            VD_TRY(ensure(c->hand[t], (size_t)hand_cap[t] * vd::handoff_bytes(t)));
        }
        // arena workers of the last pass: one per CU at most, as many as its
        // cells of earlier builds at least 4 (they loop over the cells)
        int arena_workers = (int)(c->seen[3] > 4u ? c->seen[3] : 4u);
        if (arena_workers > c->num_cu) arena_workers = c->num_cu;
        VD_TRY(ensure(c->arena, (size_t)arena_workers * vd::arena_bytes_per_worker()));

        for (int tier = 0; tier < vd::kTiers; ++tier) {
            const bool last = tier + 1 == vd::kTiers;
            a.tier = tier;
            a.work_counter = misc + 16 + vd::kWorkRanges * tier;
            a.list = tier ? as<uint32_t>(c->lists[tier]) : nullptr;
            a.list_count = tier ? misc + 4 + tier : nullptr;
            a.slots = slots[tier];
            a.deferred = misc + 1;
            a.next_list = last ? nullptr : as<uint32_t>(c->lists[tier + 1]);
            a.next_count = last ? nullptr : misc + 5 + tier;
            a.stage = stage_of(c, tier);
            a.ctr = o.counters ? as<unsigned long long>(c->ctr) + tier * vd::kCtrCount : nullptr;
            a.hand_in = tier ? c->hand[tier - 1].p : nullptr;
            a.hand_in_cap = tier ? hand_cap[tier - 1] : 0u;
            a.hand_out = last ? nullptr : c->hand[tier].p;
            a.hand_out_cap = last ? 0u : hand_cap[tier];
            const int workers = last ? arena_workers : vd::clip_grid_workers(tier, c->num_cu);
            if (prof && tier == 0) VD_HIP(hipEventRecord(c->ev[1], s));
            VD_HIP(vd::launch_clip(a, workers, last ? c->arena.p : nullptr, s));
            if (prof && tier == 0) VD_HIP(hipEventRecord(c->ev[2], s));
            if (prof && tier == 1) VD_HIP(hipEventRecord(c->ev[6], s));
        }
        if (prof) VD_HIP(hipEventRecord(c->ev[3], s));
        VD_HIP(vd::scan_counts(as<uint32_t>(c->cnt_v), n, as<int64_t>(c->offv), as<int64_t>(c->scan_tmp), s));
        VD_HIP(vd::scan_counts(as<uint32_t>(c->cnt_f), n, as<int64_t>(c->offf), as<int64_t>(c->scan_tmp), s));
        VD_HIP(vd::scan_counts(as<uint32_t>(c->cnt_n), n, as<int64_t>(c->offn), as<int64_t>(c->scan_tmp), s));
        VD_HIP(hipMemcpyAsync(&tot[0], as<int64_t>(c->offv) + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        VD_HIP(hipMemcpyAsync(&tot[1], as<int64_t>(c->offf) + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        VD_HIP(hipMemcpyAsync(&tot[2], as<int64_t>(c->offn) + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        if (prof) VD_HIP(hipEventRecord(c->ev[4], s));
        VD_HIP(hipMemcpyAsync(st, c->stats.p, sizeof(st), hipMemcpyDeviceToHost, s));
        VD_HIP(hipMemcpyAsync(hmisc, misc, sizeof(hmisc), hipMemcpyDeviceToHost, s));
        if (prof) VD_HIP(hipEventRecord(c->ev[5], s));
        VD_HIP(hipStreamSynchronize(s));  // the one synchronisation of a build
        if (hmisc[0] & 1u) return fail(VD_ERR_INVALID_ARG, "vd_build: non-finite site coordinate or weight");
        if (hmisc[0] & 2u) return fail(VD_ERR_INVALID_ARG, "vd_build: degenerate bounding box");
        c->tier_slots[0] = (int)n;
        bool short_before = false;
        for (int t = 1; t < vd::kTiers; ++t) {
            const uint32_t cnt = hmisc[4 + t];
            c->tier_slots[t] = (int)cnt;
            // behind a pass that left cells undone the counts are too low
            const uint32_t want = short_before ? 2u * cnt + 16u : cnt;
            if (want > c->seen[t]) c->seen[t] = want;
            if (cnt > slots[t]) short_before = true;
        }
        if (hmisc[1] == 0) break;
        if (attempt >= 2 * vd::kTiers)
            return fail(VD_ERR_HIP, "vd_build: the larger passes kept outgrowing their buffers");
    }
    c->profiled = prof;
    c->counted = o.counters != 0;

    vd_sizes z{};
    z.n = n;
    z.n_vert = tot[0];
    z.n_facet = tot[1];
    z.n_nbr = tot[2];
    z.n_fv = 3 * tot[0];
    z.n_empty = (int64_t)st[vd::kStatEmpty];
    z.n_large = (int64_t)st[vd::kStatLarge];
    z.n_uncertain = (int64_t)st[vd::kStatUncertain];
    z.n_failed = (int64_t)st[vd::kStatFailed];
    z.n_fp64 = (int64_t)st[vd::kStatFP64];
    z.n_huge = c->tier_slots[3];
    z.n_resumed = (int64_t)st[vd::kStatResumed];
    z.n_perturbed = (int64_t)st[vd::kStatPerturbed];
    c->sizes = z;
    c->n = n;
    c->order = order;
    c->skeys = skeys;
    c->root = root;
    c->leaf_size = o.leaf_size;
    c->box_given = bbox != nullptr;
    c->valid = true;
    *sizes = z;
    if (z.n_failed > 0)
        return fail(VD_ERR_CAPACITY, "vd_build: " + std::to_string(z.n_failed) +
                                         " cells exceeded the largest capacity (" +
                                         std::to_string(kTierCap[vd::kTiers - 1]) + " vertices); they are flagged");
    return VD_OK;
}

VD_API vd_status vd_write(vd_context* c, const vd_outputs* out, void* stream) {
    g_err.clear();
    if (!c || !out) return fail(VD_ERR_INVALID_ARG, "vd_write: null argument");
    if (!c->valid) return fail(VD_ERR_STATE, "vd_write: no successful build");
    VD_HIP(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = c->n;
    const bool prof = c->profiled;
    if (prof) VD_HIP(hipEventRecord(c->ev[7], s));
    vd::WriteArgs a{};
    a.n = n;
    a.inv = as<uint32_t>(c->inv);
    a.loc = as<uint32_t>(c->loc);
    for (int t = 0; t < vd::kTiers; ++t) a.stage[t] = stage_of(c, t);
    a.cnt_v = as<uint32_t>(c->cnt_v);
    a.cnt_f = as<uint32_t>(c->cnt_f);
    a.cnt_n = as<uint32_t>(c->cnt_n);
    a.off_v = as<int64_t>(c->offv);
    a.off_f = as<int64_t>(c->offf);
    a.off_n = as<int64_t>(c->offn);
    a.nbr = out->nbr;
    a.facet_nbr = out->facet_nbr;
    a.fv_off = out->fv_off;
    a.fv = out->fv;
    a.vert = out->vert;
    a.vert_planes = out->vert_planes;
    if (a.nbr || a.facet_nbr || a.fv_off || a.fv || a.vert || a.vert_planes) VD_HIP(vd::launch_write(a, s));
    const size_t off_bytes = (size_t)(n + 1) * sizeof(int64_t);
    if (out->nbr_off) VD_HIP(hipMemcpyAsync(out->nbr_off, c->offn.p, off_bytes, hipMemcpyDeviceToDevice, s));
    if (out->facet_off) VD_HIP(hipMemcpyAsync(out->facet_off, c->offf.p, off_bytes, hipMemcpyDeviceToDevice, s));
    if (out->vert_off) VD_HIP(hipMemcpyAsync(out->vert_off, c->offv.p, off_bytes, hipMemcpyDeviceToDevice, s));
    if (out->fv_off) VD_HIP(vd::launch_set_i64(out->fv_off + c->sizes.n_facet, c->sizes.n_fv, s));
    if (out->vol) VD_HIP(hipMemcpyAsync(out->vol, c->vol.p, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (out->centroid)
        VD_HIP(hipMemcpyAsync(out->centroid, c->cen.p, 3 * (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (out->flags) VD_HIP(hipMemcpyAsync(out->flags, c->flags.p, (size_t)n, hipMemcpyDeviceToDevice, s));
    if (prof) {
        VD_HIP(hipEventRecord(c->ev[8], s));
        c->write_profiled = true;
    }
    return VD_OK;
}

VD_API vd_status vd_tetrahedra(vd_context* c, int32_t* tets, int64_t capacity, int64_t* count, void* stream) {
    g_err.clear();
    if (!c || !count) return fail(VD_ERR_INVALID_ARG, "vd_tetrahedra: null argument");
    if (!c->valid) return fail(VD_ERR_STATE, "vd_tetrahedra: no successful build");
    VD_HIP(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = c->n;
    VD_TRY(ensure(c->tet_cnt, (size_t)n * sizeof(uint32_t)));
    VD_TRY(ensure(c->tet_off, (size_t)(n + 1) * sizeof(int64_t)));
    vd::TetArgs a{};
    a.n = n;
    a.inv = as<uint32_t>(c->inv);
    a.loc = as<uint32_t>(c->loc);
    for (int t = 0; t < vd::kTiers; ++t) a.stage[t] = stage_of(c, t);
    a.cnt_v = as<uint32_t>(c->cnt_v);
    a.cnt_t = as<uint32_t>(c->tet_cnt);
    a.off_t = as<int64_t>(c->tet_off);
    VD_HIP(vd::launch_tet_count(a, s));
    VD_HIP(vd::scan_counts(a.cnt_t, n, as<int64_t>(c->tet_off), as<int64_t>(c->scan_tmp), s));
    int64_t total = 0;
    VD_HIP(hipMemcpyAsync(&total, as<int64_t>(c->tet_off) + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    VD_HIP(hipStreamSynchronize(s));
    *count = total;
    if (!tets) return VD_OK;
    if (capacity < total) return fail(VD_ERR_INVALID_ARG, "vd_tetrahedra: capacity below the count");
    a.tets = tets;
    if (total > 0) VD_HIP(vd::launch_tet_write(a, s));
    return VD_OK;
}

VD_API vd_status vd_inspect_bvh(vd_context* c, uint64_t* morton, uint64_t* sorted_keys, uint32_t* order,
                                void* nodes, uint32_t* leaf_of, uint32_t* root, void* stream) {
    g_err.clear();
    if (!c || !root) return fail(VD_ERR_INVALID_ARG, "vd_inspect_bvh: null argument");
    if (!c->valid) return fail(VD_ERR_STATE, "vd_inspect_bvh: no successful build");
    VD_HIP(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = c->n;
    *root = c->root;
    if (morton) {
        // codes of the sites in the caller's order, recomputed as the build made them
        VD_TRY(ensure(c->inspect, (size_t)n * sizeof(uint32_t)));
        VD_HIP(vd::launch_morton(as<float4>(c->pts), n, as<float>(c->bbox), morton, as<uint32_t>(c->inspect), s));
    }
    if (sorted_keys)
        VD_HIP(hipMemcpyAsync(sorted_keys, c->skeys, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    if (order) VD_HIP(hipMemcpyAsync(order, c->order, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    const bool tree = !vd::ref_is_leaf(c->root);
    if (nodes && tree)
        VD_HIP(hipMemcpyAsync(nodes, c->nodes.p, (size_t)(n - 1) * sizeof(vd::Node), hipMemcpyDeviceToDevice, s));
    if (leaf_of && tree)
        VD_HIP(hipMemcpyAsync(leaf_of, c->pleaf.p, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    return VD_OK;
}

VD_API vd_status vd_get_timings(vd_context* c, float* ms, int32_t count) {
    if (!c || !ms || count < 0) return fail(VD_ERR_INVALID_ARG, "vd_get_timings: bad argument");
    if (!c->valid || !c->profiled) return fail(VD_ERR_STATE, "vd_get_timings: last build was not profiled");
    VD_HIP(hipSetDevice(c->device));
    float t[VD_PHASE_COUNT] = {};
    VD_HIP(hipEventSynchronize(c->ev[5]));
    VD_HIP(hipEventElapsedTime(&t[VD_PHASE_LBVH], c->ev[0], c->ev[1]));
    VD_HIP(hipEventElapsedTime(&t[VD_PHASE_CLIP], c->ev[1], c->ev[2]));
    VD_HIP(hipEventElapsedTime(&t[VD_PHASE_CLIP_LARGE], c->ev[2], c->ev[3]));
    VD_HIP(hipEventElapsedTime(&t[VD_PHASE_SCAN], c->ev[3], c->ev[4]));
    VD_HIP(hipEventElapsedTime(&t[VD_PHASE_BUILD], c->ev[0], c->ev[5]));
    if (c->tier_slots[1] > 0) VD_HIP(hipEventElapsedTime(&t[VD_PHASE_CLIP_TIER1], c->ev[2], c->ev[6]));
    if (c->write_profiled) {
        VD_HIP(hipEventSynchronize(c->ev[8]));
        VD_HIP(hipEventElapsedTime(&t[VD_PHASE_WRITE], c->ev[7], c->ev[8]));
    }
    if (c->bwd_profiled) {
        VD_HIP(hipEventSynchronize(c->ev[10]));
        VD_HIP(hipEventElapsedTime(&t[VD_PHASE_BACKWARD], c->ev[9], c->ev[10]));
    }
    for (int k = 0; k < count && k < VD_PHASE_COUNT; ++k) ms[k] = t[k];
    return VD_OK;
}

}  // extern "C"

namespace {

// Scratch of one backward: FP64 facet shares, per-site shares, asymmetric
// remainders and (box of the sites) the box-face partials, sums and sites.
struct BwdScratch {
    double4* facet = nullptr;
    double4* self = nullptr;
    double* orphan = nullptr;
    double* box = nullptr;  // nwaves * 6 partials, 6 sums, then 6 uint32 face sites
};

size_t bwd_box_bytes(int64_t nwaves) { return (size_t)(nwaves * 6 + 6) * sizeof(double) + 6 * sizeof(uint32_t); }

// Argument checks shared by both backward entry points.
vd_status bwd_check(vd_context* c, const float* g_xyz, const char* who) {
    g_err.clear();
    if (!c || !g_xyz) return fail(VD_ERR_INVALID_ARG, std::string(who) + ": null argument");
    if (!c->valid) return fail(VD_ERR_STATE, std::string(who) + ": no successful build");
    return VD_OK;
}

// The backward kernels over the last build, with the given scratch.  The
// remainders start at zero and the face sites at 0xFFFFFFFF: cleared with
// memsets (fill = false) or with a fill kernel (fill = true).
vd_status bwd_run(vd_context* c, const float* g_vol, const float* g_cen, const float* g_vert, float* g_xyz,
                  float* g_w, const BwdScratch& sc, bool fill, hipStream_t s) {
    const int64_t n = c->n;
    const int64_t nwaves = vd::bwd_waves(n);
    const bool moving_box = !c->box_given;
    const bool prof = c->profiled;
    if (prof) VD_HIP(hipEventRecord(c->ev[9], s));
    double* box_part = moving_box ? sc.box : nullptr;
    uint32_t* box_arg = moving_box ? reinterpret_cast<uint32_t*>(box_part + nwaves * 6 + 6) : nullptr;
    if (fill) {
        VD_HIP(vd::launch_fill_u64(reinterpret_cast<uint64_t*>(sc.orphan), n * 4, 0ull, s));
        // the six 32-bit face sites are three 64-bit words (8-byte aligned:
        // they follow whole doubles)
        if (moving_box) VD_HIP(vd::launch_fill_u64(reinterpret_cast<uint64_t*>(box_arg), 3, ~0ull, s));
    } else {
        VD_HIP(hipMemsetAsync(sc.orphan, 0, (size_t)n * 4 * sizeof(double), s));
        if (moving_box) VD_HIP(hipMemsetAsync(box_arg, 0xFF, 6 * sizeof(uint32_t), s));
    }
    vd::BwdArgs a{};
    a.n = n;
    a.pts = as<float4>(c->spts);
    a.inv = as<uint32_t>(c->inv);
    a.loc = as<uint32_t>(c->loc);
    for (int t = 0; t < vd::kTiers; ++t) a.stage[t] = stage_of(c, t);
    a.cnt_v = as<uint32_t>(c->cnt_v);
    a.cnt_f = as<uint32_t>(c->cnt_f);
    a.cnt_n = as<uint32_t>(c->cnt_n);
    a.off_v = as<int64_t>(c->offv);
    a.off_f = as<int64_t>(c->offf);
    a.bbox = as<float>(c->bbox);
    a.g_vol = g_vol;
    a.g_cen = g_cen;
    a.g_vert = g_vert;
    a.gf = sc.facet;
    a.gself = sc.self;
    a.orphan = sc.orphan;
    a.g_xyz = g_xyz;
    a.g_w = g_w;
    a.moving_box = moving_box ? 1 : 0;
    a.pts_orig = as<float4>(c->pts);
    a.box_part = box_part;
    a.box_sum = moving_box ? box_part + nwaves * 6 : nullptr;
    a.box_arg = box_arg;
    VD_HIP(vd::launch_backward(a, s));
    if (prof) {
        VD_HIP(hipEventRecord(c->ev[10], s));
        c->bwd_profiled = true;
    }
    return VD_OK;
}

}  // namespace

extern "C" {

VD_API vd_status vd_backward(vd_context* c, const float* g_vol, const float* g_cen, const float* g_vert,
                             float* g_xyz, float* g_w, void* stream) {
    VD_TRY(bwd_check(c, g_xyz, "vd_backward"));
    VD_HIP(hipSetDevice(c->device));
    const int64_t n = c->n;
    const size_t nf = (size_t)(c->sizes.n_facet > 0 ? c->sizes.n_facet : 1);
    VD_TRY(ensure(c->bwd_facet, nf * sizeof(double4)));
    VD_TRY(ensure(c->bwd_self, (size_t)n * sizeof(double4)));
    VD_TRY(ensure(c->bwd_orphan, (size_t)n * 4 * sizeof(double)));
    if (!c->box_given) VD_TRY(ensure(c->bwd_box, bwd_box_bytes(vd::bwd_waves(n))));
    BwdScratch sc;
    sc.facet = as<double4>(c->bwd_facet);
    sc.self = as<double4>(c->bwd_self);
    sc.orphan = as<double>(c->bwd_orphan);
    sc.box = as<double>(c->bwd_box);
    return bwd_run(c, g_vol, g_cen, g_vert, g_xyz, g_w, sc, false, static_cast<hipStream_t>(stream));
}

VD_API vd_status vd_backward_noalloc(vd_context* c, const float* g_vol, const float* g_cen, const float* g_vert,
                                     float* g_xyz, float* g_w, void* stream) {
    VD_TRY(bwd_check(c, g_xyz, "vd_backward_noalloc"));
    if (!c->fixed_scratch) return fail(VD_ERR_STATE, "vd_backward_noalloc: no fixed scratch on this device");
    VD_HIP(hipSetDevice(c->device));
    const int64_t n = c->n;
    const size_t nf = (size_t)(c->sizes.n_facet > 0 ? c->sizes.n_facet : 1);
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_facet = up(nf * sizeof(double4)), b_self = up((size_t)n * sizeof(double4)),
                 b_orphan = up((size_t)n * 4 * sizeof(double));
    const size_t b_box = c->box_given ? 0 : up(bwd_box_bytes(vd::bwd_waves(n)));
    const size_t need = b_facet + b_self + b_orphan + b_box;
    if (need > vd::kBwdScratchBytes)
        return fail(VD_ERR_INVALID_ARG, "vd_backward_noalloc: this diagram (" + std::to_string(n) + " sites, " +
                                            std::to_string(c->sizes.n_facet) + " facets) needs " +
                                            std::to_string(need) + " bytes of scratch, above the fixed " +
                                            std::to_string(vd::kBwdScratchBytes) + "; use vd_backward");
    unsigned char* base = static_cast<unsigned char*>(c->fixed_scratch);
    BwdScratch sc;
    sc.facet = reinterpret_cast<double4*>(base);
    sc.self = reinterpret_cast<double4*>(base + b_facet);
    sc.orphan = reinterpret_cast<double*>(base + b_facet + b_self);
    sc.box = c->box_given ? nullptr : reinterpret_cast<double*>(base + b_facet + b_self + b_orphan);
    return bwd_run(c, g_vol, g_cen, g_vert, g_xyz, g_w, sc, true, static_cast<hipStream_t>(stream));
}

VD_API vd_status vd_get_counters(const vd_context* c, uint64_t* out, int32_t count) {
    if (!c || !out || count < 0) return fail(VD_ERR_INVALID_ARG, "vd_get_counters: bad argument");
    if (!c->valid || !c->counted) return fail(VD_ERR_STATE, "vd_get_counters: last build did not count");
    unsigned long long h[vd::kTiers * vd::kCtrCount];
    VD_HIP(hipMemcpy(h, c->ctr.p, sizeof(h), hipMemcpyDeviceToHost));
    for (int k = 0; k < count && k < vd::kTiers * vd::kCtrCount; ++k) out[k] = (uint64_t)h[k];
    return VD_OK;
}

}  // extern "C"
