// gsr_api.cpp -- host side of the C ABI declared in include/gsr.h.
//
// A plan carries the host-known sizes (views, tiles, capacity, sort passes)
// and the layout of the caller's workspace; launches are enqueued on the
// caller's stream.  Kernel launch shapes depend only on the plan, never on
// device-side counts, so a call sequence can be captured into a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "gsr.h"
#include "kernels.h"
#include "order.h"

using namespace gsr;

static thread_local std::string g_err;

static gsr_status fail(gsr_status s, const char* what)
{
    g_err = what;
    return s;
}

static gsr_status hip_fail(hipError_t e, const char* where)
{
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return GSR_EHIP;
}

struct gsr_plan {
    int64_t n = 0;
    int32_t V = 0;
    gsr_config cfg{};
    DevCfg dcfg{};
    ViewTable vt{};
    int64_t capacity = 0;
    int64_t total_pixels = 0;
    int32_t total_tiles = 0, tile_bits = 0, passes = 0, chunks = 0, chunk_mult = 1, max_tiles_view = 0;
    int32_t bwd_blocks = 0, map_tiles = 0;
    size_t off_counters = 0, off_views = 0, off_geom = 0, off_conic = 0, off_rgbd = 0, off_qthr = 0, off_grad2d = 0, off_acc = 0;
    size_t off_stage = 0;
    size_t off_keys = 0, off_vals = 0, off_seg = 0, off_ranges = 0, off_cnt = 0;
    size_t off_live = 0, off_live_count = 0, off_live_mask = 0, off_fwd_queue = 0, off_tile_blocks = 0;
    int64_t mask_words = 0;     // ceil(n / 64): liveness ballot words per view
    size_t off_xip = 0, off_xip_sh = 0, off_order = 0, off_buckets = 0, off_track = 0, off_map = 0, off_stamps = 0, off_left = 0, total = 0;
    char* ws = nullptr;
    Counters host_counters{};
    std::vector<uint32_t> identity_order;
    // optional per-group device timing (host event objects only)
    bool timing = false;
    std::vector<hipEvent_t> event_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[GSR_T_COUNT];
    double timed_ms[GSR_T_COUNT] = {};
    int64_t timed_launches[GSR_T_COUNT] = {};
    // the long-segment sort runs on a second stream of the plan, forked from
    // and joined back to the caller's stream by two events (host objects,
    // created when the plan is bound; default stream priority)
    hipStream_t side = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;

    ~gsr_plan()
    {
        if (fork_ev) (void)hipEventDestroy(fork_ev);
        if (join_ev) (void)hipEventDestroy(join_ev);
        if (side) (void)hipStreamDestroy(side);
        for (auto& v : pending)
            for (auto& pr : v) {
                (void)hipEventDestroy(pr.first);
                (void)hipEventDestroy(pr.second);
            }
        for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    }
};

static hipEvent_t take_event(gsr_plan* p)
{
    if (!p->event_pool.empty()) {
        hipEvent_t e = p->event_pool.back();
        p->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

// Brackets one launch group with events on its stream while timing is on and
// the stream is not being captured.
class Timed {
public:
    Timed(gsr_plan* p, int group, hipStream_t s) : p_(p), group_(group), s_(s)
    {
        if (!p->timing) return;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
        e0_ = take_event(p);
        if (e0_ && hipEventRecord(e0_, s) != hipSuccess) {
            p->event_pool.push_back(e0_);
            e0_ = nullptr;
        }
    }
    ~Timed()
    {
        if (!e0_) return;
        hipEvent_t e1 = take_event(p_);
        if (e1 && hipEventRecord(e1, s_) == hipSuccess) {
            p_->pending[group_].push_back({e0_, e1});
            return;
        }
        p_->event_pool.push_back(e0_);
        if (e1) p_->event_pool.push_back(e1);
    }
    Timed(const Timed&) = delete;
    Timed& operator=(const Timed&) = delete;

private:
    gsr_plan* p_;
    int group_;
    hipStream_t s_;
    hipEvent_t e0_ = nullptr;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

static int ilog2(int x)
{
    int r = 0;
    while ((1 << r) < x) ++r;
    return r;
}

extern "C" gsr_status gsr_plan_create(int64_t n, int32_t n_views, const gsr_camera* cams, const gsr_config* cfg,
                                      int64_t pair_capacity, gsr_plan** out)
{
    g_err.clear();
    if (!out || !cams || !cfg) return fail(GSR_EINVAL, "null argument");
    *out = nullptr;
    if (n < 0) return fail(GSR_EINVAL, "n < 0");
    if (n_views < 1 || n_views > GSR_MAX_VIEWS) return fail(GSR_EINVAL, "n_views out of range");
    if ((uint64_t)n * (uint64_t)n_views >= (1ull << 32)) return fail(GSR_EINVAL, "n * n_views >= 2^32");
    if (pair_capacity < 0 || pair_capacity >= (int64_t)(1ull << 32))
        return fail(GSR_EINVAL, "pair_capacity out of range");
    if (!pow2(cfg->tile_w) || !pow2(cfg->tile_h)) return fail(GSR_EINVAL, "tile sizes must be powers of two");
    int tpx = cfg->tile_w * cfg->tile_h;
    if (tpx != 64 && tpx != 128 && tpx != 256 && tpx != 512)
        return fail(GSR_EUNSUPPORTED, "tile pixel count not in {64,128,256,512}");
    // the 64 lanes of a tile's wavefront own whole columns
    if (cfg->tile_w > 64) return fail(GSR_EUNSUPPORTED, "tile_w above 64");
    if (cfg->batch != 0 && cfg->batch != 64 && cfg->batch != 128 && cfg->batch != 256)
        return fail(GSR_EUNSUPPORTED, "batch must be 0 (default 128), 64, 128 or 256");
    if (cfg->sh_degree < -1 || cfg->sh_degree > 3) return fail(GSR_EINVAL, "sh_degree not in -1..3");
    if (!(cfg->alpha_min >= 0.0f) || !(cfg->alpha_max > 0.0f) || !(cfg->alpha_max <= 1.0f) ||
        !(cfg->alpha_min <= cfg->alpha_max))
        return fail(GSR_EINVAL, "alpha bounds");
    if (!(cfg->T_min >= 0.0f) || !(cfg->T_min < 1.0f)) return fail(GSR_EINVAL, "T_min");
    if (cfg->deterministic != 0 && cfg->deterministic != 1) return fail(GSR_EINVAL, "deterministic not 0 or 1");
    if (cfg->precision != GSR_PRECISION_FP32 && cfg->precision != GSR_PRECISION_MIXED)
        return fail(GSR_EINVAL, "precision not GSR_PRECISION_FP32 or GSR_PRECISION_MIXED");
    if (!(cfg->dilation >= 0.0f) || !std::isfinite(cfg->z_near)) return fail(GSR_EINVAL, "dilation / z_near");

    gsr_plan* p = new (std::nothrow) gsr_plan();
    if (!p) return fail(GSR_EINVAL, "out of host memory");
    p->n = n;
    p->V = n_views;
    p->cfg = *cfg;
    if (p->cfg.batch == 0) p->cfg.batch = 128;
    p->capacity = pair_capacity;
    p->dcfg.tile_w = cfg->tile_w;
    p->dcfg.tile_h = cfg->tile_h;
    p->dcfg.log2_tw = ilog2(cfg->tile_w);
    p->dcfg.log2_th = ilog2(cfg->tile_h);
    p->dcfg.sh_degree = cfg->sh_degree;
    p->dcfg.mixed = cfg->precision == GSR_PRECISION_MIXED ? 1 : 0;
    p->dcfg.z_near = cfg->z_near;
    p->dcfg.dilation = cfg->dilation;
    p->dcfg.alpha_min = cfg->alpha_min;
    p->dcfg.alpha_max = cfg->alpha_max;
    p->dcfg.T_min = cfg->T_min;
    p->dcfg.bg0 = cfg->bg[0];
    p->dcfg.bg1 = cfg->bg[1];
    p->dcfg.bg2 = cfg->bg[2];
    int64_t tiles = 0, pix = 0;
    p->vt.n = n_views;
    for (int v = 0; v < n_views; ++v) {
        const gsr_camera& c = cams[v];
        if (c.width <= 0 || c.height <= 0 || c.width > 65536 || c.height > 65536 ||
            !std::isfinite(c.fx) || !std::isfinite(c.fy) || !std::isfinite(c.cx) || !std::isfinite(c.cy)) {
            delete p;
            return fail(GSR_EINVAL, "camera");
        }
        ViewInfo& vi = p->vt.v[v];
        vi.width = c.width;
        vi.height = c.height;
        vi.tiles_x = (c.width + cfg->tile_w - 1) / cfg->tile_w;
        vi.tiles_y = (c.height + cfg->tile_h - 1) / cfg->tile_h;
        vi.tile_base = (int32_t)tiles;
        vi.pix_base = (int32_t)pix;
        vi.fx = c.fx;
        vi.fy = c.fy;
        vi.cx = c.cx;
        vi.cy = c.cy;
        tiles += (int64_t)vi.tiles_x * vi.tiles_y;
        pix += (int64_t)c.width * c.height;
        if (tiles >= (1ll << 31) || 3 * pix >= (1ll << 31)) {
            delete p;
            return fail(GSR_EINVAL, "too many tiles or pixels");
        }
    }
    p->vt.total_tiles = (int32_t)tiles;
    p->total_tiles = (int32_t)tiles;
    p->total_pixels = pix;
    p->tile_bits = tiles > 1 ? ilog2((int)tiles) : 0;
    // per-tile sort of (depth bits << 32 | index): at most 4 depth digits plus
    // the digits of the Gaussian index
    p->passes = 4 + (n > 1 ? (ilog2((int)std::min<int64_t>(n, 1ll << 30)) + 7) / 8 : 0);
    for (int v = 0; v < n_views; ++v)
        p->max_tiles_view = std::max(p->max_tiles_view, p->vt.v[v].tiles_x * p->vt.v[v].tiles_y);
    // binning chunks of GSR_BIN_CHUNK * chunk_mult live slots per block (the
    // slots of a view whose tile rectangle is not empty, listed by the
    // binning's first pass).  Each block writes a count row of its view's
    // tiles; one staged group per block measured best on MI355X (larger
    // chunks shorten the count matrix but leave fewer, longer blocks).  The
    // grid is sized for a view whose every slot is live, and blocks past a
    // view's live count exit at once
    p->chunk_mult = GSR_BIN_CHUNK_MULT;
    p->chunks = (int32_t)std::max<int64_t>(
        1, (n + (int64_t)GSR_BIN_CHUNK * p->chunk_mult - 1) / ((int64_t)GSR_BIN_CHUNK * p->chunk_mult));
    p->bwd_blocks = (int32_t)((n + 255) / 256);
    if (p->bwd_blocks == 0) p->bwd_blocks = 1;

    const int64_t S = n * n_views;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + (bytes ? bytes : 1));
        return at;
    };
    p->off_counters = take(sizeof(Counters));
    p->off_views = take(sizeof(ViewTable));
    p->off_geom = take(sizeof(float4) * S);
    p->off_conic = take(sizeof(float4) * S);
    p->off_rgbd = take(sizeof(float4) * S);
    p->off_qthr = take(sizeof(float) * S);
    p->off_stage = take(sizeof(StageRec) * S);
    p->off_grad2d = take(sizeof(double) * GSR_G2 * S);
    p->off_acc = take(cfg->deterministic ? sizeof(unsigned long long) * GSR_G2 * GSR_FIX_LIMBS * S : 0);
    p->off_keys = take(sizeof(unsigned long long) * pair_capacity);
    p->off_vals = take(sizeof(uint32_t) * pair_capacity);
    p->off_seg = take(sizeof(unsigned long long) * pair_capacity);
    p->off_ranges = take(sizeof(uint2) * tiles);
    p->off_order = take(sizeof(uint32_t) * tiles);
    p->off_buckets = take(sizeof(uint32_t) * 66);
    p->off_fwd_queue = take(sizeof(uint32_t));
    p->off_cnt = take(sizeof(uint32_t) * (size_t)p->chunks * (size_t)tiles);
    p->mask_words = (n + 63) / 64;
    p->off_live_mask = take(sizeof(uint64_t) * (size_t)n_views * (size_t)p->mask_words);
    p->off_live = take(sizeof(uint32_t) * S);

    p->off_live_count = take(sizeof(uint32_t) * GSR_LIVE_STRIDE * GSR_MAX_VIEWS);  // one 256-byte line per view
    p->off_tile_blocks = take(sizeof(unsigned long long) * (size_t)((p->total_tiles + 63) / 64 + 1));
    p->off_xip = take(sizeof(double) * 6 * (size_t)n_views * p->bwd_blocks);
    p->off_xip_sh = take(sizeof(double) * 6 * (size_t)n_views * p->bwd_blocks);
    p->off_track = take(sizeof(double) * GSR_TRACK_SLOTS * GSR_TRACK_BLOCKS * (size_t)n_views);
    for (int v = 0; v < n_views; ++v)
        p->map_tiles = std::max(p->map_tiles, ((p->vt.v[v].width + 31) / 32) * ((p->vt.v[v].height + 31) / 32));
    p->off_map = take(sizeof(double) * 2 * (size_t)p->map_tiles * (size_t)n_views);
    p->off_stamps = take(sizeof(unsigned long long) * ((size_t)n_views + 1));
    p->off_left = take(sizeof(unsigned long long) * (size_t)n_views);
    p->total = o;
    p->host_counters = Counters{};
    p->host_counters.capacity = (unsigned long long)pair_capacity;
    *out = p;
    return GSR_OK;
}

extern "C" void gsr_plan_destroy(gsr_plan* plan) { delete plan; }

extern "C" size_t gsr_plan_workspace_bytes(const gsr_plan* plan) { return plan ? plan->total : 0; }

extern "C" gsr_status gsr_plan_bind(gsr_plan* plan, void* workspace, size_t bytes, void* stream)
{
    g_err.clear();
    if (!plan || !workspace) return fail(GSR_EINVAL, "null argument");
    if (bytes < plan->total) return fail(GSR_EINVAL, "workspace too small");
    if (((uintptr_t)workspace & 255) != 0) return fail(GSR_EINVAL, "workspace not 256-byte aligned");
    plan->ws = (char*)workspace;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(plan->ws + plan->off_counters, &plan->host_counters, sizeof(Counters),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(plan->ws + plan->off_views, &plan->vt, sizeof(ViewTable), hipMemcpyHostToDevice, s);
    // empty tile ranges and an identity tile order until the first binning
    if (e == hipSuccess)
        e = hipMemsetAsync(plan->ws + plan->off_ranges, 0, sizeof(uint2) * (size_t)plan->total_tiles, s);
    // the per-view tile counters of the completion stamps start at zero, and
    // the live lists empty until the first projection
    if (e == hipSuccess)
        e = hipMemsetAsync(plan->ws + plan->off_left, 0, sizeof(unsigned long long) * (size_t)plan->V, s);
    if (e == hipSuccess)
        e = hipMemsetAsync(plan->ws + plan->off_live_mask, 0, sizeof(uint64_t) * (size_t)plan->V * plan->mask_words, s);
    // every slot starts culled (NaN geometry): the projection rewrites the
    // culled marker only where a slot was live at the previous projection
    if (e == hipSuccess)
        e = hipMemsetAsync(plan->ws + plan->off_geom, 0xff, sizeof(float4) * (size_t)plan->V * (size_t)plan->n, s);
    if (e == hipSuccess) {
        plan->identity_order.resize((size_t)plan->total_tiles);
        for (int32_t t = 0; t < plan->total_tiles; ++t) plan->identity_order[(size_t)t] = (uint32_t)t;
        e = hipMemcpyAsync(plan->ws + plan->off_order, plan->identity_order.data(),
                           sizeof(uint32_t) * (size_t)plan->total_tiles, hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && !plan->side) e = hipStreamCreateWithFlags(&plan->side, hipStreamNonBlocking);
    if (e == hipSuccess && !plan->fork_ev) e = hipEventCreateWithFlags(&plan->fork_ev, hipEventDisableTiming);
    if (e == hipSuccess && !plan->join_ev) e = hipEventCreateWithFlags(&plan->join_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        plan->ws = nullptr;
        return hip_fail(e, "gsr_plan_bind");
    }
    return GSR_OK;
}


extern "C" gsr_status gsr_plan_layout(const gsr_plan* plan, gsr_layout* out)
{
    if (!plan || !out) return fail(GSR_EINVAL, "null argument");
    out->counters = plan->off_counters;
    out->geom = plan->off_geom;
    out->conic_o = plan->off_conic;
    out->rgb_d = plan->off_rgbd;
    out->qthr = plan->off_qthr;
    out->stage = plan->off_stage;
    out->grad2d = plan->off_grad2d;
    out->keys = plan->off_keys;
    out->vals = plan->off_vals;
    out->ranges = plan->off_ranges;
    out->stamps = plan->off_stamps;
    out->live_mask = plan->off_live_mask;
    out->total = plan->total;
    return GSR_OK;
}

extern "C" gsr_status gsr_plan_get_info(const gsr_plan* plan, gsr_plan_info* out)
{
    if (!plan || !out) return fail(GSR_EINVAL, "null argument");
    out->n = plan->n;
    out->slots = plan->n * plan->V;
    out->capacity = plan->capacity;
    out->total_pixels = plan->total_pixels;
    out->n_views = plan->V;
    out->total_tiles = plan->total_tiles;
    out->sort_passes = plan->passes;
    out->tile_bits = plan->tile_bits;
    return GSR_OK;
}

template <class T>
static T* at(const gsr_plan* p, size_t off)
{
    return reinterpret_cast<T*>(p->ws + off);
}

static gsr_status check_bound(const gsr_plan* p)
{
    if (!p) return fail(GSR_EINVAL, "null plan");
    if (!p->ws) return fail(GSR_ESTATE, "plan not bound to a workspace");
    return GSR_OK;
}

static gsr_status check_gaussians(const gsr_plan* p, const gsr_gaussians* g)
{
    if (!g) return fail(GSR_EINVAL, "null gaussians");
    if (g->n != p->n) return fail(GSR_EINVAL, "gaussian count differs from the plan");
    if (p->n > 0 && (!g->mean || !g->quat || !g->log_scale || !g->opacity_logit || !g->colour))
        return fail(GSR_EINVAL, "null parameter plane");
    return GSR_OK;
}

extern "C" gsr_status gsr_project(gsr_plan* plan, const gsr_gaussians* g, const float* poses, void* stream)
{
    g_err.clear();
    gsr_status st = check_bound(plan);
    if (st != GSR_OK) return st;
    if ((st = check_gaussians(plan, g)) != GSR_OK) return st;
    if (!poses) return fail(GSR_EINVAL, "null poses");
    ProjectArgs a{};
    a.n = plan->n;
    a.mean = g->mean;
    a.quat = g->quat;
    a.log_scale = g->log_scale;
    a.opacity_logit = g->opacity_logit;
    a.colour = g->colour;
    a.poses = poses;
    a.views = at<ViewTable>(plan, plan->off_views);
    a.cfg = plan->dcfg;
    a.geom = at<float4>(plan, plan->off_geom);
    a.conic_o = at<float4>(plan, plan->off_conic);
    a.rgb_d = at<float4>(plan, plan->off_rgbd);
    a.qthr = at<float>(plan, plan->off_qthr);
    a.stage = at<void>(plan, plan->off_stage);
    a.grad2d = at<double>(plan, plan->off_grad2d);
    a.acc = plan->cfg.deterministic ? at<unsigned long long>(plan, plan->off_acc) : nullptr;
    a.stamps = at<unsigned long long>(plan, plan->off_stamps);
    a.counters = at<Counters>(plan, plan->off_counters);
    a.live_mask = at<uint64_t>(plan, plan->off_live_mask);
    a.mask_words = plan->mask_words;
    Timed t(plan, GSR_T_PROJECT, (hipStream_t)stream);
    hipError_t e = launch_project(a, plan->cfg.sh_degree, (hipStream_t)stream);
    return e == hipSuccess ? GSR_OK : hip_fail(e, "gsr_project");
}

extern "C" gsr_status gsr_bin(gsr_plan* plan, void* stream)
{
    g_err.clear();
    gsr_status st = check_bound(plan);
    if (st != GSR_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    BinArgs b{};
    b.n = plan->n;
    b.n_views = plan->V;
    b.views = at<ViewTable>(plan, plan->off_views);
    b.cfg = plan->dcfg;
    b.geom = at<float4>(plan, plan->off_geom);
    b.rgb_d = at<float4>(plan, plan->off_rgbd);
    b.conic_o = at<float4>(plan, plan->off_conic);
    b.qthr = at<float>(plan, plan->off_qthr);
    b.chunks = plan->chunks;
    b.chunk_mult = plan->chunk_mult;
    b.total_tiles = plan->total_tiles;
    b.cnt = at<uint32_t>(plan, plan->off_cnt);
    b.live_mask = at<uint64_t>(plan, plan->off_live_mask);
    b.mask_words = plan->mask_words;
    b.live = at<uint32_t>(plan, plan->off_live);
    b.live_count = at<uint32_t>(plan, plan->off_live_count);
    b.tile_blocks = at<unsigned long long>(plan, plan->off_tile_blocks);
    b.counters = at<Counters>(plan, plan->off_counters);
    b.ranges = at<uint2>(plan, plan->off_ranges);
    b.seg = at<unsigned long long>(plan, plan->off_seg);
    RangeArgs r{};
    r.counters = b.counters;
    r.ranges = b.ranges;
    r.total_tiles = plan->total_tiles;
    r.order = at<uint32_t>(plan, plan->off_order);
    r.buckets = at<uint32_t>(plan, plan->off_buckets);
    SegArgs g{};
    g.counters = b.counters;
    g.views = b.views;
    g.ranges = b.ranges;
    g.order = r.order;
    g.seg = b.seg;
    g.keys = at<unsigned long long>(plan, plan->off_keys);
    g.vals = at<uint32_t>(plan, plan->off_vals);
    g.queue = r.buckets + 64;
    g.n = plan->n;
    hipError_t e;
    {
        Timed t(plan, GSR_T_BIN_EMIT, s);
        e = launch_bin(b, plan->max_tiles_view, s);
    }
    if (e != hipSuccess) return hip_fail(e, "gsr_bin: emit");
    {
        Timed t(plan, GSR_T_BIN_RANGES, s);
        e = launch_order(r, s);
    }
    if (e != hipSuccess) return hip_fail(e, "gsr_bin: order");
    {
        Timed t(plan, GSR_T_BIN_SORT, s);
        e = launch_seg_sort(g, plan->total_tiles, plan->capacity, s, plan->side, plan->fork_ev, plan->join_ev);
    }
    return e == hipSuccess ? GSR_OK : hip_fail(e, "gsr_bin: sort");
}

static RasterArgs raster_args(const gsr_plan* plan)
{
    RasterArgs a{};
    a.views = at<ViewTable>(plan, plan->off_views);
    a.cfg = plan->dcfg;
    a.counters = at<Counters>(plan, plan->off_counters);
    a.ranges = at<uint2>(plan, plan->off_ranges);
    a.order = at<uint32_t>(plan, plan->off_order);
    a.vals = at<uint32_t>(plan, plan->off_vals);
    a.geom = at<float4>(plan, plan->off_geom);
    a.stage = at<void>(plan, plan->off_stage);
    a.grad2d = at<double>(plan, plan->off_grad2d);
    a.acc = plan->cfg.deterministic ? at<unsigned long long>(plan, plan->off_acc) : nullptr;
    a.slots = plan->n * plan->V;
    a.tiles_done = at<unsigned long long>(plan, plan->off_left);
    a.stamps = at<unsigned long long>(plan, plan->off_stamps);
    a.fwd_queue = at<uint32_t>(plan, plan->off_fwd_queue);
    return a;
}

extern "C" gsr_status gsr_render_fwd(gsr_plan* plan, void* rgb, float* T_final, int32_t* n_contrib,
                                     int32_t* n_blend, void* stream)
{
    g_err.clear();
    gsr_status st = check_bound(plan);
    if (st != GSR_OK) return st;
    if (!rgb || !T_final || !n_contrib) return fail(GSR_EINVAL, "null output");
    RasterArgs a = raster_args(plan);
    a.rgb = rgb;
    a.T_final = T_final;
    a.n_contrib = n_contrib;
    a.n_blend = n_blend;
    Timed t(plan, GSR_T_RASTER_FWD, (hipStream_t)stream);
    hipError_t e = launch_raster_fwd(a, plan->total_tiles, plan->cfg.tile_w * plan->cfg.tile_h, plan->cfg.batch,
                                     (hipStream_t)stream, plan->side, plan->fork_ev, plan->join_ev);
    return e == hipSuccess ? GSR_OK : hip_fail(e, "gsr_render_fwd");
}

extern "C" gsr_status gsr_loss_l1(gsr_plan* plan, const void* rgb, const float* target, float* dL_drgb,
                                  void* stream)
{
    g_err.clear();
    if (!plan) return fail(GSR_EINVAL, "null plan");
    if (!rgb || !target || !dL_drgb) return fail(GSR_EINVAL, "null buffer");
    LossArgs a{};
    a.rgb = rgb;
    a.half_image = plan->dcfg.mixed;
    a.target = target;
    a.dL_drgb = dL_drgb;
    a.count = 3 * plan->total_pixels;
    a.scale = a.count ? 1.0f / (float)a.count : 0.0f;
    Timed t(plan, GSR_T_LOSS_L1, (hipStream_t)stream);
    hipError_t e = launch_loss_l1(a, (hipStream_t)stream);
    return e == hipSuccess ? GSR_OK : hip_fail(e, "gsr_loss_l1");
}

extern "C" gsr_status gsr_loss_track(gsr_plan* plan, const float* rgb, const float* T_final, const float* target,
                                     double tau_alpha, double tau_grad, double* loss, double* exposure,
                                     float* dL_drgb, float* dL_dT, void* stream)
{
    g_err.clear();
    if (!plan) return fail(GSR_EINVAL, "null plan");
    if (!rgb || !T_final || !target || !loss || !exposure || !dL_drgb) return fail(GSR_EINVAL, "null buffer");
    if (!(tau_alpha > 0.0) || !(tau_grad > 0.0) || !std::isfinite(tau_alpha) || !std::isfinite(tau_grad))
        return fail(GSR_EINVAL, "tau_alpha and tau_grad must be positive and finite");
    if (plan->dcfg.mixed) return fail(GSR_EUNSUPPORTED, "gsr_loss_track reads float32 images (mixed plan)");
    gsr_status st = check_bound(plan);
    if (st != GSR_OK) return st;
    TrackArgs a{};
    a.views = at<ViewTable>(plan, plan->off_views);
    a.rgb = rgb;
    a.T_final = T_final;
    a.target = target;
    a.tau_alpha = tau_alpha;
    a.tau_grad = tau_grad;
    a.part = at<double>(plan, plan->off_track);
    a.loss = loss;
    a.exposure = exposure;
    a.dL_drgb = dL_drgb;
    a.dL_dT = dL_dT;
    Timed t(plan, GSR_T_LOSS_TRACK, (hipStream_t)stream);
    hipError_t e = launch_loss_track(a, plan->V, (hipStream_t)stream);
    return e == hipSuccess ? GSR_OK : hip_fail(e, "gsr_loss_track");
}

extern "C" gsr_status gsr_loss_mapping(gsr_plan* plan, const float* rgb, const float* target, double lambda,
                                       double* loss, float* dL_drgb, void* stream)
{
    g_err.clear();
    if (!plan) return fail(GSR_EINVAL, "null plan");
    if (!rgb || !target || !loss || !dL_drgb) return fail(GSR_EINVAL, "null buffer");
    if (!(lambda >= 0.0 && lambda <= 1.0)) return fail(GSR_EINVAL, "lambda must lie in [0, 1]");
    if (plan->dcfg.mixed) return fail(GSR_EUNSUPPORTED, "gsr_loss_mapping reads float32 images (mixed plan)");
    gsr_status st = check_bound(plan);
    if (st != GSR_OK) return st;
    MapLossArgs a{};
    a.views = at<ViewTable>(plan, plan->off_views);
    a.rgb = rgb;
    a.target = target;
    // the Gaussian window of standard deviation 1.5 over offsets -5..5,
    // normalised to sum 1
    double w[11], wsum = 0.0;
    for (int i = 0; i < 11; ++i) {
        const double d = (double)(i - 5);
        w[i] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
        wsum += w[i];
    }
    for (int i = 0; i < 11; ++i) a.w[i] = (float)(w[i] / wsum);
    a.c1 = (float)(0.01 * 0.01);
    a.c2 = (float)(0.03 * 0.03);
    const double n = 3.0 * (double)plan->total_pixels;
    a.lambda = lambda;
    a.inv_n = 1.0 / n;
    a.scale_ssim = (float)(-lambda / n);
    a.scale_l1 = (float)((1.0 - lambda) / n);
    a.max_tiles = plan->map_tiles;
    a.part = at<double>(plan, plan->off_map);
    a.loss = loss;
    a.dL_drgb = dL_drgb;
    Timed t(plan, GSR_T_LOSS_MAP, (hipStream_t)stream);
    hipError_t e = launch_loss_mapping(a, plan->V, (hipStream_t)stream);
    return e == hipSuccess ? GSR_OK : hip_fail(e, "gsr_loss_mapping");
}

extern "C" gsr_status gsr_raster_bwd(gsr_plan* plan, const float* T_final, const int32_t* n_contrib,
                                     const float* dL_drgb, const float* dL_dT, void* stream)
{
    g_err.clear();
    gsr_status st = check_bound(plan);
    if (st != GSR_OK) return st;
    if (!dL_drgb || !T_final || !n_contrib) return fail(GSR_EINVAL, "null T_final, n_contrib or dL_drgb");
    RasterArgs a = raster_args(plan);
    a.T_final_in = T_final;
    a.n_contrib_in = n_contrib;
    a.dL_drgb = dL_drgb;
    a.dL_dT = dL_dT;
    hipError_t e;
    {
        Timed t(plan, GSR_T_CLEAR_GRAD2D, (hipStream_t)stream);
        e = launch_clear_grad2d(a, (hipStream_t)stream);
    }
    if (e != hipSuccess) return hip_fail(e, "gsr_raster_bwd: clear");
    Timed t(plan, GSR_T_RASTER_BWD, (hipStream_t)stream);
    e = launch_raster_bwd(a, plan->total_tiles, plan->cfg.tile_w * plan->cfg.tile_h, plan->cfg.batch,
                          (hipStream_t)stream);
    return e == hipSuccess ? GSR_OK : hip_fail(e, "gsr_raster_bwd");
}

extern "C" gsr_status gsr_project_bwd(gsr_plan* plan, const gsr_gaussians* g, const float* poses,
                                      const uint8_t* pose_only, gsr_grads* grads, float* d_xi, void* stream)
{
    g_err.clear();
    gsr_status st = check_bound(plan);
    if (st != GSR_OK) return st;
    if ((st = check_gaussians(plan, g)) != GSR_OK) return st;
    if (!poses) return fail(GSR_EINVAL, "null poses");
    if (grads && plan->n > 0 &&
        (!grads->d_mean || !grads->d_quat || !grads->d_log_scale || !grads->d_opacity_logit || !grads->d_colour))
        return fail(GSR_EINVAL, "null gradient plane");
    ProjectBwdArgs b{};
    b.n = plan->n;
    b.mean = g->mean;
    b.quat = g->quat;
    b.log_scale = g->log_scale;
    b.opacity_logit = g->opacity_logit;
    b.colour = g->colour;
    b.poses = poses;
    b.views = at<ViewTable>(plan, plan->off_views);
    b.cfg = plan->dcfg;
    b.live_mask = at<uint64_t>(plan, plan->off_live_mask);
    b.grad2d = at<double>(plan, plan->off_grad2d);
    unsigned long long mask = 0;
    for (int v = 0; v < plan->V; ++v)
        if (pose_only && pose_only[v]) mask |= 1ull << v;
    // without gradient planes every view is pose-only and no parameter store happens
    if (!grads) mask = ~0ull;
    b.pose_only = mask;
    b.d_mean = grads ? grads->d_mean : nullptr;
    b.d_quat = grads ? grads->d_quat : nullptr;
    b.d_log_scale = grads ? grads->d_log_scale : nullptr;
    b.d_opacity_logit = grads ? grads->d_opacity_logit : nullptr;
    b.d_colour = grads ? grads->d_colour : nullptr;
    b.xi_partial = at<double>(plan, plan->off_xip);
    b.xi_partial_sh = at<double>(plan, plan->off_xip_sh);
    b.blocks = plan->bwd_blocks;
    Timed t(plan, GSR_T_PROJECT_BWD, (hipStream_t)stream);
    hipError_t e = launch_project_bwd(b, plan->cfg.sh_degree, d_xi, plan->V, (hipStream_t)stream);
    return e == hipSuccess ? GSR_OK : hip_fail(e, "gsr_project_bwd");
}

extern "C" gsr_status gsr_render_bwd(gsr_plan* plan, const gsr_gaussians* g, const float* poses,
                                     const float* T_final, const int32_t* n_contrib, const float* dL_drgb,
                                     const float* dL_dT, const uint8_t* pose_only, gsr_grads* grads, float* d_xi,
                                     void* stream)
{
    gsr_status st = check_bound(plan);
    if (st != GSR_OK) return st;
    if ((st = check_gaussians(plan, g)) != GSR_OK) return st;
    if (!poses) return fail(GSR_EINVAL, "null poses");
    st = gsr_raster_bwd(plan, T_final, n_contrib, dL_drgb, dL_dT, stream);
    if (st != GSR_OK) return st;
    return gsr_project_bwd(plan, g, poses, pose_only, grads, d_xi, stream);
}

extern "C" gsr_status gsr_pair_count(gsr_plan* plan, int64_t* required, int32_t* overflow, void* stream)
{
    g_err.clear();
    gsr_status st = check_bound(plan);
    if (st != GSR_OK) return st;
    Counters c{};
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(&c, plan->ws + plan->off_counters, sizeof(Counters), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "gsr_pair_count");
    if (required) *required = (int64_t)c.pairs;
    if (overflow) *overflow = (int32_t)c.overflow;
    return c.overflow ? GSR_ECAPACITY : GSR_OK;
}

extern "C" gsr_status gsr_plan_set_timing(gsr_plan* plan, int32_t enable)
{
    g_err.clear();
    if (!plan) return fail(GSR_EINVAL, "null plan");
    for (auto& v : plan->pending) {
        for (auto& pr : v) {
            plan->event_pool.push_back(pr.first);
            plan->event_pool.push_back(pr.second);
        }
        v.clear();
    }
    for (int k = 0; k < GSR_T_COUNT; ++k) {
        plan->timed_ms[k] = 0.0;
        plan->timed_launches[k] = 0;
    }
    plan->timing = enable != 0;
    return GSR_OK;
}

extern "C" gsr_status gsr_plan_read_timing(gsr_plan* plan, int32_t timer, double* total_ms, int64_t* launches)
{
    g_err.clear();
    if (!plan) return fail(GSR_EINVAL, "null plan");
    if (timer < 0 || timer >= GSR_T_COUNT) return fail(GSR_EINVAL, "unknown timer");
    auto& v = plan->pending[timer];
    size_t done = 0;
    hipError_t e = hipSuccess;
    for (; done < v.size(); ++done) {
        e = hipEventSynchronize(v[done].second);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, v[done].first, v[done].second);
        if (e != hipSuccess) break;
        plan->timed_ms[timer] += ms;
        plan->timed_launches[timer] += 1;
        plan->event_pool.push_back(v[done].first);
        plan->event_pool.push_back(v[done].second);
    }
    v.erase(v.begin(), v.begin() + (std::ptrdiff_t)done);
    if (e != hipSuccess) return hip_fail(e, "gsr_plan_read_timing");
    if (total_ms) *total_ms = plan->timed_ms[timer];
    if (launches) *launches = plan->timed_launches[timer];
    return GSR_OK;
}

extern "C" const char* gsr_status_str(gsr_status s)
{
    switch (s) {
    case GSR_OK: return "ok";
    case GSR_EINVAL: return "invalid argument";
    case GSR_ECAPACITY: return "pair capacity exceeded";
    case GSR_EHIP: return "HIP error";
    case GSR_EUNSUPPORTED: return "unsupported configuration";
    case GSR_ESTATE: return "plan not bound";
    }
    return "unknown status";
}

extern "C" const char* gsr_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// one-shot seeding

extern "C" gsr_status gsr_seed_triangulate(int64_t n, int32_t n_neighbours, const gsr_seed_view* views,
                                           const gsr_seed_config* cfg, const float* x_ref, const float* x_nb,
                                           const float* kappa, float* mean, float* colour, float* opacity_logit,
                                           int32_t* valid, int32_t* best, float* err, float* angle, float* kappa_bar,
                                           void* stream)
{
    g_err.clear();
    if (n < 0 || n >= (1ll << 31)) return fail(GSR_EINVAL, "n out of range");
    if (n_neighbours < 1 || n_neighbours > GSR_SEED_MAX_NEIGHBOURS) return fail(GSR_EINVAL, "n_neighbours out of range");
    if (!views || !cfg) return fail(GSR_EINVAL, "null views or config");
    if (!(cfg->max_reproj > 0.0) || !(cfg->min_parallax >= 0.0) || !(cfg->alpha_lo > 0.0) ||
        !(cfg->alpha_lo <= cfg->alpha_hi) || !(cfg->alpha_hi < 1.0))
        return fail(GSR_EINVAL, "config: need max_reproj > 0, min_parallax >= 0, 0 < alpha_lo <= alpha_hi < 1");
    SeedArgs a{};
    for (int v = 0; v <= n_neighbours; ++v) {
        const gsr_seed_view& s = views[v];
        if (s.width < 1 || s.height < 1 || !s.image) return fail(GSR_EINVAL, "view without an image");
        if (!(s.gain != 0.0) || !std::isfinite(s.gain) || !std::isfinite(s.bias))
            return fail(GSR_EINVAL, "view exposure: gain must be finite and non-zero");
        SeedView& d = a.views[v];
        for (int k = 0; k < 12; ++k) d.P[k] = s.P[k];
        for (int k = 0; k < 3; ++k) d.centre[k] = s.centre[k];
        d.width = s.width;
        d.height = s.height;
        d.image = s.image;
        d.gain = s.gain;
        d.bias = s.bias;
    }
    if (n == 0) return GSR_OK;
    if (!x_ref || !x_nb || !kappa || !mean || !colour || !opacity_logit || !valid)
        return fail(GSR_EINVAL, "null buffer");
    a.n = n;
    a.K = n_neighbours;
    a.max_reproj = cfg->max_reproj;
    a.min_parallax = cfg->min_parallax;
    a.alpha_lo = cfg->alpha_lo;
    a.alpha_hi = cfg->alpha_hi;
    a.x_ref = x_ref;
    a.x_nb = x_nb;
    a.kappa = kappa;
    a.mean = mean;
    a.colour = colour;
    a.opacity_logit = opacity_logit;
    a.valid = valid;
    a.best = best;
    a.err = err;
    a.angle = angle;
    a.kappa_bar = kappa_bar;
    hipError_t e = launch_seed_triangulate(a, (hipStream_t)stream);
    return e == hipSuccess ? GSR_OK : hip_fail(e, "gsr_seed_triangulate");
}

namespace {
struct KnnLayout {
    size_t bpart, grid, cell_count, cell_start, cell_of, rank, sorted, total;
    size_t opart, fine_count, fine_start, fine_of, fine_rank, fine_pts, cell_pts, scan_tot, bf_list, bf_count;
    int64_t max_cells;
    int32_t table_bits;
};

KnnLayout knn_layout(int64_t n)
{
    KnnLayout L{};
    L.max_cells = 4 * n + 64;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + (bytes ? bytes : 1));
        return at;
    };
    L.bpart = take(sizeof(float) * 8 * GSR_KNN_BLOCKS);
    L.grid = take(sizeof(KnnGrid));
    L.cell_count = take(sizeof(uint32_t) * (size_t)(L.max_cells + 1));
    L.cell_start = take(sizeof(uint32_t) * (size_t)(L.max_cells + 1));
    L.cell_of = take(sizeof(uint32_t) * (size_t)n);
    L.rank = take(sizeof(uint32_t) * (size_t)n);
    L.sorted = take(sizeof(uint32_t) * (size_t)n);
    // fine grid: a hash table of at least two buckets per seed
    L.table_bits = 10;
    while (((int64_t)1 << L.table_bits) < 2 * n) ++L.table_bits;
    const int64_t T = (int64_t)1 << L.table_bits;
    L.opart = take(sizeof(double) * GSR_KNN_BLOCKS);
    L.fine_count = take(sizeof(uint32_t) * GSR_KNN_LEVELS * (size_t)(T + 1));
    L.fine_start = take(sizeof(uint32_t) * GSR_KNN_LEVELS * (size_t)(T + 1));
    L.fine_of = take(sizeof(uint32_t) * GSR_KNN_LEVELS * (size_t)n);
    L.fine_rank = take(sizeof(uint32_t) * GSR_KNN_LEVELS * (size_t)n);
    L.fine_pts = take(sizeof(float) * 4 * GSR_KNN_LEVELS * (size_t)n);
    L.cell_pts = take(sizeof(float) * 4 * (size_t)n);
    const int64_t scan_blocks = std::max((L.max_cells + 1 + 1023) / 1024, (T + 1 + 1023) / 1024);
    L.scan_tot = take(sizeof(uint32_t) * (size_t)scan_blocks);
    L.bf_list = take(sizeof(uint32_t) * (size_t)n);
    L.bf_count = take(sizeof(uint32_t));
    L.total = o;
    return L;
}
}  // namespace

extern "C" size_t gsr_seed_scale_workspace_bytes(int64_t n)
{
    if (n < 0 || n >= (1ll << 31)) return 0;
    return knn_layout(n).total;
}

static KnnArgs knn_args(int64_t n, const float* mean, const int32_t* valid, float floor_scale, void* workspace,
                        const KnnLayout& L)
{
    char* ws = (char*)workspace;
    KnnArgs a{};
    a.n = n;
    a.mean = mean;
    a.valid = valid;
    a.floor_scale = floor_scale;
    a.max_cells = L.max_cells;
    a.bpart = (float*)(ws + L.bpart);
    a.grid = (KnnGrid*)(ws + L.grid);
    a.cell_count = (uint32_t*)(ws + L.cell_count);
    a.cell_start = (uint32_t*)(ws + L.cell_start);
    a.cell_of = (uint32_t*)(ws + L.cell_of);
    a.rank = (uint32_t*)(ws + L.rank);
    a.sorted = (uint32_t*)(ws + L.sorted);
    a.table_bits = L.table_bits;
    a.opart = (double*)(ws + L.opart);
    a.fine_count = (uint32_t*)(ws + L.fine_count);
    a.fine_start = (uint32_t*)(ws + L.fine_start);
    a.fine_of = (uint32_t*)(ws + L.fine_of);
    a.fine_rank = (uint32_t*)(ws + L.fine_rank);
    a.fine_pts = (float4*)(ws + L.fine_pts);
    a.cell_pts = (float4*)(ws + L.cell_pts);
    a.scan_tot = (uint32_t*)(ws + L.scan_tot);
    a.bf_list = (uint32_t*)(ws + L.bf_list);
    a.bf_count = (uint32_t*)(ws + L.bf_count);
    return a;
}

static gsr_status knn_run(int64_t n, const float* mean, const int32_t* valid, float floor_scale, void* workspace,
                          size_t workspace_bytes, float* log_scale, int32_t* nn_index, void* stream, const char* who)
{
    const KnnLayout L = knn_layout(n);
    if (workspace_bytes < L.total) return fail(GSR_EINVAL, "workspace too small");
    KnnArgs a = knn_args(n, mean, valid, floor_scale, workspace, L);
    a.log_scale = log_scale;
    a.nn_index = nn_index;
    hipError_t e = launch_seed_scale(a, (hipStream_t)stream);
    return e == hipSuccess ? GSR_OK : hip_fail(e, who);
}

extern "C" gsr_status gsr_seed_frame(int64_t n, const float* mean, const int32_t* valid, const float* err,
                                     const float* angle, const double* P_ref, const double* centre_ref, double radius,
                                     double c_par, float floor_scale, void* workspace, size_t workspace_bytes,
                                     float* quat, float* log_scale, void* stream)
{
    g_err.clear();
    if (n < 0 || n >= (1ll << 31)) return fail(GSR_EINVAL, "n out of range");
    if (!P_ref || !centre_ref) return fail(GSR_EINVAL, "null reference view");
    if (!(radius > 0.0) || !std::isfinite(radius)) return fail(GSR_EINVAL, "radius must be positive and finite");
    if (!(c_par > 0.0) || !std::isfinite(c_par)) return fail(GSR_EINVAL, "c_par must be positive and finite");
    if (!(floor_scale > 0.0f) || !std::isfinite(floor_scale)) return fail(GSR_EINVAL, "floor_scale must be positive");
    for (int k = 0; k < 12; ++k)
        if (!std::isfinite(P_ref[k])) return fail(GSR_EINVAL, "non-finite projection");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(centre_ref[k])) return fail(GSR_EINVAL, "non-finite centre");
    if (n == 0) return GSR_OK;
    if (!mean || !valid || !err || !angle || !quat || !log_scale || !workspace) return fail(GSR_EINVAL, "null buffer");
    const KnnLayout L = knn_layout(n);
    if (workspace_bytes < L.total) return fail(GSR_EINVAL, "workspace too small");
    KnnArgs a = knn_args(n, mean, valid, floor_scale, workspace, L);
    a.fine_levels = 1;  // only the level of cells of the radius
    FrameArgs f{};
    for (int k = 0; k < 12; ++k) f.P[k] = P_ref[k];
    for (int k = 0; k < 3; ++k) f.centre[k] = centre_ref[k];
    f.radius = radius;
    f.c_par = c_par;
    f.floor_scale = floor_scale;
    f.err = err;
    f.angle = angle;
    f.quat = quat;
    f.log_scale = log_scale;
    hipError_t e = launch_seed_frame(a, f, (hipStream_t)stream);
    return e == hipSuccess ? GSR_OK : hip_fail(e, "gsr_seed_frame");
}

extern "C" gsr_status gsr_seed_scale(int64_t n, const float* mean, const int32_t* valid, float floor_scale,
                                     void* workspace, size_t workspace_bytes, float* log_scale, void* stream)
{
    g_err.clear();
    if (n < 0 || n >= (1ll << 31)) return fail(GSR_EINVAL, "n out of range");
    if (!(floor_scale > 0.0f) || !std::isfinite(floor_scale)) return fail(GSR_EINVAL, "floor_scale must be positive");
    if (n == 0) return GSR_OK;
    if (!mean || !valid || !log_scale || !workspace) return fail(GSR_EINVAL, "null buffer");
    return knn_run(n, mean, valid, floor_scale, workspace, workspace_bytes, log_scale, nullptr, stream,
                   "gsr_seed_scale");
}

extern "C" gsr_status gsr_nearest(int64_t n, const float* mean, const int32_t* valid, void* workspace,
                                  size_t workspace_bytes, int32_t* nn_index, void* stream)
{
    g_err.clear();
    if (n < 0 || n >= (1ll << 31)) return fail(GSR_EINVAL, "n out of range");
    if (n == 0) return GSR_OK;
    if (!mean || !valid || !nn_index || !workspace) return fail(GSR_EINVAL, "null buffer");
    return knn_run(n, mean, valid, 1.0f, workspace, workspace_bytes, nullptr, nn_index, stream, "gsr_nearest");
}

// ---- map maintenance ------------------------------------------------------

extern "C" gsr_status gsr_adam_step(int64_t n, int32_t colour_rows, const gsr_planes* params,
                                    const gsr_planes* grads, const gsr_planes* m, const gsr_planes* v, float* anchor,
                                    const gsr_adam_config* cfg, void* workspace, double* norm, void* stream)
{
    g_err.clear();
    if (!params || !grads || !m || !v || !cfg || !workspace) return fail(GSR_EINVAL, "null argument");
    if (n < 0 || n > (1ll << 36) || colour_rows < 1 || colour_rows > 48) return fail(GSR_EINVAL, "n or colour_rows");
    if (((uintptr_t)workspace & 7) != 0) return fail(GSR_EINVAL, "workspace not 8-byte aligned");
    if (cfg->step < 1) return fail(GSR_EINVAL, "step must be at least 1");
    if (!(cfg->beta1 >= 0.0 && cfg->beta1 < 1.0) || !(cfg->beta2 >= 0.0 && cfg->beta2 < 1.0) ||
        !(cfg->eps > 0.0f) || !(cfg->ema >= 0.0f && cfg->ema <= 1.0f) || !std::isfinite(cfg->max_grad_norm))
        return fail(GSR_EINVAL, "adam settings");
    for (int k = 0; k < 5; ++k)
        if (!std::isfinite(cfg->lr[k])) return fail(GSR_EINVAL, "learning rate");
    if (n == 0) return GSR_OK;
    const gsr_planes* sets[4] = {params, grads, m, v};
    const int rows[5] = {3, 4, 3, 1, colour_rows};
    AdamArgs a{};
    bool vec = true;
    for (int k = 0; k < 5; ++k) {
        float* ptr[4];
        for (int j = 0; j < 4; ++j) {
            const gsr_planes* q = sets[j];
            ptr[j] = k == 0 ? q->mean : k == 1 ? q->quat : k == 2 ? q->log_scale : k == 3 ? q->opacity_logit : q->colour;
            if (!ptr[j]) return fail(GSR_EINVAL, "null plane");
            if (((uintptr_t)ptr[j] & 15) != 0) vec = false;
        }
        a.p[k] = ptr[0];
        a.g[k] = ptr[1];
        a.m[k] = ptr[2];
        a.v[k] = ptr[3];
        a.len[k] = rows[k] * n;
        if (a.len[k] % 4 != 0) vec = false;
        a.step_size[k] = (float)((double)cfg->lr[k] / (1.0 - std::pow(cfg->beta1, cfg->step)));
    }
    if (anchor && ((uintptr_t)anchor & 15) != 0) vec = false;
    a.inv_sqrt_bc2 = (float)(1.0 / std::sqrt(1.0 - std::pow(cfg->beta2, cfg->step)));
    a.beta1 = (float)cfg->beta1;
    a.beta2 = (float)cfg->beta2;
    a.omb1 = (float)(1.0 - cfg->beta1);
    a.omb2 = (float)(1.0 - cfg->beta2);
    a.eps = cfg->eps;
    a.max_norm = cfg->max_grad_norm;
    a.ema = cfg->ema;
    a.anchor = anchor;
    a.part = (double*)workspace;
    a.norm = norm;
    hipError_t e = launch_adam(a, vec, (hipStream_t)stream);
    return e == hipSuccess ? GSR_OK : hip_fail(e, "gsr_adam_step");
}

extern "C" gsr_status gsr_covis(int64_t pixels, int32_t n_frames, const float* T_key, const float* T_frames,
                                float tau, uint64_t* counts, double* iou, void* stream)
{
    g_err.clear();
    if (!T_key || !T_frames || !counts || !iou) return fail(GSR_EINVAL, "null argument");
    if (pixels < 0 || n_frames < 0 || n_frames > 65535 || !std::isfinite(tau))
        return fail(GSR_EINVAL, "pixels, n_frames or tau");
    if (n_frames == 0) return GSR_OK;
    CovisArgs a{};
    a.pixels = pixels;
    a.frames = n_frames;
    a.tau = tau;
    a.T_key = T_key;
    a.T_frames = T_frames;
    a.counts = (unsigned long long*)counts;
    a.iou = iou;
    hipError_t e = launch_covis(a, (hipStream_t)stream);
    return e == hipSuccess ? GSR_OK : hip_fail(e, "gsr_covis");
}

extern "C" size_t gsr_prune_workspace_bytes(int64_t n)
{
    if (n < 0 || n > (1ll << 31) - 1) return 0;
    return sizeof(uint32_t) * (size_t)((n + GSR_PRUNE_CHUNK - 1) / GSR_PRUNE_CHUNK + 1);
}

// the pruning scan over a given block-count buffer (the caller's workspace
// or the no-allocation scratch); arguments already hold n in range
static gsr_status prune_run(int64_t n, const int32_t* m_obs, const float* v_vis, const float* log_scale,
                            const float* opacity_logit, const gsr_prune_config* cfg, int32_t* keep_index,
                            int64_t* kept, uint32_t* block_count, void* stream, const char* where)
{
    PruneArgs a{};
    a.n = n;
    a.blocks = (int32_t)((n + GSR_PRUNE_CHUNK - 1) / GSR_PRUNE_CHUNK);
    a.m_obs = m_obs;
    a.v_vis = v_vis;
    a.log_scale = log_scale;
    a.opacity_logit = opacity_logit;
    a.m_min = cfg->m_min;
    a.v_min = cfg->v_min;
    a.sigma_max2 = (double)cfg->sigma_max * (double)cfg->sigma_max;
    a.alpha_min = cfg->alpha_min;
    a.block_count = block_count;
    a.keep_index = keep_index;
    a.kept = (long long*)kept;
    hipError_t e = launch_prune(a, (hipStream_t)stream);
    return e == hipSuccess ? GSR_OK : hip_fail(e, where);
}

static gsr_status prune_args_ok(int64_t n, const int32_t* m_obs, const float* v_vis, const float* log_scale,
                                const float* opacity_logit, const gsr_prune_config* cfg, const int32_t* keep_index,
                                const int64_t* kept)
{
    if (!m_obs || !v_vis || !log_scale || !opacity_logit || !cfg || !keep_index || !kept)
        return fail(GSR_EINVAL, "null argument");
    if (n <= 0 || n > (1ll << 31) - 1) return fail(GSR_EINVAL, "n must lie in [1, 2^31)");
    if (!std::isfinite(cfg->v_min) || !std::isfinite(cfg->sigma_max) || !std::isfinite(cfg->alpha_min))
        return fail(GSR_EINVAL, "prune settings");
    return GSR_OK;
}

extern "C" gsr_status gsr_prune(int64_t n, const int32_t* m_obs, const float* v_vis, const float* log_scale,
                                const float* opacity_logit, const gsr_prune_config* cfg, int32_t* keep_index,
                                int64_t* kept, void* workspace, void* stream)
{
    g_err.clear();
    gsr_status st = prune_args_ok(n, m_obs, v_vis, log_scale, opacity_logit, cfg, keep_index, kept);
    if (st != GSR_OK) return st;
    if (!workspace) return fail(GSR_EINVAL, "null argument");
    return prune_run(n, m_obs, v_vis, log_scale, opacity_logit, cfg, keep_index, kept, (uint32_t*)workspace,
                     stream, "gsr_prune");
}

// ---- pruning without allocation --------------------------------------------
// The block counts of the pruning scan live in this file-scope device array
// (one copy per GPU, held until the process ends) instead of a caller
// workspace.  Host code never passes `scratch` itself to a kernel: its name
// on the host is a stand-in, not a device address.  The address on each
// device is taken once, with that device current, by hipGetSymbolAddress,
// and used from then on.  Every call on one GPU shares the array: calls that
// overlap on one GPU (two streams, two threads) race.  The scan writes every
// count it later reads, so nothing needs clearing between calls.
static __device__ __align__(256) uint32_t scratch[(GSR_PRUNE_NOALLOC_MAX_N + GSR_PRUNE_CHUNK - 1) / GSR_PRUNE_CHUNK + 1];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[GSR_MAX_DEVICES];

static gsr_status scratch_address(uint32_t** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "gsr_prune_noalloc: hipGetDevice");
    if (dev < 0 || dev >= GSR_MAX_DEVICES) return fail(GSR_EUNSUPPORTED, "gsr_prune_noalloc: device index too large");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "gsr_prune_noalloc: hipGetSymbolAddress");
        if (!ptr) return fail(GSR_EHIP, "gsr_prune_noalloc: null scratch address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = (uint32_t*)g_scratch_ptr[dev];
    return GSR_OK;
}

extern "C" gsr_status gsr_prune_noalloc(int64_t n, const int32_t* m_obs, const float* v_vis, const float* log_scale,
                                        const float* opacity_logit, const gsr_prune_config* cfg, int32_t* keep_index,
                                        int64_t* kept, void* stream)
{
    g_err.clear();
    gsr_status st = prune_args_ok(n, m_obs, v_vis, log_scale, opacity_logit, cfg, keep_index, kept);
    if (st != GSR_OK) return st;
    if (n > GSR_PRUNE_NOALLOC_MAX_N)
        return fail(GSR_EINVAL, "gsr_prune_noalloc: n exceeds GSR_PRUNE_NOALLOC_MAX_N (2^27 Gaussians), the size "
                                "its fixed device scratch covers; use gsr_prune with a workspace");
    uint32_t* block_count = nullptr;
    st = scratch_address(&block_count);
    if (st != GSR_OK) return st;
    return prune_run(n, m_obs, v_vis, log_scale, opacity_logit, cfg, keep_index, kept, block_count, stream,
                     "gsr_prune_noalloc");
}

extern "C" gsr_status gsr_compact(int64_t n, int32_t rows, const float* src, const int32_t* keep_index,
                                  const int64_t* kept, float* dst, void* stream)
{
    g_err.clear();
    if (!src || !keep_index || !kept || !dst) return fail(GSR_EINVAL, "null argument");
    if (n <= 0 || n > (1ll << 31) - 1 || rows < 1 || rows > 65535) return fail(GSR_EINVAL, "n or rows");
    const size_t span = sizeof(float) * (size_t)rows * (size_t)n;
    if ((uintptr_t)src < (uintptr_t)dst + span && (uintptr_t)dst < (uintptr_t)src + span)
        return fail(GSR_EINVAL, "src and dst overlap");
    CompactArgs a{};
    a.n = n;
    a.rows = rows;
    a.src = src;
    a.keep_index = keep_index;
    a.kept = (const long long*)kept;
    a.dst = dst;
    hipError_t e = launch_compact(a, (hipStream_t)stream);
    return e == hipSuccess ? GSR_OK : hip_fail(e, "gsr_compact");
}

// ---- spatial storage order -------------------------------------------------

// workspace carve-up of gsr_spatial_order: code[2], val[2], hist, box
// partials, digit totals, each on a 256-byte boundary
static size_t order_layout(int64_t n, size_t off[7])
{
    const int64_t blocks = (n + GSR_RADIX_TILE - 1) / GSR_RADIX_TILE;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t o = at;
        at = (at + bytes + 255) & ~(size_t)255;
        return o;
    };
    for (int k = 0; k < 4; ++k) off[k] = take(sizeof(uint32_t) * (size_t)n);
    off[4] = take(sizeof(uint32_t) * 256 * (size_t)blocks);
    off[5] = take(sizeof(uint32_t) * 8 * GSR_BOX_BLOCKS);
    off[6] = take(sizeof(uint32_t) * 256);
    return at;
}

extern "C" size_t gsr_spatial_order_workspace_bytes(int64_t n)
{
    if (n < 1 || n > (1ll << 31) - 1) return 0;
    size_t off[7];
    return order_layout(n, off);
}

// the least P >= max(1, floor(0.618... F + 0.5)) with gcd(P, F) = 1
static int64_t brick_multiplier(int64_t full)
{
    if (full <= 1) return 1;
    int64_t p = (int64_t)std::floor(0.6180339887498949 * (double)full + 0.5);
    if (p < 1) p = 1;
    for (;; ++p) {
        int64_t x = p, y = full;
        while (y) {
            const int64_t t = x % y;
            x = y;
            y = t;
        }
        if (x == 1) return p;
    }
}

extern "C" gsr_status gsr_spatial_order(int64_t n, const float* mean, int32_t brick, int32_t* index, void* workspace,
                                        size_t workspace_bytes, void* stream)
{
    g_err.clear();
    if (!mean || !index || !workspace) return fail(GSR_EINVAL, "null argument");
    if (n < 1 || n > (1ll << 31) - 1) return fail(GSR_EINVAL, "n must lie in [1, 2^31)");
    if (brick < 1) return fail(GSR_EINVAL, "brick must be at least 1");
    if (((uintptr_t)workspace & 255) != 0) return fail(GSR_EINVAL, "workspace not 256-byte aligned");
    size_t off[7];
    const size_t need = order_layout(n, off);
    if (workspace_bytes < need) return fail(GSR_EINVAL, "workspace smaller than gsr_spatial_order_workspace_bytes(n)");
    const uintptr_t ws = (uintptr_t)workspace, ix = (uintptr_t)index, mn = (uintptr_t)mean;
    const size_t ibytes = sizeof(int32_t) * (size_t)n, mbytes = sizeof(float) * 3 * (size_t)n;
    if ((ix < ws + need && ws < ix + ibytes) || (ix < mn + mbytes && mn < ix + ibytes) ||
        (mn < ws + need && ws < mn + mbytes))
        return fail(GSR_EINVAL, "mean, index and workspace must not overlap");
    OrderArgs a{};
    a.n = n;
    a.mean = mean;
    char* base = (char*)workspace;
    for (int k = 0; k < 2; ++k) {
        a.code[k] = (uint32_t*)(base + off[k]);
        a.val[k] = (uint32_t*)(base + off[2 + k]);
    }
    a.hist = (uint32_t*)(base + off[4]);
    a.box = (uint32_t*)(base + off[5]);
    a.tot = (uint32_t*)(base + off[6]);
    a.blocks = (int32_t)((n + GSR_RADIX_TILE - 1) / GSR_RADIX_TILE);
    a.brick = brick;
    a.full = n / brick;
    a.mult = brick_multiplier(a.full);
    a.index = index;
    hipError_t e = launch_spatial_order(a, (hipStream_t)stream);
    return e == hipSuccess ? GSR_OK : hip_fail(e, "gsr_spatial_order");
}

extern "C" gsr_status gsr_device_clock_hz(double* hz)
{
    g_err.clear();
    if (!hz) return fail(GSR_EINVAL, "null argument");
    int dev = 0, khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return hip_fail(e, "gsr_device_clock_hz");
    *hz = 1000.0 * (double)khz;
    return GSR_OK;
}

extern "C" gsr_status gsr_merge(int64_t n, int32_t colour_rows, const gsr_planes* params, const float* v_vis,
                                const int32_t* nn_index, double radius, double colour_tol, gsr_planes* out,
                                int32_t* keep, void* stream)
{
    g_err.clear();
    if (!params || !out || !v_vis || !nn_index || !keep) return fail(GSR_EINVAL, "null argument");
    if (n < 0 || n > (1ll << 31) - 1 || colour_rows < 3 || colour_rows > 48)
        return fail(GSR_EINVAL, "n or colour_rows");
    if (!(radius >= 0.0) || !std::isfinite(radius) || !(colour_tol >= 0.0) || !std::isfinite(colour_tol))
        return fail(GSR_EINVAL, "radius and colour_tol must be finite and non-negative");
    if (n == 0) return GSR_OK;
    MergeArgs a{};
    a.n = n;
    a.colour_rows = colour_rows;
    const gsr_planes* sets[2] = {params, out};
    for (int k = 0; k < 5; ++k) {
        for (int s = 0; s < 2; ++s) {
            const gsr_planes* q = sets[s];
            float* ptr = k == 0 ? q->mean : k == 1 ? q->quat : k == 2 ? q->log_scale : k == 3 ? q->opacity_logit
                                                                                           : q->colour;
            if (!ptr) return fail(GSR_EINVAL, "null plane");
            if (s == 0) a.in[k] = ptr;
            else a.out[k] = ptr;
        }
        if (a.in[k] == a.out[k]) return fail(GSR_EINVAL, "merge output planes must not alias the input");
    }
    a.v_vis = v_vis;
    a.nn = nn_index;
    a.radius = radius;
    a.colour_tol = colour_tol;
    a.keep = keep;
    hipError_t e = launch_merge(a, (hipStream_t)stream);
    return e == hipSuccess ? GSR_OK : hip_fail(e, "gsr_merge");
}

extern "C" gsr_status gsr_keep_list(int64_t n, const int32_t* mask, int32_t* keep_index, int64_t* kept,
                                    void* workspace, void* stream)
{
    g_err.clear();
    if (!mask || !keep_index || !kept || !workspace) return fail(GSR_EINVAL, "null argument");
    if (n <= 0 || n > (1ll << 31) - 1) return fail(GSR_EINVAL, "n must lie in [1, 2^31)");
    PruneArgs a{};
    a.n = n;
    a.blocks = (int32_t)((n + GSR_PRUNE_CHUNK - 1) / GSR_PRUNE_CHUNK);
    a.mask = mask;
    a.block_count = (uint32_t*)workspace;
    a.keep_index = keep_index;
    a.kept = (long long*)kept;
    hipError_t e = launch_prune(a, (hipStream_t)stream);
    return e == hipSuccess ? GSR_OK : hip_fail(e, "gsr_keep_list");
}
