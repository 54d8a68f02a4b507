// api.hip -- the C ABI declared in include/fic.h: host-side validation,
// workspace planning and launches on the caller's stream.
//
// Every entry point validates all of its arguments on the host before it
// touches HIP, so invalid calls return a status and launch nothing; only
// then does a context without a device (device = -1, used to test the
// validation on machines without a GPU) answer FIC_ERR_DEVICE.
#include <new>
#include <string.h>
#include <math.h>
#include <stdint.h>
#include <vector>

#include "fic_internal.h"

using fic::Geom;
using fic::u64;

struct fic_ctx {
    int32_t device;      // -1: host-only context
    int32_t num_cu;
    u64 *counters;
    // stage tracing: (stage, begin event, end event) per recorded stage
    struct Rec { int stage; hipEvent_t a, b; };
    bool timing;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> spare;
    int open_stage;
    hipEvent_t open_ev;
    fic::Tracer tracer;
    // batch graphs, keyed by the batch's descriptors, workspace and counters;
    // most recently used last
    struct Graph { std::vector<unsigned char> key; hipGraphExec_t exec; };
    bool use_graph;
    std::vector<Graph> graphs;
    hipStream_t cap;     // capture stream, created with the first graph
    fic::BatchStreams side;   // batch preparation streams (side.ns == 0 until created)
};

namespace {

hipEvent_t take_event(fic_ctx *c)
{
    if (!c->spare.empty()) {
        hipEvent_t e = c->spare.back();
        c->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void mark_stage(void *self, int stage, int begin, hipStream_t s)
{
    fic_ctx *c = (fic_ctx *)self;
    hipEvent_t e = take_event(c);
    if (!e) return;
    (void)hipEventRecord(e, s);
    if (begin) {
        if (c->open_ev) c->spare.push_back(c->open_ev);
        c->open_ev = e;
        c->open_stage = stage;
    } else if (c->open_ev && c->open_stage == stage) {
        c->recs.push_back({stage, c->open_ev, e});
        c->open_ev = nullptr;
    } else {
        c->spare.push_back(e);
    }
}

const fic::Tracer *tracer_of(fic_ctx *c) { return c->timing ? &c->tracer : nullptr; }

}  // namespace

namespace {

constexpr int kMaxSide = 16384;

bool geom_ok(const fic_geom *g)
{
    if (!g) return false;
    const int b = g->range_size;
    if (b != 4 && b != 8 && b != 16) return false;
    if (g->height <= 0 || g->width <= 0 || g->height > kMaxSide || g->width > kMaxSide) return false;
    if (g->height % b || g->width % b) return false;
    if (g->height < 2 * b || g->width < 2 * b) return false;
    if (g->domain_step < 1) return false;
    if (g->pitch < g->width) return false;
    return true;
}

// Decoding also takes 32x32 ranges: 16x16 codes applied at twice the size.
bool decode_geom_ok(const fic_geom *g)
{
    if (!g) return false;
    if (g->range_size == 32) {
        fic_geom h = *g;
        h.range_size = 16;
        if (h.height % 32 || h.width % 32 || h.height < 64 || h.width < 64) return false;
        return geom_ok(&h);
    }
    return geom_ok(g);
}

Geom to_geom(const fic_geom *g)
{
    Geom r;
    r.h = g->height; r.w = g->width; r.pitch = g->pitch; r.b = g->range_size; r.t = g->domain_step;
    r.n = r.b * r.b;
    r.rcols = r.w / r.b; r.rrows = r.h / r.b;
    r.dcols = (r.w - 2 * r.b) / r.t + 1; r.drows = (r.h - 2 * r.b) / r.t + 1;
    r.R = (int64_t)r.rcols * r.rrows;
    r.D = (int64_t)r.dcols * r.drows;
    return r;
}

// Bits of the largest F = 4096 * Srr' <= 4096 * n^2 * 255^2 / 4, plus the
// domain index and the isometry, must fit the 64-bit key. The 4x4 and 8x8
// searches address their B operand (2n bytes per domain, padded to whole
// blocks) with 32-bit buffer offsets, so it must stay below 2^31 bytes
// (at 8x8 the key already bounds it to 2^30).
bool key_fits(const Geom &g)
{
    const double fmax = 1024.0 * (double)g.n * (double)g.n * 65025.0;
    int fbits = 0;
    while (ldexp(1.0, fbits) <= fmax) ++fbits;
    int dbits = 1;
    while (((int64_t)1 << dbits) < g.D) ++dbits;
    if (g.b != 16 && (double)(g.D + 64) * (double)g.n * 2.0 >= 2147483648.0) return false;
    return fbits + dbits + 3 <= 64;
}

fic_status dev_status(hipError_t e) { return e == hipSuccess ? FIC_OK : FIC_ERR_DEVICE; }

fic_status enter(fic_ctx *ctx)
{
    if (ctx->device < 0) return FIC_ERR_DEVICE;
    return hipSetDevice(ctx->device) == hipSuccess ? FIC_OK : FIC_ERR_DEVICE;
}


constexpr size_t kMaxGraphs = 4;

template <class T> void put(std::vector<unsigned char> &k, const T &v)
{
    const unsigned char *b = (const unsigned char *)&v;
    k.insert(k.end(), b, b + sizeof(T));
}

// Identity of a batch call as far as its recorded graph is concerned: every
// descriptor field, the workspace and the counters (field by field, so no
// padding bytes enter the key).
std::vector<unsigned char> batch_key(int32_t n, const fic_image_desc *d, const void *ws,
                                     size_t ws_bytes, const u64 *counters)
{
    std::vector<unsigned char> k;
    put(k, n);
    for (int32_t i = 0; i < n; ++i) {
        put(k, d[i].img);
        put(k, d[i].geom.height); put(k, d[i].geom.width); put(k, d[i].geom.pitch);
        put(k, d[i].geom.range_size); put(k, d[i].geom.domain_step);
        put(k, d[i].tol);
        put(k, d[i].codes);
    }
    put(k, ws);
    put(k, ws_bytes);
    put(k, counters);
    return k;
}

constexpr int kSideStreams = 4;   // the hardware queues a process gets by default

// The context's batch side streams and events, created on first use
// (default priority). Returns null when they cannot be created.
const fic::BatchStreams *side_streams(fic_ctx *c)
{
    if (c->side.ns > 0) return &c->side;
    fic::BatchStreams b;
    b.ns = 0;
    if (hipEventCreateWithFlags(&b.fork, hipEventDisableTiming) != hipSuccess) return nullptr;
    for (int q = 0; q < kSideStreams; ++q) {
        if (hipStreamCreateWithFlags(&b.side[q], hipStreamNonBlocking) != hipSuccess) break;
        if (hipEventCreateWithFlags(&b.join[q], hipEventDisableTiming) != hipSuccess) {
            (void)hipStreamDestroy(b.side[q]);
            break;
        }
        b.ns = q + 1;
    }
    if (b.ns < kSideStreams) {
        for (int q = 0; q < b.ns; ++q) { (void)hipEventDestroy(b.join[q]); (void)hipStreamDestroy(b.side[q]); }
        (void)hipEventDestroy(b.fork);
        return nullptr;
    }
    c->side = b;
    return &c->side;
}

void drop_side_streams(fic_ctx *c)
{
    if (c->side.ns == 0) return;
    for (int q = 0; q < c->side.ns; ++q) {
        (void)hipEventDestroy(c->side.join[q]);
        (void)hipStreamDestroy(c->side.side[q]);
    }
    (void)hipEventDestroy(c->side.fork);
    c->side.ns = 0;
}

void drop_graphs(fic_ctx *c)
{
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

bool batch_jobs(int32_t n, const fic_image_desc *descs, std::vector<fic::BatchJob> &jobs)
{
    jobs.resize(n);
    for (int32_t i = 0; i < n; ++i) {
        const fic_image_desc &d = descs[i];
        jobs[i].img = d.img;
        jobs[i].g = to_geom(&d.geom);
        jobs[i].tol = d.tol;
        jobs[i].pooled = isfinite(d.tol) || d.tol < 0;
        jobs[i].codes = d.codes;
    }
    return true;
}

}  // namespace

extern "C" {

const char *fic_status_string(fic_status s)
{
    switch (s) {
    case FIC_OK: return "ok";
    case FIC_ERR_INVALID_ARG: return "invalid argument";
    case FIC_ERR_UNSUPPORTED: return "unsupported";
    case FIC_ERR_WORKSPACE: return "workspace too small";
    case FIC_ERR_CAPACITY: return "search key capacity exceeded";
    case FIC_ERR_DEVICE: return "device error";
    default: return "unknown status";
    }
}

fic_status fic_create(int32_t device, fic_ctx **out)
{
    if (!out) return FIC_ERR_INVALID_ARG;
    *out = nullptr;
    if (device < -1) return FIC_ERR_INVALID_ARG;
    fic_ctx *c = new (std::nothrow) fic_ctx;
    if (!c) return FIC_ERR_DEVICE;
    c->device = device;
    c->num_cu = 0;
    c->counters = nullptr;
    c->timing = false;
    c->open_stage = -1;
    c->open_ev = nullptr;
    c->tracer.self = c;
    c->tracer.mark = mark_stage;
    c->use_graph = true;
    c->cap = nullptr;
    c->side.ns = 0;
    if (device >= 0) {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || device >= n) {
            delete c;
            return FIC_ERR_DEVICE;
        }
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
            delete c;
            return FIC_ERR_DEVICE;
        }
        if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            delete c;
            return FIC_ERR_UNSUPPORTED;
        }
        c->num_cu = prop.multiProcessorCount;
        if (hipSetDevice(device) != hipSuccess || fic::init_search_occupancy() != hipSuccess) {
            delete c;
            return FIC_ERR_DEVICE;
        }
    }
    *out = c;
    return FIC_OK;
}

fic_status fic_destroy(fic_ctx *ctx)
{
    if (!ctx) return FIC_ERR_INVALID_ARG;
    if (ctx->device >= 0) {
        for (auto &r : ctx->recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        for (auto e : ctx->spare) (void)hipEventDestroy(e);
        if (ctx->open_ev) (void)hipEventDestroy(ctx->open_ev);
        drop_graphs(ctx);
        drop_side_streams(ctx);
        if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    }
    delete ctx;
    return FIC_OK;
}

fic_status fic_timing_enable(fic_ctx *ctx, int32_t enable)
{
    if (!ctx) return FIC_ERR_INVALID_ARG;
    for (auto &r : ctx->recs) { ctx->spare.push_back(r.a); ctx->spare.push_back(r.b); }
    ctx->recs.clear();
    if (ctx->open_ev) { ctx->spare.push_back(ctx->open_ev); ctx->open_ev = nullptr; }
    ctx->timing = enable != 0;
    return FIC_OK;
}

fic_status fic_timing_read(fic_ctx *ctx, int32_t *stages, float *ms, int32_t capacity,
                           int32_t *count)
{
    if (!ctx || !count || capacity < 0 || (capacity > 0 && (!stages || !ms)))
        return FIC_ERR_INVALID_ARG;
    *count = (int32_t)ctx->recs.size();
    if (ctx->recs.empty()) return FIC_OK;
    fic_status st = enter(ctx);
    if (st != FIC_OK) return st;
    for (int32_t i = 0; i < (int32_t)ctx->recs.size() && i < capacity; ++i) {
        const auto &r = ctx->recs[i];
        float t = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
            return FIC_ERR_DEVICE;
        stages[i] = r.stage;
        ms[i] = t;
    }
    return FIC_OK;
}

fic_status fic_set_counters(fic_ctx *ctx, uint64_t *counters)
{
    if (!ctx) return FIC_ERR_INVALID_ARG;
    ctx->counters = (u64 *)counters;
    return FIC_OK;
}

int64_t fic_num_ranges(const fic_geom *g) { return geom_ok(g) ? to_geom(g).R : 0; }
int64_t fic_num_domains(const fic_geom *g) { return geom_ok(g) ? to_geom(g).D : 0; }

fic_status fic_fd_classify(fic_ctx *ctx, const uint8_t *img, const fic_geom *g, int32_t block,
                           int32_t step, double *fd64, float *fd32, void *stream)
{
    if (!ctx || !img || !g || !fd64) return FIC_ERR_INVALID_ARG;
    if (block != 4 && block != 8 && block != 16 && block != 32) return FIC_ERR_INVALID_ARG;
    if (step < 1 || g->height < block || g->width < block || g->pitch < g->width ||
        g->height > kMaxSide || g->width > kMaxSide)
        return FIC_ERR_INVALID_ARG;
    fic_status st = enter(ctx);
    if (st != FIC_OK) return st;
    return dev_status(fic::launch_fd_classify(img, g->height, g->width, g->pitch, block, step, fd64,
                                              fd32, (hipStream_t)stream, tracer_of(ctx)));
}

size_t fic_pool_workspace_bytes(int64_t n_range, int64_t n_domain)
{
    if (n_range < 0 || n_domain < 0) return 0;
    return fic::pool_ws_bytes(n_range, n_domain);
}

fic_status fic_build_domain_pool(fic_ctx *ctx, const double *fd_range, int32_t n_range,
                                 const double *fd_domain, int32_t n_domain, double tol,
                                 uint32_t *perm, uint32_t *lo, uint32_t *hi, void *ws,
                                 size_t ws_bytes, void *stream)
{
    if (!ctx || !fd_range || !fd_domain || !perm || !lo || !hi || !ws) return FIC_ERR_INVALID_ARG;
    if (n_range < 1 || n_domain < 1 || isnan(tol)) return FIC_ERR_INVALID_ARG;
    if (ws_bytes < fic::pool_ws_bytes(n_range, n_domain)) return FIC_ERR_WORKSPACE;
    fic_status st = enter(ctx);
    if (st != FIC_OK) return st;
    return dev_status(fic::launch_pool(fd_range, n_range, fd_domain, n_domain, tol, perm, lo, hi, ws,
                                       (hipStream_t)stream, tracer_of(ctx)));
}

size_t fic_encode_workspace_bytes(const fic_geom *g, int32_t pooled)
{
    if (!geom_ok(g)) return 0;
    fic::EncodePlan p;
    fic::plan_encode(to_geom(g), pooled ? 1 : 0, p);
    return p.total;
}

fic_status fic_encode_pifs(fic_ctx *ctx, const uint8_t *img, const fic_geom *g,
                           const uint32_t *perm, const uint32_t *lo, const uint32_t *hi,
                           int32_t kernel, fic_code *codes, void *ws, size_t ws_bytes,
                           void *stream)
{
    if (!ctx || !img || !codes || !ws || !geom_ok(g)) return FIC_ERR_INVALID_ARG;
    const int nset = (perm != nullptr) + (lo != nullptr) + (hi != nullptr);
    if (nset != 0 && nset != 3) return FIC_ERR_INVALID_ARG;
    if (kernel != FIC_KERNEL_MFMA && kernel != FIC_KERNEL_PLAIN) return FIC_ERR_INVALID_ARG;
    const Geom gg = to_geom(g);
    if (!key_fits(gg)) return FIC_ERR_CAPACITY;
    fic::EncodePlan p;
    fic::plan_encode(gg, nset == 3, p);
    if (ws_bytes < p.total) return FIC_ERR_WORKSPACE;
    fic_status st = enter(ctx);
    if (st != FIC_OK) return st;
    return dev_status(fic::run_encode(p, img, perm, lo, hi, kernel, codes, ws, ctx->num_cu,
                                      ctx->counters, (hipStream_t)stream, tracer_of(ctx)));
}

size_t fic_batch_workspace_bytes(int32_t n_images, const fic_image_desc *descs)
{
    if (n_images < 1 || !descs) return 0;
    for (int32_t i = 0; i < n_images; ++i)
        if (!geom_ok(&descs[i].geom)) return 0;
    std::vector<fic::BatchJob> jobs;
    batch_jobs(n_images, descs, jobs);
    fic::BatchPlan bp;
    fic::plan_batch(jobs.data(), n_images, bp);
    return bp.total;
}

fic_status fic_set_batch_graph(fic_ctx *ctx, int32_t enable)
{
    if (!ctx) return FIC_ERR_INVALID_ARG;
    ctx->use_graph = enable != 0;
    if (!ctx->use_graph && ctx->device >= 0 && enter(ctx) == FIC_OK) drop_graphs(ctx);
    return FIC_OK;
}

fic_status fic_encode_pifs_batch(fic_ctx *ctx, int32_t n_images, const fic_image_desc *descs,
                                 void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx || n_images < 1 || !descs || !ws) return FIC_ERR_INVALID_ARG;
    for (int i = 0; i < n_images; ++i) {
        const fic_image_desc &d = descs[i];
        if (!d.img || !d.codes || !geom_ok(&d.geom) || isnan(d.tol)) return FIC_ERR_INVALID_ARG;
        if (!key_fits(to_geom(&d.geom))) return FIC_ERR_CAPACITY;
    }
    std::vector<fic::BatchJob> jobs;
    batch_jobs(n_images, descs, jobs);
    fic::BatchPlan bp;
    fic::plan_batch(jobs.data(), n_images, bp);
    if (bp.items > (int64_t)0xffffffffll) return FIC_ERR_CAPACITY;   // one 32-bit item queue
    if (ws_bytes < bp.total) return FIC_ERR_WORKSPACE;
    fic_status st = enter(ctx);
    if (st != FIC_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const fic::BatchStreams *side = side_streams(ctx);
    if (!side) return FIC_ERR_DEVICE;
    if (!ctx->use_graph)
        return dev_status(fic::run_encode_batch(jobs.data(), bp, ws, ctx->num_cu, ctx->counters, s,
                                                tracer_of(ctx), side));
    std::vector<unsigned char> key = batch_key(n_images, descs, ws, ws_bytes, ctx->counters);
    size_t hit = ctx->graphs.size();
    for (size_t i = 0; i < ctx->graphs.size(); ++i)
        if (ctx->graphs[i].key == key) { hit = i; break; }
    if (hit == ctx->graphs.size()) {
        // record the whole batch once, on a capture stream of our own
        if (!ctx->cap && hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking) != hipSuccess) {
            ctx->cap = nullptr;
            return FIC_ERR_DEVICE;
        }
        if (hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return FIC_ERR_DEVICE;
        const hipError_t e = fic::run_encode_batch(jobs.data(), bp, ws, ctx->num_cu, ctx->counters,
                                                   ctx->cap, nullptr, side);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(ctx->cap, &graph);
        hipGraphExec_t exec = nullptr;
        hipError_t e3 = hipErrorUnknown;
        if (e == hipSuccess && e2 == hipSuccess && graph)
            e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e3 != hipSuccess) return FIC_ERR_DEVICE;
        if (ctx->graphs.size() >= kMaxGraphs) {
            (void)hipGraphExecDestroy(ctx->graphs.front().exec);
            ctx->graphs.erase(ctx->graphs.begin());
        }
        ctx->graphs.push_back({std::move(key), exec});
    } else if (hit + 1 != ctx->graphs.size()) {
        fic_ctx::Graph g = std::move(ctx->graphs[hit]);
        ctx->graphs.erase(ctx->graphs.begin() + hit);
        ctx->graphs.push_back(std::move(g));
    }
    const fic::Tracer *tr = tracer_of(ctx);
    fic::trace(tr, FIC_STAGE_BATCH, 1, s);
    const hipError_t e = hipGraphLaunch(ctx->graphs.back().exec, s);
    fic::trace(tr, FIC_STAGE_BATCH, 0, s);
    return dev_status(e);
}

// ---------------------------------------------------------------- quadtree
namespace {
bool quad_geoms_ok(const fic_geom *g1, const fic_geom *g2)
{
    if (!geom_ok(g1) || !geom_ok(g2)) return false;
    if (g1->range_size != 2 * g2->range_size) return false;
    return g1->height == g2->height && g1->width == g2->width && g1->pitch == g2->pitch;
}
bool pooled_of(double tol) { return isfinite(tol) || tol < 0; }
}  // namespace

size_t fic_quadtree_workspace_bytes(const fic_geom *g1, double tol1, const fic_geom *g2,
                                    double tol2)
{
    if (!quad_geoms_ok(g1, g2) || isnan(tol1) || isnan(tol2)) return 0;
    fic::QuadPlan qp;
    fic::plan_quadtree(to_geom(g1), tol1, to_geom(g2), tol2, qp);
    return qp.total;
}

fic_status fic_encode_quadtree(fic_ctx *ctx, const uint8_t *img, const fic_geom *g1, double tol1,
                               const fic_geom *g2, double tol2, double rms_split,
                               fic_code *codes1, fic_code *codes2, void *ws, size_t ws_bytes,
                               void *stream)
{
    if (!ctx || !img || !codes1 || !codes2 || !ws) return FIC_ERR_INVALID_ARG;
    if (!quad_geoms_ok(g1, g2) || isnan(tol1) || isnan(tol2)) return FIC_ERR_INVALID_ARG;
    if (isnan(rms_split) || rms_split < 0) return FIC_ERR_INVALID_ARG;
    const Geom gg1 = to_geom(g1), gg2 = to_geom(g2);
    if (!key_fits(gg1) || !key_fits(gg2)) return FIC_ERR_CAPACITY;
    fic::QuadPlan qp;
    fic::plan_quadtree(gg1, tol1, gg2, tol2, qp);
    if (ws_bytes < qp.total) return FIC_ERR_WORKSPACE;
    // E is split when E > 4096 * n^2 * rms^2 (fp64, in this operation order),
    // i.e. when it exceeds that bound floored to an integer.
    const double n1 = (double)gg1.n;
    const double t = rms_split * rms_split * (4096.0 * n1 * n1);
    const int64_t emax = t < 9.0e18 ? (int64_t)floor(t) : INT64_MAX;
    fic_status st = enter(ctx);
    if (st != FIC_OK) return st;
    return dev_status(fic::run_quadtree(qp, img, emax, codes1, codes2, ws, ctx->num_cu,
                                        ctx->counters, (hipStream_t)stream, tracer_of(ctx)));
}

fic_status fic_decode_quadtree(fic_ctx *ctx, const fic_code *codes1, const fic_geom *g1,
                               const fic_code *codes2, const fic_geom *g2, int32_t max_iters,
                               const uint8_t *init, uint8_t *out, void *scratch,
                               size_t scratch_bytes, int32_t *iters_done, void *stream)
{
    if (!ctx || !codes1 || !codes2 || !out || !scratch || !iters_done) return FIC_ERR_INVALID_ARG;
    if (!quad_geoms_ok(g1, g2)) return FIC_ERR_INVALID_ARG;
    if (max_iters < 0 || max_iters > fic::decode_max_iters()) return FIC_ERR_INVALID_ARG;
    const Geom gg1 = to_geom(g1), gg2 = to_geom(g2);
    if (scratch_bytes < fic::decode_ws_bytes(gg1)) return FIC_ERR_WORKSPACE;
    fic_status st = enter(ctx);
    if (st != FIC_OK) return st;
    return dev_status(fic::run_decode_quadtree(gg1, codes1, gg2, codes2, max_iters, init, out,
                                               scratch, iters_done, (hipStream_t)stream,
                                               tracer_of(ctx)));
}

// ---------------------------------------------------------------- colour
namespace {
// An RGB geometry: pitch in bytes >= 3 * width; the rest as for gray.
bool color_geom_ok(const fic_geom *g)
{
    if (!g || g->pitch < 3 * (int64_t)g->width) return false;
    fic_geom p = *g;
    p.pitch = g->width;
    return geom_ok(&p);
}
}  // namespace

size_t fic_color_workspace_bytes(const fic_geom *g, double tol)
{
    if (!color_geom_ok(g) || isnan(tol)) return 0;
    fic::ColorPlan cp;
    fic::plan_color(to_geom(g), tol, cp);
    return cp.total;
}

fic_status fic_encode_color(fic_ctx *ctx, const uint8_t *rgb, const fic_geom *g, double tol,
                            int32_t fd_source, fic_code *codes_r, fic_code *codes_g,
                            fic_code *codes_b, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx || !rgb || !codes_r || !codes_g || !codes_b || !ws) return FIC_ERR_INVALID_ARG;
    if (!color_geom_ok(g) || isnan(tol) || (fd_source != 0 && fd_source != 1))
        return FIC_ERR_INVALID_ARG;
    const Geom gg = to_geom(g);
    if (!key_fits(gg)) return FIC_ERR_CAPACITY;
    fic::ColorPlan cp;
    fic::plan_color(gg, tol, cp);
    if (ws_bytes < cp.total) return FIC_ERR_WORKSPACE;
    fic_status st = enter(ctx);
    if (st != FIC_OK) return st;
    fic_code *const codes[3] = {codes_r, codes_g, codes_b};
    return dev_status(fic::run_color(cp, rgb, g->pitch, fd_source, codes, ws, ctx->num_cu,
                                     ctx->counters, (hipStream_t)stream, tracer_of(ctx)));
}

int64_t fic_packed_words(const fic_geom *g)
{
    return geom_ok(g) ? fic::packed_words(to_geom(g)) : 0;
}

fic_status fic_pack_codes(fic_ctx *ctx, const fic_code *codes, const fic_geom *g, uint32_t *words,
                          int64_t nwords, void *stream)
{
    if (!ctx || !codes || !words || !geom_ok(g)) return FIC_ERR_INVALID_ARG;
    const Geom gg = to_geom(g);
    if (nwords < fic::packed_words(gg)) return FIC_ERR_WORKSPACE;
    fic_status st = enter(ctx);
    if (st != FIC_OK) return st;
    return dev_status(fic::run_pack(gg, codes, words, (hipStream_t)stream));
}

fic_status fic_unpack_codes(fic_ctx *ctx, const uint32_t *words, int64_t nwords, const fic_geom *g,
                            fic_code *codes, void *stream)
{
    if (!ctx || !codes || !words || !geom_ok(g)) return FIC_ERR_INVALID_ARG;
    const Geom gg = to_geom(g);
    if (nwords < fic::packed_words(gg)) return FIC_ERR_INVALID_ARG;
    fic_status st = enter(ctx);
    if (st != FIC_OK) return st;
    return dev_status(fic::run_unpack(gg, words, codes, (hipStream_t)stream));
}

size_t fic_decode_workspace_bytes(const fic_geom *g)
{
    if (!decode_geom_ok(g)) return 0;
    return fic::decode_ws_bytes(to_geom(g));
}

fic_status fic_decode_pifs(fic_ctx *ctx, const fic_code *codes, const fic_geom *g,
                           int32_t max_iters, const uint8_t *init, uint8_t *out, void *scratch,
                           size_t scratch_bytes, int32_t *iters_done, void *stream)
{
    if (!ctx || !codes || !out || !scratch || !iters_done || !decode_geom_ok(g))
        return FIC_ERR_INVALID_ARG;
    if (max_iters < 0 || max_iters > fic::decode_max_iters()) return FIC_ERR_INVALID_ARG;
    const Geom gg = to_geom(g);
    if (scratch_bytes < fic::decode_ws_bytes(gg)) return FIC_ERR_WORKSPACE;
    fic_status st = enter(ctx);
    if (st != FIC_OK) return st;
    return dev_status(
        fic::run_decode(gg, codes, max_iters, init, out, scratch, iters_done, (hipStream_t)stream,
                        tracer_of(ctx)));
}

}  // extern "C"
