// api.hip -- the C ABI declared in include/fic.h: host-side validation,
// workspace planning and launches on the caller's stream.
//
// Every entry point validates all of its arguments on the host before it
// touches HIP, so invalid calls return a status and launch nothing; only
// then does a context without a device (device = -1, used to test the
// validation on machines without a GPU) answer FIC_ERR_DEVICE.
#include <new>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "fic_internal.h"

using fic::Geom;
using fic::u64;

// Device scratch of fic_encode_pifs_noalloc: one copy on every GPU the
// library runs on, held until the process ends. In host code this name is a
// host-side stand-in, not a device address: fic_create looks the device
// address up with hipGetSymbolAddress (with the context's device current)
// and only that address is ever passed to kernels.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

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
    uint32_t dbg;        // fic_set_debug switches
    bool batch_separate; // tuned: one search launch per range size in batches
    void *scratch_dev;   // device address of `scratch` on this device (null: host-only)
    char arch[64];       // gcnArchName of the device (tuning cache key)
    // tuned search parameters per (range size, floor(log2 D)); classes
    // without a row use fic::default_tune_row
    struct TuneEntry { int32_t b, dlog; fic::TuneRow row; };
    std::vector<TuneEntry> tune;
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

int dlog2_of(int64_t D)
{
    int l = 0;
    while (((int64_t)2 << l) <= D) ++l;
    return l;                        // floor(log2 D), D >= 1
}

fic::TuneRow tune_row(const fic_ctx *c, int b, int64_t D)
{
    const int dl = dlog2_of(D);
    for (const auto &t : c->tune)
        if (t.b == b && t.dlog == dl) return t.row;
    return fic::default_tune_row(b);
}

void set_tune_row(fic_ctx *c, int b, int dlog, const fic::TuneRow &row)
{
    for (auto &t : c->tune)
        if (t.b == b && t.dlog == dlog) { t.row = row; return; }
    c->tune.push_back({b, dlog, row});
}

// The context's parameters and switches on a plan (before it runs).
void apply_ctx(const fic_ctx *c, fic::EncodePlan &p)
{
    p.tune = tune_row(c, p.g.b, p.g.D);
    p.dbg = c->dbg;
}

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
    if (fbits + dbits + 3 > 64) return false;
    // the work list (every group x every chunk of the narrowest item width)
    // is counted in 32 bits
    fic::EncodePlan p;
    fic::plan_encode(g, 1, p);
    return p.max_items <= (int64_t)0xffffffffll;
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
                                     size_t ws_bytes, const u64 *counters, uint32_t dbg)
{
    std::vector<unsigned char> k;
    put(k, n);
    put(k, dbg);
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
    c->dbg = 0;
    c->batch_separate = false;
    c->scratch_dev = nullptr;
    snprintf(c->arch, sizeof c->arch, "%s", "none");
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
        snprintf(c->arch, sizeof c->arch, "%s", prop.gcnArchName);
        c->num_cu = prop.multiProcessorCount;
        if (hipSetDevice(device) != hipSuccess || fic::init_search_occupancy() != hipSuccess) {
            delete c;
            return FIC_ERR_DEVICE;
        }
        // this device's copy of the no-allocation scratch
        void *sp = nullptr;
        if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) {
            delete c;
            return FIC_ERR_DEVICE;
        }
        c->scratch_dev = sp;
        // tuned parameters from the cache file named by FIC_TUNE_CACHE, when
        // it was written for this architecture and these kernels
        const char *cache = getenv("FIC_TUNE_CACHE");
        if (cache && *cache) (void)fic_tune_load(c, cache);
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
    apply_ctx(ctx, p);
    fic_status st = enter(ctx);
    if (st != FIC_OK) return st;
    return dev_status(fic::run_encode(p, img, perm, lo, hi, kernel, codes, ws, ctx->num_cu,
                                      ctx->counters, (hipStream_t)stream, tracer_of(ctx)));
}

size_t fic_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

fic_status fic_encode_pifs_noalloc(fic_ctx *ctx, const uint8_t *img, const fic_geom *g,
                                   const uint32_t *perm, const uint32_t *lo, const uint32_t *hi,
                                   int32_t kernel, fic_code *codes, void *stream)
{
    if (!ctx || !img || !codes || !geom_ok(g)) return FIC_ERR_INVALID_ARG;
    const int nset = (perm != nullptr) + (lo != nullptr) + (hi != nullptr);
    if (nset != 0 && nset != 3) return FIC_ERR_INVALID_ARG;
    if (kernel != FIC_KERNEL_MFMA && kernel != FIC_KERNEL_PLAIN) return FIC_ERR_INVALID_ARG;
    const Geom gg = to_geom(g);
    if (!key_fits(gg)) return FIC_ERR_CAPACITY;
    fic::EncodePlan p;
    fic::plan_encode(gg, nset == 3, p);
    if (p.total > kNoAllocScratchBytes) return FIC_ERR_WORKSPACE;
    apply_ctx(ctx, p);
    fic_status st = enter(ctx);
    if (st != FIC_OK) return st;
    if (!ctx->scratch_dev) return FIC_ERR_DEVICE;
    // the same kernels as fic_encode_pifs, on the static scratch; no stage
    // events (creating them could allocate)
    return dev_status(fic::run_encode(p, img, perm, lo, hi, kernel, codes, ctx->scratch_dev,
                                      ctx->num_cu, ctx->counters, (hipStream_t)stream, nullptr));
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
    for (auto &pt : bp.part) apply_ctx(ctx, pt.plan);
    bp.dbg = ctx->dbg | (ctx->batch_separate ? fic::kDbgSeparate : 0u);
    fic_status st = enter(ctx);
    if (st != FIC_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const fic::BatchStreams *side = side_streams(ctx);
    if (!side) return FIC_ERR_DEVICE;
    if (!ctx->use_graph)
        return dev_status(fic::run_encode_batch(jobs.data(), bp, ws, ctx->num_cu, ctx->counters, s,
                                                tracer_of(ctx), side));
    std::vector<unsigned char> key = batch_key(n_images, descs, ws, ws_bytes, ctx->counters, bp.dbg);
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
    apply_ctx(ctx, qp.part[0].plan);
    apply_ctx(ctx, qp.part[1].plan);
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
    apply_ctx(ctx, cp.part.plan);
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

// ---------------------------------------------------------------- debug switches
fic_status fic_set_debug(fic_ctx *ctx, uint32_t flags)
{
    if (!ctx ||
        (flags & ~(uint32_t)(FIC_DEBUG_REVERSE_ITEMS | FIC_DEBUG_VERIFY16 | FIC_DEBUG_SEPARATE_SEARCHES)))
        return FIC_ERR_INVALID_ARG;
    ctx->dbg = flags;
    return FIC_OK;
}

// ---------------------------------------------------------------- autotuner
#ifndef FIC_KERNEL_HASH
#define FIC_KERNEL_HASH "unknown"
#endif

const char *fic_kernel_hash(void) { return FIC_KERNEL_HASH; }

fic_status fic_tune_reset(fic_ctx *ctx)
{
    if (!ctx) return FIC_ERR_INVALID_ARG;
    ctx->tune.clear();
    ctx->batch_separate = false;
    if (ctx->device >= 0 && enter(ctx) == FIC_OK) drop_graphs(ctx);
    return FIC_OK;
}

fic_status fic_tune_query(fic_ctx *ctx, const fic_geom *g, int32_t pooled, double pool_fraction,
                          int32_t *chunk_log2, int32_t *flush_at, int32_t *xcd)
{
    if (!ctx || !g || !chunk_log2 || !flush_at || !geom_ok(g)) return FIC_ERR_INVALID_ARG;
    if (pooled && !(pool_fraction >= 0.0 && pool_fraction <= 1.0)) return FIC_ERR_INVALID_ARG;
    const Geom gg = to_geom(g);
    const fic::TuneRow row = tune_row(ctx, gg.b, gg.D);
    const int k = pooled ? fic::tune_bucket_of_fraction(pool_fraction) : 0;
    *chunk_log2 = row.chunk_log2[k];
    *flush_at = row.flush_at[k];
    if (xcd) *xcd = row.xcd[k];
    return FIC_OK;
}

size_t fic_autotune_workspace_bytes(int32_t n_images, const fic_image_desc *descs)
{
    if (n_images < 1 || !descs) return 0;
    size_t m = 0;
    for (int32_t i = 0; i < n_images; ++i) {
        const size_t b = fic_batch_workspace_bytes(1, descs + i);
        if (b == 0) return 0;
        m = b > m ? b : m;
    }
    return m;
}

namespace {
struct TuneImage {
    fic::BatchJob job;
    fic::BatchPlan bp;
    int b, dlog, bucket;
};

// Events around the search launch only: the tuned parameters change the
// work list and the search, and the rest of an encode (classification,
// pool, preparation, finalization) would only add its own noise.
struct SearchTimer {
    hipEvent_t b, e;
    hipError_t err;
    static void mark(void *self, int stage, int begin, hipStream_t s)
    {
        SearchTimer *t = (SearchTimer *)self;
        if (stage == FIC_STAGE_SEARCH && t->err == hipSuccess)
            t->err = hipEventRecord(begin ? t->b : t->e, s);
    }
};

// One whole encode of image `im` (classify, pool, prep, search, finalize)
// with row `row`; ms = the search launch's time, from events on s. Blocks
// the host.
hipError_t timed_encode(fic_ctx *c, TuneImage &im, const fic::TuneRow &row, void *ws, hipStream_t s,
                        hipEvent_t e0, hipEvent_t e1, float &ms)
{
    im.bp.part[0].plan.tune = row;
    im.bp.part[0].plan.dbg = 0;
    im.bp.dbg = 0;
    SearchTimer st{e0, e1, hipSuccess};
    const fic::Tracer tr{&st, &SearchTimer::mark};
    hipError_t e = fic::run_encode_batch(&im.job, im.bp, ws, c->num_cu, nullptr, s, &tr, nullptr);
    if (e == hipSuccess) e = st.err;
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    return e;
}
}  // namespace

fic_status fic_autotune(fic_ctx *ctx, int32_t n_images, const fic_image_desc *descs, void *ws,
                        size_t ws_bytes, int32_t reps, fic_tune_entry *report, int32_t report_cap,
                        int32_t *report_count, void *stream)
{
    if (!ctx || n_images < 1 || !descs || !ws || reps < 1 || reps > 16 || report_cap < 0 ||
        (report_cap > 0 && !report))
        return FIC_ERR_INVALID_ARG;
    for (int32_t i = 0; i < n_images; ++i) {
        const fic_image_desc &d = descs[i];
        if (!d.img || !d.codes || !geom_ok(&d.geom) || isnan(d.tol)) return FIC_ERR_INVALID_ARG;
        if (!key_fits(to_geom(&d.geom))) return FIC_ERR_CAPACITY;
    }
    if (ws_bytes < fic_autotune_workspace_bytes(n_images, descs)) return FIC_ERR_WORKSPACE;
    if (report_count) *report_count = 0;
    fic_status st = enter(ctx);
    if (st != FIC_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    std::vector<TuneImage> ims(n_images);
    for (int32_t i = 0; i < n_images; ++i) {
        std::vector<fic::BatchJob> one;
        batch_jobs(1, descs + i, one);
        ims[i].job = one[0];
        fic::plan_batch(&ims[i].job, 1, ims[i].bp);
        ims[i].b = ims[i].job.g.b;
        ims[i].dlog = dlog2_of(ims[i].job.g.D);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return FIC_ERR_DEVICE;
    }
    hipError_t e = hipSuccess;
    // the bucket of every image: one (warm-up) encode, then its pool sum
    for (auto &im : ims) {
        float ms = 0.0f;
        e = timed_encode(ctx, im, tune_row(ctx, im.b, im.job.g.D), ws, s, e0, e1, ms);
        if (e != hipSuccess) break;
        const fic::EncodePlan &pl = im.bp.part[0].plan;
        uint64_t psum = 0;
        e = hipMemcpy(&psum, (const char *)ws + im.bp.part[0].off_enc + pl.off_ctr + 32, 8,
                      hipMemcpyDeviceToHost);
        if (e != hipSuccess) break;
        im.bucket = fic::tune_bucket(im.job.pooled, psum, im.job.g.R, im.job.g.D);
    }
    // one tuning class at a time: (range size, log2 D, bucket); a candidate's
    // cost is the sum over the class's images of the best of `reps` encodes
    std::vector<char> done(n_images, 0);
    int32_t nrep = 0;
    for (int32_t i = 0; i < n_images && e == hipSuccess; ++i) {
        if (done[i]) continue;
        std::vector<int32_t> cls;
        for (int32_t j = i; j < n_images; ++j)
            if (!done[j] && ims[j].b == ims[i].b && ims[j].dlog == ims[i].dlog &&
                ims[j].bucket == ims[i].bucket) {
                cls.push_back(j);
                done[j] = 1;
            }
        const int k = ims[i].bucket;
        const fic::TuneRow base = tune_row(ctx, ims[i].b, ims[i].job.g.D);
        auto cost = [&](const fic::TuneRow &row, float &total) {
            total = 0.0f;
            for (int32_t j : cls) {
                float best = 1e30f;
                for (int r = 0; r < reps && e == hipSuccess; ++r) {
                    float ms = 0.0f;
                    e = timed_encode(ctx, ims[j], row, ws, s, e0, e1, ms);
                    best = ms < best ? ms : best;
                }
                total += best;
            }
        };
        float t_base = 0.0f;
        cost(base, t_base);
        fic::TuneRow best = base;
        float t_best = t_base;
        // coordinate descent: the item width, then the flush trigger
        for (int cl = fic::kChunkLog2Min; cl <= fic::kChunkLog2Max && e == hipSuccess; ++cl) {
            if (cl == best.chunk_log2[k]) continue;
            fic::TuneRow cand = best;
            cand.chunk_log2[k] = (int8_t)cl;
            float t = 0.0f;
            cost(cand, t);
            if (t < t_best) { t_best = t; best = cand; }
        }
        static const int kFlush[] = {0, 16, 32, 64, 128};
        for (int fi = 0; fi < 5 && e == hipSuccess; ++fi) {
            if (kFlush[fi] == best.flush_at[k]) continue;
            fic::TuneRow cand = best;
            cand.flush_at[k] = (int16_t)kFlush[fi];
            float t = 0.0f;
            cost(cand, t);
            if (t < t_best) { t_best = t; best = cand; }
        }
        if (e == hipSuccess) {          // one queue per XCD, or one queue
            fic::TuneRow cand = best;
            cand.xcd[k] = best.xcd[k] ? 0 : 1;
            float t = 0.0f;
            cost(cand, t);
            if (t < t_best) { t_best = t; best = cand; }
        }
        if (e != hipSuccess) break;
        // measure the starting row and the winner again, interleaved, and keep
        // the winner only if it is still faster
        float tb = 0.0f, tw = 0.0f, sb = 1e30f, sw = 1e30f;
        for (int r = 0; r < 2 && e == hipSuccess; ++r) {
            cost(base, tb);
            cost(best, tw);
            sb = tb < sb ? tb : sb;
            sw = tw < sw ? tw : sw;
        }
        if (e != hipSuccess) break;
        if (!(sw < sb)) { best = base; sw = sb; }
        set_tune_row(ctx, ims[i].b, ims[i].dlog, best);
        if (nrep < report_cap) {
            fic_tune_entry &r = report[nrep];
            r.range_size = ims[i].b;
            r.dlog2 = ims[i].dlog;
            r.bucket = k;
            r.images = (int32_t)cls.size();
            r.chunk_log2 = best.chunk_log2[k];
            r.flush_at = best.flush_at[k];
            r.xcd = best.xcd[k];
            r.base_chunk_log2 = base.chunk_log2[k];
            r.base_flush_at = base.flush_at[k];
            r.base_xcd = base.xcd[k];
            r.base_ms = sb;
            r.tuned_ms = sw;
        }
        ++nrep;
    }
    // the launch structure of a batch with both 4x4 and 8x8 images: one
    // combined persistent search, or one per range size (best of 3 whole
    // batches each, interleaved, with the tuned rows)
    bool has4 = false, has8 = false;
    for (const auto &im : ims) { has4 = has4 || im.b == 4; has8 = has8 || im.b == 8; }
    if (e == hipSuccess && has4 && has8 && ws_bytes >= fic_batch_workspace_bytes(n_images, descs)) {
        std::vector<fic::BatchJob> jobs;
        batch_jobs(n_images, descs, jobs);
        fic::BatchPlan bp;
        fic::plan_batch(jobs.data(), n_images, bp);
        for (auto &pt : bp.part) apply_ctx(ctx, pt.plan);
        const fic::BatchStreams *side = side_streams(ctx);
        float best[2] = {1e30f, 1e30f};
        for (int r = 0; r < 3 && e == hipSuccess && side; ++r)
            for (int sep = 0; sep < 2 && e == hipSuccess; ++sep) {
                bp.dbg = sep ? fic::kDbgSeparate : 0u;
                float ms = 0.0f;
                e = hipEventRecord(e0, s);
                if (e == hipSuccess)
                    e = fic::run_encode_batch(jobs.data(), bp, ws, ctx->num_cu, nullptr, s, nullptr, side);
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                best[sep] = ms < best[sep] ? ms : best[sep];
            }
        if (e == hipSuccess && side) {
            ctx->batch_separate = best[1] < best[0];
            if (nrep < report_cap) {
                fic_tune_entry &r = report[nrep];
                memset(&r, 0, sizeof r);
                r.range_size = 0;             // the batch's launch structure
                r.images = n_images;
                r.flush_at = ctx->batch_separate ? 1 : 0;
                r.base_ms = best[0];
                r.tuned_ms = ctx->batch_separate ? best[1] : best[0];
            }
            ++nrep;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    drop_graphs(ctx);                // recorded batches carry the old parameters
    if (report_count) *report_count = nrep;
    return dev_status(e);
}

fic_status fic_tune_save(fic_ctx *ctx, const char *path)
{
    if (!ctx || !path) return FIC_ERR_INVALID_ARG;
    std::string out = "{\n \"format\": \"fic-tune-1\",\n";
    char line[512];
    snprintf(line, sizeof line,
             " \"arch\": \"%s\",\n \"kernel_hash\": \"%s\",\n \"batch_separate\": %d,\n"
             " \"rows\": [",
             ctx->arch, FIC_KERNEL_HASH, ctx->batch_separate ? 1 : 0);
    out += line;
    for (size_t i = 0; i < ctx->tune.size(); ++i) {
        const auto &t = ctx->tune[i];
        snprintf(line, sizeof line, "%s\n  {\"range_size\": %d, \"dlog2\": %d, \"chunk_log2\": [",
                 i ? "," : "", t.b, t.dlog);
        out += line;
        for (int k = 0; k < fic::kTuneBuckets; ++k) {
            snprintf(line, sizeof line, "%s%d", k ? ", " : "", (int)t.row.chunk_log2[k]);
            out += line;
        }
        out += "], \"flush_at\": [";
        for (int k = 0; k < fic::kTuneBuckets; ++k) {
            snprintf(line, sizeof line, "%s%d", k ? ", " : "", (int)t.row.flush_at[k]);
            out += line;
        }
        out += "], \"xcd\": [";
        for (int k = 0; k < fic::kTuneBuckets; ++k) {
            snprintf(line, sizeof line, "%s%d", k ? ", " : "", (int)t.row.xcd[k]);
            out += line;
        }
        out += "]}";
    }
    out += "\n ]\n}\n";
    FILE *f = fopen(path, "wb");
    if (!f) return FIC_ERR_INVALID_ARG;
    const bool ok = fwrite(out.data(), 1, out.size(), f) == out.size();
    return (fclose(f) == 0 && ok) ? FIC_OK : FIC_ERR_INVALID_ARG;
}

}  // extern "C"

// JSON helpers of the tuning cache (C++ types: outside the C block)
namespace {
// The string value of "key" in text (after the key's colon), or "".
std::string json_str(const char *text, const char *key)
{
    std::string k = std::string("\"") + key + "\"";
    const char *p = strstr(text, k.c_str());
    if (!p) return "";
    p = strchr(p + k.size(), ':');
    if (!p) return "";
    p = strchr(p, '"');
    if (!p) return "";
    const char *q = strchr(p + 1, '"');
    if (!q) return "";
    return std::string(p + 1, q);
}
// Integer after "key": in [p, end); advances p past it. False if missing.
bool json_int(const char *&p, const char *end, const char *key, long &v)
{
    std::string k = std::string("\"") + key + "\"";
    const char *q = strstr(p, k.c_str());
    if (!q || q >= end) return false;
    q = strchr(q + k.size(), ':');
    if (!q || q >= end) return false;
    char *e = nullptr;
    v = strtol(q + 1, &e, 10);
    if (e == q + 1) return false;
    p = e;
    return true;
}
// kTuneBuckets integers of the array after "key".
bool json_ints(const char *&p, const char *end, const char *key, long *v)
{
    std::string k = std::string("\"") + key + "\"";
    const char *q = strstr(p, k.c_str());
    if (!q || q >= end) return false;
    q = strchr(q + k.size(), '[');
    if (!q || q >= end) return false;
    ++q;
    for (int i = 0; i < fic::kTuneBuckets; ++i) {
        char *e = nullptr;
        v[i] = strtol(q, &e, 10);
        if (e == q) return false;
        q = e;
        while (*q == ' ' || *q == ',' || *q == '\n') ++q;
    }
    if (*q != ']') return false;
    p = q + 1;
    return true;
}
}  // namespace

extern "C" {

fic_status fic_tune_load(fic_ctx *ctx, const char *path)
{
    if (!ctx || !path) return FIC_ERR_INVALID_ARG;
    FILE *f = fopen(path, "rb");
    if (!f) return FIC_ERR_INVALID_ARG;
    std::string text;
    char buf[4096];
    size_t nr;
    while ((nr = fread(buf, 1, sizeof buf, f)) > 0) {
        text.append(buf, nr);
        if (text.size() > (1u << 20)) break;
    }
    fclose(f);
    if (json_str(text.c_str(), "format") != "fic-tune-1") return FIC_ERR_INVALID_ARG;
    if (json_str(text.c_str(), "arch") != ctx->arch ||
        json_str(text.c_str(), "kernel_hash") != FIC_KERNEL_HASH)
        return FIC_ERR_UNSUPPORTED;   // written for another device or other kernels
    std::vector<fic_ctx::TuneEntry> rows;
    const char *p = strstr(text.c_str(), "\"rows\"");
    const char *end = text.c_str() + text.size();
    if (!p) return FIC_ERR_INVALID_ARG;
    // the batch launch structure: optional (0: one combined search); a
    // top-level key (no row has one), so it may come anywhere
    long sep = 0;
    {
        const char *sk = strstr(text.c_str(), "\"batch_separate\"");
        if (sk) {
            const char *q = sk;
            if (!json_int(q, end, "batch_separate", sep) || (sep != 0 && sep != 1))
                return FIC_ERR_INVALID_ARG;
        }
    }
    for (;;) {
        const char *q = strstr(p, "\"range_size\"");
        if (!q) break;
        long b = 0, dl = 0, cl[fic::kTuneBuckets], fl[fic::kTuneBuckets], xc[fic::kTuneBuckets];
        if (!json_int(q, end, "range_size", b) || !json_int(q, end, "dlog2", dl) ||
            !json_ints(q, end, "chunk_log2", cl) || !json_ints(q, end, "flush_at", fl))
            return FIC_ERR_INVALID_ARG;
        // "xcd" is optional (0: one queue); it belongs to this row only if it
        // comes before the next row
        {
            const char *nx = strstr(q, "\"range_size\"");
            const char *xk = strstr(q, "\"xcd\"");
            if (xk && (!nx || xk < nx)) {
                if (!json_ints(q, end, "xcd", xc)) return FIC_ERR_INVALID_ARG;
            } else {
                for (int k = 0; k < fic::kTuneBuckets; ++k) xc[k] = 0;
            }
        }
        if ((b != 4 && b != 8 && b != 16) || dl < 0 || dl > 40) return FIC_ERR_INVALID_ARG;
        fic_ctx::TuneEntry t;
        t.b = (int32_t)b;
        t.dlog = (int32_t)dl;
        for (int k = 0; k < fic::kTuneBuckets; ++k) {
            if (cl[k] < fic::kChunkLog2Min || cl[k] > fic::kChunkLog2Max || fl[k] < 0 || fl[k] > 256)
                return FIC_ERR_INVALID_ARG;
            if (xc[k] != 0 && xc[k] != 1) return FIC_ERR_INVALID_ARG;
            t.row.chunk_log2[k] = (int8_t)cl[k];
            t.row.flush_at[k] = (int16_t)fl[k];
            t.row.xcd[k] = (uint8_t)xc[k];
        }
        rows.push_back(t);
        p = q;
    }
    ctx->tune.clear();
    for (const auto &t : rows) set_tune_row(ctx, t.b, t.dlog, t.row);
    ctx->batch_separate = sep != 0;
    if (ctx->device >= 0 && enter(ctx) == FIC_OK) drop_graphs(ctx);
    return FIC_OK;
}

}  // extern "C"
