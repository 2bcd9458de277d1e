// C ABI of the t3pcf library (declared in include/t3pcf.h).
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <cstring>
#include <new>

#include "t3_internal.h"

namespace t3 {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

static thread_local Budget *g_budget = nullptr;
static thread_local Arena *g_arena = nullptr;

Budget *active_budget() { return g_budget; }

BudgetScope::BudgetScope(Budget *b) : prev(g_budget) { g_budget = b; }

BudgetScope::~BudgetScope() { g_budget = prev; }

ArenaScope::ArenaScope(Arena *a) : prev(g_arena), mine(a) { g_arena = a; }

ArenaScope::~ArenaScope()
{
    // every buffer carved in the scope gets its plan-owned state back
    for (auto it = mine->saved.rbegin(); it != mine->saved.rend(); ++it) *it->first = it->second;
    mine->saved.clear();
    g_arena = prev;
}

static bool in_arena(const Arena *ar, const void *p)
{
    return ar && p && (const char *)p >= ar->base && (const char *)p < ar->base + ar->size;
}

int DevBuf::reserve(size_t want)
{
    if (Arena *ar = g_arena) {
        // carve from the arena: no allocation, no synchronisation
        const bool carved = in_arena(ar, ptr);
        if (carved && want <= bytes) return T3_OK;
        const size_t need = arena_bytes(want);
        if (need > ar->size - ar->used)
            return fail(T3_ENOMEM, "scratch: " + std::to_string(need) + " more bytes needed, " +
                                       std::to_string(ar->size - ar->used) + " of " + std::to_string(ar->size) +
                                       " left");
        if (!carved) ar->saved.emplace_back(this, *this);
        ptr = ar->base + ar->used;
        bytes = need;
        ar->used += need;
        return T3_OK;
    }
    if (want <= bytes && ptr) return T3_OK;
    const size_t b = want < 256 ? 256 : want;
    Budget *bg = g_budget;
    // the limit is checked before the old buffer is given up, so a refused
    // request leaves the plan as it was
    if (bg && bg->limit > 0 && bg->used - (int64_t)bytes + (int64_t)b > bg->limit)
        return fail(T3_ENOMEM, "workspace limit: " + std::to_string(b) + " bytes more would exceed "
                                   "max_workspace_bytes = " + std::to_string(bg->limit) + " (in use " +
                                   std::to_string(bg->used) + ")");
    if (ptr) (void)hipDeviceSynchronize();  // earlier launches may still read the old buffer
    release();
    if (hipMalloc(&ptr, b) != hipSuccess) {
        (void)hipGetLastError();
        ptr = nullptr;
        bytes = 0;
        return fail(T3_ENOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
    }
    bytes = b;
    if (bg) {
        bg->used += (int64_t)b;
        bg->peak = std::max(bg->peak, bg->used);
    }
    return T3_OK;
}

void DevBuf::release()
{
    if (in_arena(g_arena, ptr)) {  // carved, not allocated
        ptr = nullptr;
        bytes = 0;
        return;
    }
    if (ptr) {
        (void)hipFree(ptr);
        if (g_budget) g_budget->used -= (int64_t)bytes;
    }
    ptr = nullptr;
    bytes = 0;
}

int timing_begin_call(t3_plan *plan)
{
    plan->events_used = 0;
    for (int i = 0; i < 4; ++i) {
        plan->stage_ms[i] = 0.0;
        plan->stage_launches[i] = 0;
    }
    return T3_OK;
}

int timing_mark(t3_plan *plan, int stage, bool start, hipStream_t s)
{
    if (!(plan->flags & T3_FLAG_TIMING)) return T3_OK;
    if (start) {
        if (plan->events.size() < 2 * (plan->events_used + 1)) {
            hipEvent_t a, b;
            T3_HIP_CHECK(hipEventCreate(&a));
            T3_HIP_CHECK(hipEventCreate(&b));
            plan->events.push_back(a);
            plan->events.push_back(b);
            plan->event_stage.push_back(0);
        }
        plan->event_stage[plan->events_used] = stage;
        T3_HIP_CHECK(hipEventRecord(plan->events[2 * plan->events_used], s));
    } else {
        T3_HIP_CHECK(hipEventRecord(plan->events[2 * plan->events_used + 1], s));
        ++plan->events_used;
        ++plan->stage_launches[stage];
    }
    return T3_OK;
}

int timing_end_call(t3_plan *plan)
{
    if (!(plan->flags & T3_FLAG_TIMING)) return T3_OK;
    for (size_t i = 0; i < plan->events_used; ++i) {
        float ms = 0.f;
        T3_HIP_CHECK(hipEventElapsedTime(&ms, plan->events[2 * i], plan->events[2 * i + 1]));
        plan->stage_ms[plan->event_stage[i]] += ms;
    }
    return T3_OK;
}

int choose_chunk(const t3_plan *plan, const ChunkLayout &L)
{
    int K = plan->chunk_req;
    if (K <= 0) {
        // Large chunks: every chunk ends with a partly filled round of
        // stage-1 workgroups (512 resident, 4 centres each), so fewer,
        // longer launches waste less (measured on the 1M field: 8.7k centres
        // per chunk 1125 ms of stage 1, 64k centres 994 ms).  About 1 GiB of
        // planes per catalog, at most 64k centres, whole rounds of 2048: the
        // n_max = 30 pass gains under 1% from 4 GiB chunks (262k centres),
        // not worth four times the memory.  The order-segment pass, whose centres take about four
        // times longer each, gains from 4 GiB (4M field, n_max = 40: 139k
        // centres per chunk 4.5% faster than 35k).  Stage 2 addresses a
        // catalog's planes with 32-bit float offsets: below 2^30 floats here.
        const bool seg = scan_uses_segments(plan);
        const double per_centre = (double)L.n_planes() * L.B * sizeof(float);
        K = (int)((seg ? 4.0 : 1.0) * 1024 * 1024 * 1024 / per_centre);
        if (K > (seg ? 262144 : 65536)) K = seg ? 262144 : 65536;
        K = K >= 2048 ? (K & ~2047) : K;
    }
    if (K < 256) K = 256;
    K = (K + 255) & ~255;
    return K;
}

static int check_catalog(const t3_catalog *c, const char *what)
{
    if (!c) return fail(T3_EINVAL, std::string(what) + ": null catalog");
    if (c->n < 0 || c->n > (int64_t)0x7fffffff)
        return fail(T3_EINVAL, std::string(what) + ": catalog size out of range");
    if (c->n > 0 && (!c->x || !c->y || !c->g1 || !c->g2 || !c->w))
        return fail(T3_EINVAL, std::string(what) + ": null catalog array");
    return T3_OK;
}

static int prepare_small(t3_plan *plan, hipStream_t s)
{
    T3_TRY(plan->flag.reserve(sizeof(int) * 4));
    T3_TRY(plan->counter.reserve(sizeof(unsigned long long) * 4));
    T3_HIP_CHECK(hipMemsetAsync(plan->flag.ptr, 0, sizeof(int) * 4, s));
    T3_HIP_CHECK(hipMemsetAsync(plan->counter.ptr, 0, sizeof(unsigned long long) * 4, s));
    return T3_OK;
}

static ChunkLayout layout_of(const t3_plan *plan)
{
    ChunkLayout L;
    L.n_max = plan->n_max;
    L.w_max = plan->w_max;
    L.B = plan->B;
    L.K = 0;
    L.K = choose_chunk(plan, L);
    return L;
}

// Forward pass over n_z catalogs: centres of catalog z1 (list or all)
// against every catalog; output block [z1][z2][z3] (n_z = 1: one block).
static int forward_impl(t3_plan *plan, const t3_catalog *cats, int n_z, const int32_t *const *centres,
                        const int64_t *n_centres, double *ups_out, int64_t *n_pairs, hipStream_t s)
{
    T3_TRY(timing_begin_call(plan));
    T3_TRY(prepare_small(plan, s));
    if (plan->scan_var < 0) T3_TRY(scan_prepare(plan));
    int64_t n_all = 0;
    for (int z = 0; z < n_z; ++z) n_all += cats[z].n;
    const CellGrid grid = choose_grid(plan, n_all > 0 ? n_all / n_z : 0);
    T3_TRY(timing_mark(plan, 0, true, s));
    for (int z = 0; z < n_z; ++z) T3_TRY(build_cells(plan, plan->cats[z], cats[z], grid, s));
    for (int z = 0; z < n_z; ++z) {
        if (n_centres[z] >= 0)
            T3_TRY(gather_centres(plan, cats[z], centres[z], n_centres[z], plan->csets[z], s));
        else
            T3_TRY(gather_sorted_centres(plan, plan->cats[z], plan->csets[z], s));
    }
    T3_TRY(timing_mark(plan, 0, false, s));
    T3_TRY(check_flag(plan, s, n_z > 1 ? "t3_forward_tomo" : "t3_forward"));
    // leading bins with few neighbours per centre: one lane per centre
    // (the densest catalog decides for every catalog of a tomographic call)
    int n_lane = plan->B;
    for (int z = 0; z < n_z; ++z) {
        int k = 0;
        T3_TRY(lane_bins(plan, plan->cats[z], 0, plan->B, plan->lane_neighbours, s, &k));
        if (plan->cats[z].n > 0) n_lane = std::min(n_lane, k);
    }
    if (n_lane == plan->B && n_all == 0) n_lane = 0;

    ChunkLayout L = layout_of(plan);
    if (plan->chunk_req <= 0) {
        // n_z plane sets are live at once, each of the automatic size (at
        // most 8 catalogs: 8 GiB of planes at n_max <= 32; the 5-bin
        // tomography measured 7.49 s per call with 26k centres per chunk,
        // 7.39 s with 65k), and never more than the centres there are
        // (small problems keep small buffers)
        int K = L.K;
        int64_t most = 0;
        for (int z = 0; z < n_z; ++z) most = std::max<int64_t>(most, plan->csets[z].n);
        if ((int64_t)K > most) K = (int)std::min<int64_t>(K, (most + 255) & ~(int64_t)255);
        K = K < 256 ? 256 : (K & ~255);
        L.K = K;
    }
    // catalogs densest first (balances the stage-1 work queue)
    int order[8];
    for (int z = 0; z < n_z; ++z) order[z] = z;
    for (int i = 1; i < n_z; ++i)
        for (int j = i; j > 0 && cats[order[j]].n > cats[order[j - 1]].n; --j) std::swap(order[j], order[j - 1]);
    const size_t per_set = (size_t)2 * L.out_blocks() * plan->B * plan->B;
    const size_t n_out = per_set * (size_t)n_z * n_z * n_z;
    const size_t zstride = L.floats();
    // every buffer the schedule touches is reserved before it is recorded
    // (with kept planes the chunk buffer is not used)
    const bool keep = (plan->flags & T3_FLAG_KEEP_PLANES) && n_z == 1 && n_centres[0] < 0;
    if (!keep) T3_TRY(plan->chunk.reserve(sizeof(float) * zstride * (size_t)n_z));
    T3_TRY(reserve_contract(plan, L, n_z));
    T3_TRY(plan->queue.reserve(sizeof(unsigned) * 4));
    const SortedCatalog *cl[8];
    for (int z = 0; z < n_z; ++z) cl[z] = &plan->cats[z];
    const bool jk = !(plan->flags & T3_FLAG_KEEP_JK);
    const bool timing = (plan->flags & T3_FLAG_TIMING) != 0;
    const bool graph = !timing && !(plan->flags & T3_FLAG_NO_GRAPH);
    // every chunk's planes in a buffer of their own, for t3_backward
    plan->kept_seq = -1;
    if (keep) {
        const int64_t n_chunks = (plan->csets[0].n + L.K - 1) / L.K;
        T3_TRY(plan->kept.reserve(sizeof(float) * zstride * (size_t)std::max<int64_t>(n_chunks, 1)));
    }

    // the captured schedule writes into a plan-owned buffer, copied to the
    // caller's output after each launch, so that a replay does not depend
    // on where the caller's output lives
    if (graph) T3_TRY(plan->graph_out.reserve(sizeof(double) * n_out));
    double *const sched_out = graph ? plan->graph_out.as<double>() : ups_out;
    auto schedule = [&](hipStream_t q) -> int {
        T3_TRY(zero_doubles(sched_out, n_out, q));
        for (int z1 = 0; z1 < n_z; ++z1) {
            const CentreSet &cs = plan->csets[z1];
            double *out = sched_out + per_set * (size_t)n_z * n_z * z1;
            for (int64_t c0 = 0; c0 < cs.n; c0 += L.K) {
                const int n = (int)((cs.n - c0) < L.K ? (cs.n - c0) : L.K);
                float *planes = keep ? plan->kept.as<float>() + (size_t)(c0 / L.K) * zstride : plan->chunk.as<float>();
                T3_TRY(timing_mark(plan, 1, true, q));
                T3_TRY(scan_chunk(plan, cl, order, n_z, cs, c0, n, L, planes, zstride,
                                  plan->counter.as<unsigned long long>(), plan->scan_mode, q, 0, plan->B, n_lane));
                T3_TRY(timing_mark(plan, 1, false, q));
                T3_TRY(timing_mark(plan, 2, true, q));
                T3_TRY(contract_chunk(plan, cs, c0, n, L, planes, zstride, n_z, jk, out, q));
                T3_TRY(timing_mark(plan, 2, false, q));
            }
        }
        return T3_OK;
    };

    if (graph) {
        // The captured schedule bakes in every launch shape and kernel
        // argument: shapes, buffer addresses, the cell grid, the lane-bin
        // split, launch mode, precision and flags.  It is captured once per
        // such key and replayed by later calls (the cell lists and centre
        // sets it reads are rebuilt in place before each launch).
        std::vector<int64_t> key;
        auto put = [&](int64_t v) { key.push_back(v); };
        int dev = 0;
        (void)hipGetDevice(&dev);
        put(dev);
        put(n_z);
        put(L.K);
        put(L.n_max);
        put(L.w_max);
        put(L.B);
        put(n_lane);
        put(plan->scan_mode);
        put(plan->scan_var);
        put(plan->tile_mode);
        put(plan->precision);
        put((int64_t)plan->flags);
        put(keep ? 1 : 0);
        put(jk ? 1 : 0);
        for (const void *p : {plan->graph_out.ptr, plan->chunk.ptr, plan->kept.ptr, plan->partial.ptr, plan->diag.ptr,
                              plan->scales.ptr, plan->counter.ptr, plan->queue.ptr, plan->dest.ptr})
            put((int64_t)(uintptr_t)p);
        for (int z = 0; z < n_z; ++z) {
            const SortedCatalog &c = plan->cats[z];
            const CentreSet &cs = plan->csets[z];
            for (int64_t v : {(int64_t)order[z], c.n, (int64_t)(uintptr_t)c.pos.ptr, (int64_t)(uintptr_t)c.cw.ptr,
                              (int64_t)(uintptr_t)c.cell_start.ptr, (int64_t)c.grid.cell, (int64_t)c.grid.ncx,
                              (int64_t)c.grid.ncy, (int64_t)c.grid.ox, (int64_t)c.grid.oy, cs.n,
                              (int64_t)(uintptr_t)cs.pos.ptr, (int64_t)(uintptr_t)cs.cw.ptr})
                put(v);
        }
        if (!(plan->graph_exec && key == plan->graph_key)) {
            if (!plan->cap_stream)
                T3_HIP_CHECK(hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking));
            if (plan->graph_exec) {
                (void)hipGraphExecDestroy(plan->graph_exec);
                plan->graph_exec = nullptr;
                plan->graph_key.clear();
            }
            T3_HIP_CHECK(hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal));
            const int rc = schedule(plan->cap_stream);
            hipGraph_t g = nullptr;
            const hipError_t ec = hipStreamEndCapture(plan->cap_stream, &g);
            if (rc != T3_OK) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (ec != hipSuccess) return fail(T3_EHIP, std::string("graph capture: ") + hipGetErrorString(ec));
            const hipError_t ei = hipGraphInstantiate(&plan->graph_exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ei != hipSuccess) return fail(T3_EHIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
            plan->graph_key = std::move(key);
            ++plan->graph_captures;
        }
        T3_HIP_CHECK(hipGraphLaunch(plan->graph_exec, s));
        ++plan->graph_replays;
        T3_HIP_CHECK(hipMemcpyAsync(ups_out, sched_out, sizeof(double) * n_out, hipMemcpyDeviceToDevice, s));
    } else {
        T3_TRY(schedule(s));
    }
    unsigned long long pairs = 0;
    T3_HIP_CHECK(hipMemcpyAsync(&pairs, plan->counter.ptr, sizeof(pairs), hipMemcpyDeviceToHost, s));
    T3_HIP_CHECK(hipStreamSynchronize(s));
    T3_TRY(timing_end_call(plan));
    if (n_pairs) *n_pairs = (int64_t)pairs;
    if (keep) {
        plan->kept_L = L;
        plan->kept_cat = cats[0];
        plan->kept_seq = plan->cells_seq;
    }
    return T3_OK;
}

// Scratch of the no-allocation forward pass: one static array per GPU the
// library runs on, held until the process ends.  Host code never passes the
// array's name to a kernel (in host code it is a stand-in, not a device
// address): its device address is looked up once per device with that
// device current and kept.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[256] = {};

static int scratch_of_current_device(void **out)
{
    int dev = 0;
    T3_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 256) return fail(T3_EHIP, "scratch: device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(T3_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return T3_OK;
}

// Arena bytes a non-tomographic forward pass over n galaxies and n_c centres
// reserves with chunk layout L (the reservations of forward_impl in order:
// error flag and pair counter, destination tables, cell list, centre set,
// lane-bin counter, chunk planes, stage-2 partial sums, work counter).
static size_t noalloc_bytes(const t3_plan *plan, int64_t n, int64_t n_c, const CellGrid &g, const ChunkLayout &L)
{
    const size_t m = (size_t)(n_c > 0 ? n_c : 1);
    return arena_bytes(sizeof(int) * 4) + arena_bytes(sizeof(unsigned long long) * 4) +
           arena_bytes(sizeof(short) * scan_dest_entries(plan)) + cells_arena_bytes(n, g) +
           arena_bytes(sizeof(int2) * m) + arena_bytes(sizeof(float4) * m) + arena_bytes(sizeof(unsigned) * 4) +
           arena_bytes(sizeof(float) * L.floats()) + contract_arena_bytes(plan, L, 1) +
           arena_bytes(sizeof(unsigned) * 4);
}

}  // namespace t3

using namespace t3;

extern "C" {

const char *t3_version(void) { return "t3pcf 0.1 (gfx950)"; }

const char *t3_error_string(int code)
{
    switch (code) {
        case T3_OK: return "ok";
        case T3_EINVAL: return "invalid argument";
        case T3_ERANGE: return "parameter out of supported range";
        case T3_ENOMEM: return "device allocation failed";
        case T3_EHIP: return "HIP runtime error";
        case T3_ELATTICE: return "position outside the lattice box";
        default: return "unknown error";
    }
}

const char *t3_last_error_message(void) { return g_last_error.c_str(); }

int t3_plan_create(const t3_params *p, t3_plan **out)
{
    try {
        if (!p || !out) return fail(T3_EINVAL, "t3_plan_create: null argument");
        if (p->n_bins < 1 || !p->edges) return fail(T3_EINVAL, "t3_plan_create: need n_bins >= 1 and edges");
        if (p->n_bins > kMaxRadialBins) return fail(T3_ERANGE, "t3_plan_create: at most 64 radial bins");
        if (p->n_max < 0 || p->n_max > 64) return fail(T3_ERANGE, "t3_plan_create: n_max must be in [0, 64]");
        if (p->precision < T3_PREC_FP32 || p->precision > T3_PREC_BF16X6)
            return fail(T3_EINVAL, "t3_plan_create: unknown precision");
        if (p->flags & ~(T3_FLAG_KEEP_JK | T3_FLAG_TIMING | T3_FLAG_NO_GRAPH | T3_FLAG_EDGE_CORRECT | T3_FLAG_NO_LANE |
                         T3_FLAG_KEEP_PLANES | T3_FLAG_DETERMINISTIC))
            return fail(T3_EINVAL, "t3_plan_create: unknown flag");
        if (p->max_workspace_bytes < 0) return fail(T3_EINVAL, "t3_plan_create: max_workspace_bytes must be >= 0");
        const double unit = p->lattice_unit == 0.0 ? std::ldexp(1.0, -16) : p->lattice_unit;
        if (!(unit > 0.0) || !std::isfinite(unit)) return fail(T3_EINVAL, "t3_plan_create: bad lattice unit");
        for (int b = 0; b <= p->n_bins; ++b)
            if (!std::isfinite(p->edges[b])) return fail(T3_EINVAL, "t3_plan_create: non-finite edge");
        if (!(p->edges[0] > 0.0)) return fail(T3_EINVAL, "t3_plan_create: edges[0] must be > 0");
        for (int b = 0; b < p->n_bins; ++b)
            if (!(p->edges[b + 1] > p->edges[b]))
                return fail(T3_EINVAL, "t3_plan_create: edges must increase strictly");
        if (p->edges[p->n_bins] / unit >= std::ldexp(1.0, 25))
            return fail(T3_ERANGE, "t3_plan_create: largest edge must be below 2^25 lattice steps");
        if (p->box_size <= 0) return fail(T3_EINVAL, "t3_plan_create: box_size must be > 0");
        if ((int64_t)p->box_lo_x + p->box_size > ((int64_t)1 << 31) ||
            (int64_t)p->box_lo_y + p->box_size > ((int64_t)1 << 31))
            return fail(T3_ERANGE, "t3_plan_create: box exceeds the int32 lattice");
        if (p->cell_arcmin < 0.0 || !std::isfinite(p->cell_arcmin))
            return fail(T3_EINVAL, "t3_plan_create: bad cell size");
        if (p->chunk_centres < 0) return fail(T3_EINVAL, "t3_plan_create: bad chunk size");
        if (p->scan_mode < 0 || p->scan_mode > 1) return fail(T3_EINVAL, "t3_plan_create: bad scan mode");
        if (!(p->lane_neighbours >= 0.0 && p->lane_neighbours <= kLaneNeighbours))
            return fail(T3_EINVAL, "t3_plan_create: lane_neighbours must be in [0, 128] (0: automatic)");
        if (p->tile_mode < 0 || p->tile_mode > 1) return fail(T3_EINVAL, "t3_plan_create: bad tile mode");

        t3_plan *plan = new (std::nothrow) t3_plan();
        if (!plan) return fail(T3_ENOMEM, "t3_plan_create: host allocation failed");
        plan->B = p->n_bins;
        plan->n_max = p->n_max;
        plan->w_max = (p->flags & T3_FLAG_EDGE_CORRECT) ? 2 * p->n_max : p->n_max;
        plan->precision = p->precision;
        plan->flags = p->flags;
        plan->unit = unit;
        plan->box_lo_x = p->box_lo_x;
        plan->box_lo_y = p->box_lo_y;
        plan->box_size = p->box_size;
        plan->cell_arcmin = p->cell_arcmin;
        plan->chunk_req = p->chunk_centres;
        plan->scan_mode = p->scan_mode;
        plan->lane_neighbours = p->lane_neighbours > 0.0 ? p->lane_neighbours : kLaneNeighbours;
        plan->tile_mode = p->tile_mode;
        plan->budget.limit = p->max_workspace_bytes;
        plan->edges_lat.resize(p->n_bins + 1);
        plan->e2.resize(p->n_bins + 1);
        for (int b = 0; b <= p->n_bins; ++b) {
            const double e = p->edges[b] / unit;
            plan->edges_lat[b] = e;
            plan->e2[b] = e * e;
        }
        if (hipGetDevice(&plan->device) != hipSuccess) plan->device = 0;
        *out = plan;
        return T3_OK;
    } catch (...) {
        return fail(T3_ENOMEM, "t3_plan_create: exception");
    }
}

void t3_plan_destroy(t3_plan *plan)
{
    if (!plan) return;
    (void)hipDeviceSynchronize();
    for (auto &c : plan->cats) {
        c.pos.release();
        c.cw.release();
        c.cell_start.release();
        c.perm.release();
        c.keys.release();
        c.counts.release();
        c.scan_tmp.release();
    }
    plan->centres.pos.release();
    plan->centres.cw.release();
    plan->chunk.release();
    plan->kept.release();
    plan->graph_out.release();
    plan->partial.release();
    plan->diag.release();
    plan->flag.release();
    plan->dest.release();
    plan->scales.release();
    plan->counter.release();
    plan->misc.release();
    plan->misc2.release();
    plan->det.release();
    for (auto e : plan->events) (void)hipEventDestroy(e);
    for (auto &c : plan->csets) {
        c.pos.release();
        c.cw.release();
    }
    plan->queue.release();
    plan->tune_idx.release();
    plan->tune_out.release();
    plan->sph_a.release();
    plan->sph_b.release();
    plan->sph_out.release();
    for (auto &lv : plan->grid) lv.release();
    if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
    if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
    delete plan;
}

int t3_forward(t3_plan *plan, const t3_catalog *cat, const int32_t *centres, int64_t n_centres,
               double *ups_out, int64_t *n_pairs, void *stream)
{
    try {
        if (!plan || !ups_out) return fail(T3_EINVAL, "t3_forward: null argument");
        BudgetScope budget_scope(&plan->budget);
        T3_TRY(check_catalog(cat, "t3_forward"));
        if (n_centres < 0 && centres)
            return fail(T3_EINVAL, "t3_forward: n_centres < 0 (all galaxies) needs centres == NULL");
        if (n_centres > 0 && !centres) return fail(T3_EINVAL, "t3_forward: null centre list");
        if (n_centres > (int64_t)0x7fffffff) return fail(T3_EINVAL, "t3_forward: bad centre count");
        const int32_t *cl[1] = {centres};
        const int64_t nl[1] = {n_centres};
        return forward_impl(plan, cat, 1, cl, nl, ups_out, n_pairs, (hipStream_t)stream);
    } catch (...) {
        return fail(T3_EINVAL, "t3_forward: exception");
    }
}

int t3_forward_noalloc(t3_plan *plan, const t3_catalog *cat, const int32_t *centres, int64_t n_centres,
                       double *ups_out, int64_t *n_pairs, void *stream)
{
    try {
        if (!plan || !ups_out) return fail(T3_EINVAL, "t3_forward_noalloc: null argument");
        T3_TRY(check_catalog(cat, "t3_forward_noalloc"));
        if (n_centres < 0 && centres)
            return fail(T3_EINVAL, "t3_forward_noalloc: n_centres < 0 (all galaxies) needs centres == NULL");
        if (n_centres > 0 && !centres) return fail(T3_EINVAL, "t3_forward_noalloc: null centre list");
        if (n_centres > (int64_t)0x7fffffff) return fail(T3_EINVAL, "t3_forward_noalloc: bad centre count");
        void *base = nullptr;
        T3_TRY(scratch_of_current_device(&base));
        // the largest chunk capacity (a multiple of 256 centres, at most the
        // automatic one) whose buffers fit the scratch, decided before any launch
        const int64_t n_c = n_centres < 0 ? cat->n : n_centres;
        const CellGrid g = choose_grid(plan, cat->n);
        ChunkLayout L;
        L.n_max = plan->n_max;
        L.w_max = plan->w_max;
        L.B = plan->B;
        const int keep_req = plan->chunk_req;
        plan->chunk_req = 0;
        int K = choose_chunk(plan, L);
        plan->chunk_req = keep_req;
        K = (int)std::min<int64_t>(K, std::max<int64_t>(256, (n_c + 255) & ~(int64_t)255));
        size_t need = 0;
        for (; K >= 256; K -= 256) {
            L.K = K;
            need = noalloc_bytes(plan, cat->n, n_c, g, L);
            if (need <= kScratchBytes) break;
        }
        if (K < 256)
            return fail(T3_ENOMEM, "t3_forward_noalloc: " + std::to_string(cat->n) + " galaxies and " +
                                       std::to_string(n_c) + " centres need " + std::to_string(need) +
                                       " bytes of scratch even in chunks of 256 centres, more than the " +
                                       std::to_string(kScratchBytes) + " the library holds (use t3_forward)");
        // t3_forward's path, every buffer carved from the scratch: eager
        // launches (no graph capture, no timing events), the destination
        // tables rebuilt in the scratch; the plan's own state is restored
        const uint32_t keep_flags = plan->flags;
        const int keep_var = plan->scan_var;
        size_t keep_off[4];
        for (int k = 0; k < 4; ++k) keep_off[k] = plan->scan_dest_off[k];
        plan->chunk_req = K;
        plan->flags = (keep_flags | T3_FLAG_NO_GRAPH) & ~(T3_FLAG_TIMING | T3_FLAG_KEEP_PLANES);
        plan->scan_var = -1;
        Arena arena;
        arena.base = static_cast<char *>(base);
        arena.size = kScratchBytes;
        int rc;
        {
            ArenaScope scope(&arena);
            const int32_t *cl[1] = {centres};
            const int64_t nl[1] = {n_centres};
            rc = forward_impl(plan, cat, 1, cl, nl, ups_out, n_pairs, (hipStream_t)stream);
        }
        plan->chunk_req = keep_req;
        plan->flags = keep_flags;
        plan->scan_var = keep_var;
        for (int k = 0; k < 4; ++k) plan->scan_dest_off[k] = keep_off[k];
        return rc;
    } catch (...) {
        return fail(T3_EINVAL, "t3_forward_noalloc: exception");
    }
}

int t3_forward_tomo(t3_plan *plan, const t3_catalog *cats, int32_t n_z, const int32_t *const *centres,
                    const int64_t *n_centres, double *ups_out, int64_t *n_pairs, void *stream)
{
    try {
        if (!plan || !cats || !ups_out) return fail(T3_EINVAL, "t3_forward_tomo: null argument");
        BudgetScope budget_scope(&plan->budget);
        if (n_z < 1 || n_z > 8) return fail(T3_ERANGE, "t3_forward_tomo: n_z must be in [1, 8]");
        for (int z = 0; z < n_z; ++z) T3_TRY(check_catalog(&cats[z], "t3_forward_tomo"));
        if (centres && !n_centres) return fail(T3_EINVAL, "t3_forward_tomo: centres without counts");
        const int32_t *cl[8];
        int64_t nl[8];
        for (int z = 0; z < n_z; ++z) {
            cl[z] = centres ? centres[z] : nullptr;
            nl[z] = centres ? n_centres[z] : -1;
            if (nl[z] < 0 && cl[z]) return fail(T3_EINVAL, "t3_forward_tomo: count < 0 needs a NULL list");
            if (nl[z] > 0 && !cl[z]) return fail(T3_EINVAL, "t3_forward_tomo: null centre list");
            if (nl[z] > (int64_t)0x7fffffff) return fail(T3_EINVAL, "t3_forward_tomo: bad centre count");
        }
        return forward_impl(plan, cats, n_z, cl, nl, ups_out, n_pairs, (hipStream_t)stream);
    } catch (...) {
        return fail(T3_EINVAL, "t3_forward_tomo: exception");
    }
}

int t3_harmonics(t3_plan *plan, const t3_catalog *cat, const int32_t *centres, int64_t n_centres,
                 float *G_out, float *W_out, float *D_out, void *stream)
{
    try {
        if (!plan || !G_out || !W_out || !D_out || (n_centres > 0 && !centres))
            return fail(T3_EINVAL, "t3_harmonics: null argument");
        BudgetScope budget_scope(&plan->budget);
        T3_TRY(check_catalog(cat, "t3_harmonics"));
        if (n_centres < 0 || n_centres > (int64_t)0x7fffffff)
            return fail(T3_EINVAL, "t3_harmonics: bad centre count");
        hipStream_t s = (hipStream_t)stream;
        T3_TRY(prepare_small(plan, s));
        SortedCatalog &sc = plan->cats[0];
        T3_TRY(build_cells(plan, sc, *cat, choose_grid(plan, cat->n), s));
        T3_TRY(gather_centres(plan, *cat, centres, n_centres, plan->centres, s));
        T3_TRY(check_flag(plan, s, "t3_harmonics"));
        ChunkLayout L = layout_of(plan);
        if (plan->chunk_req <= 0 && (int64_t)L.K > n_centres)  // small requests, small buffers
            L.K = (int)std::max<int64_t>(256, (n_centres + 255) & ~(int64_t)255);
        T3_TRY(plan->chunk.reserve(sizeof(float) * L.floats()));
        int n_lane = 0;
        T3_TRY(lane_bins(plan, sc, 0, plan->B, plan->lane_neighbours, s, &n_lane));
        for (int64_t c0 = 0; c0 < n_centres; c0 += L.K) {
            const int n = (int)((n_centres - c0) < L.K ? (n_centres - c0) : L.K);
            const SortedCatalog *cl[1] = {&sc};
            T3_TRY(scan_chunk(plan, cl, nullptr, 1, plan->centres, c0, n, L, plan->chunk.as<float>(), 0,
                              plan->counter.as<unsigned long long>(), plan->scan_mode, s, 0, plan->B, n_lane));
            T3_TRY(harmonics_export(plan, plan->centres, L, plan->chunk.as<float>(), c0, n, G_out,
                                    W_out, D_out, s));
        }
        T3_HIP_CHECK(hipStreamSynchronize(s));
        return T3_OK;
    } catch (...) {
        return fail(T3_EINVAL, "t3_harmonics: exception");
    }
}

int t3_normalise_resum(t3_plan *plan, const double *ups, int32_t n_sets, int32_t n_phi,
                       double *gamma_n, double *gamma_phi, void *stream)
{
    if (!plan || !ups || !gamma_n) return fail(T3_EINVAL, "t3_normalise_resum: null argument");
    BudgetScope budget_scope(&plan->budget);
    if (n_sets < 1) return fail(T3_EINVAL, "t3_normalise_resum: n_sets must be >= 1");
    int n_z = 1;
    while (n_z * n_z * n_z < n_sets) ++n_z;
    if (n_z * n_z * n_z != n_sets) return fail(T3_EINVAL, "t3_normalise_resum: n_sets must be a cube");
    if (gamma_phi && (n_phi < 1 || n_phi > 4096))
        return fail(T3_ERANGE, "t3_normalise_resum: n_phi must be in [1, 4096]");
    return normalise_resum(plan, ups, n_sets, n_z, n_phi, gamma_n, gamma_phi, (hipStream_t)stream);
}

int t3_x_to_centroid(t3_plan *plan, const double *gamma_phi_x, int32_t n_sets, int32_t n_phi,
                     const double *theta, double *gamma_phi_cent, void *stream)
{
    if (!plan || !gamma_phi_x || !gamma_phi_cent) return fail(T3_EINVAL, "t3_x_to_centroid: null argument");
    BudgetScope budget_scope(&plan->budget);
    if (n_sets < 1) return fail(T3_EINVAL, "t3_x_to_centroid: n_sets must be >= 1");
    if (n_phi < 1 || n_phi > 4096) return fail(T3_ERANGE, "t3_x_to_centroid: n_phi must be in [1, 4096]");
    if (theta)
        for (int b = 0; b < plan->B; ++b)
            if (!(theta[b] > 0.0) || !std::isfinite(theta[b]))
                return fail(T3_EINVAL, "t3_x_to_centroid: theta must be positive and finite");
    return x_to_centroid(plan, gamma_phi_x, n_sets, n_phi, theta, gamma_phi_cent, (hipStream_t)stream);
}

int t3_forward_sphere(t3_plan *plan, const t3_sphere_catalog *cat, const t3_patch *patches, int32_t n_patches,
                      double theta_max_arcmin, double *ups_out, int64_t *n_pairs, void *stream)
{
    try {
        if (!plan || !cat || !patches || !ups_out || !n_pairs)
            return fail(T3_EINVAL, "t3_forward_sphere: null argument");
        BudgetScope budget_scope(&plan->budget);
        if (n_patches < 1) return fail(T3_EINVAL, "t3_forward_sphere: need at least one patch");
        if (cat->n < 0 || cat->n > (int64_t)0x7fffffff)
            return fail(T3_EINVAL, "t3_forward_sphere: catalog size out of range");
        if (cat->n > 0 && (!cat->ra || !cat->dec || !cat->g1 || !cat->g2 || !cat->w))
            return fail(T3_EINVAL, "t3_forward_sphere: null catalog array");
        if (!(theta_max_arcmin > 0.0) || !std::isfinite(theta_max_arcmin))
            return fail(T3_EINVAL, "t3_forward_sphere: theta_max must be positive");
        if (theta_max_arcmin < plan->edges_lat[plan->B] * plan->unit)
            return fail(T3_EINVAL, "t3_forward_sphere: theta_max below the largest bin edge");
        for (int k = 0; k < n_patches; ++k) {
            const t3_patch &p = patches[k];
            if (!(p.ra_lo < p.ra_hi) || !(p.dec_lo < p.dec_hi) || p.ra_hi - p.ra_lo > 30.0 ||
                p.dec_hi - p.dec_lo > 30.0 || p.dec_lo < -89.0 || p.dec_hi > 89.0)
                return fail(T3_EINVAL, "t3_forward_sphere: bad patch (sides <= 30 deg, |dec| <= 89)");
        }
        hipStream_t s = (hipStream_t)stream;
        const size_t per = (size_t)2 * (4 * (plan->n_max + 1) + plan->w_max + 1) * plan->B * plan->B;
        T3_TRY(zero_doubles(ups_out, per, s));
        T3_TRY(plan->sph_out.reserve(sizeof(double) * per));
        int64_t total = 0;
        for (int k = 0; k < n_patches; ++k) {
            t3_catalog view{};
            const int32_t *core = nullptr;
            int64_t n_core = 0;
            T3_TRY(sphere_patch(plan, *cat, patches[k], theta_max_arcmin, &view, &core, &n_core, s));
            if (n_core == 0) continue;
            int64_t np = 0;
            T3_TRY(forward_impl(plan, &view, 1, &core, &n_core, plan->sph_out.as<double>(), &np, s));
            T3_TRY(add_doubles(ups_out, plan->sph_out.as<double>(), per, s));
            total += np;
        }
        *n_pairs = total;
        return T3_OK;
    } catch (...) {
        return fail(T3_EINVAL, "t3_forward_sphere: exception");
    }
}

int t3_forward_grid(t3_plan *plan, const t3_catalog *cat, int64_t delta, const int32_t *levels, int32_t method,
                    double *ups_out, int64_t *n_pairs, void *stream)
{
    try {
        if (!plan || !levels || !ups_out) return fail(T3_EINVAL, "t3_forward_grid: null argument");
        BudgetScope budget_scope(&plan->budget);
        T3_TRY(check_catalog(cat, "t3_forward_grid"));
        if (method != T3_GRID_AUTO && method != T3_GRID_DIRECT && method != T3_GRID_FFT)
            return fail(T3_EINVAL, "t3_forward_grid: unknown method");
        if (delta < 1 || delta > plan->box_size)
            return fail(T3_EINVAL, "t3_forward_grid: delta must be in [1, box_size] lattice steps");
        for (int b = 0; b < plan->B; ++b) {
            const int l = levels[b];
            if (l < 0 || l > kMaxGridLevels)
                return fail(T3_EINVAL, "t3_forward_grid: levels must be in [0, 8]");
            if (b > 0 && l < levels[b - 1]) return fail(T3_EINVAL, "t3_forward_grid: levels must not decrease");
            if (l > 0) {
                const int64_t side = delta << (l - 1);
                if (side > plan->box_size)
                    return fail(T3_ERANGE, "t3_forward_grid: pixel side of a level exceeds the box");
                if ((plan->box_size + side - 1) / side > 8192)
                    return fail(T3_ERANGE, "t3_forward_grid: more than 8192 pixels along the box (coarser delta "
                                           "or a smaller box)");
            }
        }
        return forward_grid(plan, *cat, delta, levels, method, ups_out, n_pairs, (hipStream_t)stream);
    } catch (...) {
        return fail(T3_EINVAL, "t3_forward_grid: exception");
    }
}

int t3_aperture_stats(t3_plan *plan, const double *gamma_phi_cent, int32_t n_sets, int32_t n_phi,
                      const double *apertures, int32_t n_ap, double *corr_out, double *stats_out, void *stream)
{
    if (!plan || !gamma_phi_cent || !apertures || !corr_out)
        return fail(T3_EINVAL, "t3_aperture_stats: null argument");
    BudgetScope budget_scope(&plan->budget);
    if (n_sets < 1 || n_ap < 1) return fail(T3_EINVAL, "t3_aperture_stats: n_sets and n_ap must be >= 1");
    if (n_phi < 1 || n_phi > 4096) return fail(T3_ERANGE, "t3_aperture_stats: n_phi must be in [1, 4096]");
    if (n_ap > 65535) return fail(T3_ERANGE, "t3_aperture_stats: at most 65535 aperture triples per call");
    for (int64_t k = 0; k < 3 * (int64_t)n_ap; ++k)
        if (!(apertures[k] > 0.0) || !std::isfinite(apertures[k]))
            return fail(T3_EINVAL, "t3_aperture_stats: aperture radii must be positive and finite");
    return aperture_stats(plan, gamma_phi_cent, n_sets, n_phi, apertures, n_ap, corr_out, stats_out,
                          (hipStream_t)stream);
}

int t3_normalise_backward(t3_plan *plan, const double *ups, int32_t n_sets, const double *grad_gamma_n,
                          double *grad_ups, void *stream)
{
    if (!plan || !ups || !grad_gamma_n || !grad_ups)
        return fail(T3_EINVAL, "t3_normalise_backward: null argument");
    BudgetScope budget_scope(&plan->budget);
    if (plan->flags & T3_FLAG_EDGE_CORRECT)
        return fail(T3_EINVAL, "t3_normalise_backward: no adjoint of the edge-corrected normalisation");
    if (n_sets < 1) return fail(T3_EINVAL, "t3_normalise_backward: n_sets must be >= 1");
    return normalise_backward(plan, ups, grad_gamma_n, n_sets, grad_ups, (hipStream_t)stream);
}

namespace {
// The settings the autotuner chooses.
struct TuneChoice {
    double cell = 0;    // cell side, arcmin
    int mode = 0;       // stage-1 launch mode
    double lane = 0;    // lane-kernel threshold, expected neighbours per centre
    int tile = 0;       // stage-2 tile shape for B <= 24
    int chunk = 0;      // chunk capacity request (0: automatic)
};

void apply_choice(t3_plan *plan, const TuneChoice &c)
{
    plan->cell_arcmin = c.cell;
    plan->scan_mode = c.mode;
    plan->lane_neighbours = c.lane;
    plan->tile_mode = c.tile;
    plan->chunk_req = c.chunk;
}

TuneChoice choice_of(const t3_plan *plan)
{
    TuneChoice c;
    c.cell = plan->cell_arcmin;
    c.mode = plan->scan_mode;
    c.lane = plan->lane_neighbours;
    c.tile = plan->tile_mode;
    c.chunk = plan->chunk_req;
    return c;
}
}  // namespace

int t3_autotune(t3_plan *plan, const t3_catalog *cats, int32_t n_z, int64_t sample_per_bin, double *best_ms,
                void *stream)
{
    try {
        if (!plan || !cats) return fail(T3_EINVAL, "t3_autotune: null argument");
        BudgetScope budget_scope(&plan->budget);
        if (n_z < 1 || n_z > 8) return fail(T3_ERANGE, "t3_autotune: n_z must be in [1, 8]");
        if (sample_per_bin < 1) return fail(T3_EINVAL, "t3_autotune: sample_per_bin must be >= 1");
        for (int z = 0; z < n_z; ++z) T3_TRY(check_catalog(&cats[z], "t3_autotune"));
        hipStream_t s = (hipStream_t)stream;
        int64_t n_all = 0;
        for (int z = 0; z < n_z; ++z) n_all += cats[z].n;
        const int64_t n_mean = n_all / n_z;
        int size_class = 0;
        for (int64_t v = n_mean; v > 1; v >>= 1) ++size_class;
        static std::mutex mu;
        static std::map<std::tuple<int, int, int, int, int, int64_t, int64_t, int>, TuneChoice> cache;
        const int64_t sample_class = sample_per_bin;
        const auto key = std::make_tuple(plan->B, plan->n_max, n_z, plan->precision, size_class, plan->box_size,
                                         sample_class, plan->chunk_req);
        {
            std::lock_guard<std::mutex> lk(mu);
            auto it = cache.find(key);
            if (it != cache.end()) {
                apply_choice(plan, it->second);
                if (best_ms) *best_ms = 0.0;
                return T3_OK;
            }
        }
        // deterministic stride sample of centres per catalog
        std::vector<int32_t> idx;
        std::vector<int64_t> cnt(n_z), off(n_z);
        for (int z = 0; z < n_z; ++z) {
            const int64_t n = cats[z].n, k = std::min<int64_t>(n, sample_per_bin);
            off[z] = (int64_t)idx.size();
            cnt[z] = k;
            for (int64_t j = 0; j < k; ++j) idx.push_back((int32_t)((j * n) / k));
        }
        T3_TRY(plan->tune_idx.reserve(sizeof(int32_t) * (idx.size() + 1)));
        T3_HIP_CHECK(hipMemcpy(plan->tune_idx.ptr, idx.data(), sizeof(int32_t) * idx.size(),
                               hipMemcpyHostToDevice));
        const int32_t *cl[8];
        for (int z = 0; z < n_z; ++z) cl[z] = plan->tune_idx.as<int32_t>() + off[z];
        const size_t n_out = (size_t)2 * (4 * (plan->n_max + 1) + plan->w_max + 1) * plan->B * plan->B *
                             n_z * n_z * n_z;
        T3_TRY(plan->tune_out.reserve(sizeof(double) * n_out));

        const double area = (double)plan->box_size * (double)plan->box_size;
        const double auto_side = std::sqrt(8.0 * area / (double)std::max<int64_t>(n_mean, 1)) * plan->unit;
        const TuneChoice keep = choice_of(plan);
        const uint32_t keep_flags = plan->flags;
        plan->flags = (plan->flags & ~T3_FLAG_TIMING) | T3_FLAG_NO_GRAPH;
        hipEvent_t e0, e1;
        T3_HIP_CHECK(hipEventCreate(&e0));
        T3_HIP_CHECK(hipEventCreate(&e1));
        int rc = T3_OK;
        // best of two timed forward passes of the sample with settings c
        auto time_of = [&](const TuneChoice &c) -> double {
            apply_choice(plan, c);
            double ms_best = 1e300;
            for (int rep = 0; rep < 2 && rc == T3_OK; ++rep) {
                if ((rc = (hipEventRecord(e0, s) == hipSuccess) ? T3_OK : T3_EHIP) != T3_OK) break;
                rc = forward_impl(plan, cats, n_z, cl, cnt.data(), plan->tune_out.as<double>(), nullptr, s);
                if (rc != T3_OK) break;
                float ms = 0.f;
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    rc = fail(T3_EHIP, "t3_autotune: event timing failed");
                    break;
                }
                ms_best = std::min(ms_best, (double)ms);
            }
            return ms_best;
        };
        // One coordinate at a time, each from the best so far (ties keep the
        // earlier candidate): cell size x stage-1 launch mode, then the
        // lane-kernel threshold, the stage-2 tile shape (B <= 24) and the
        // chunk capacity (when the plan leaves it automatic).
        TuneChoice best = keep;
        double best_t = 1e300;
        auto consider = [&](const TuneChoice &c) {
            if (rc != T3_OK) return;
            const double t = time_of(c);
            if (rc == T3_OK && t < best_t) {
                best_t = t;
                best = c;
            }
        };
        const double factors[3] = {0.6, 1.0, 1.6};
        for (int mode = 0; mode < 2; ++mode)
            for (double f : factors) {
                TuneChoice c = best;
                c.cell = f * auto_side;
                c.mode = mode;
                consider(c);
            }
        if (!(keep_flags & T3_FLAG_NO_LANE)) {
            // at most 128 expected neighbours: the bound of the FP32 lane sums
            for (double lane : {0.0, 64.0, 128.0}) {
                TuneChoice c = best;
                c.lane = lane;
                if (c.lane != best.lane) consider(c);
            }
        }
        if (plan->B <= 24) {
            TuneChoice c = best;
            c.tile = 1 - best.tile;
            consider(c);
        }
        if (keep.chunk <= 0) {
            // a capacity at or above the sample's centres per catalog runs the
            // sample as one chunk, like the automatic one: such candidates
            // cannot be told apart on the sample and are not tried
            ChunkLayout L = layout_of(plan);
            const int k_auto = choose_chunk(plan, L);
            int64_t most = 0;
            for (int z = 0; z < n_z; ++z) most = std::max<int64_t>(most, cnt[z]);
            for (int div : {2, 4}) {
                TuneChoice c = best;
                c.chunk = std::max(256, (k_auto / div) & ~255);
                if ((int64_t)c.chunk >= most) continue;
                consider(c);
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        plan->flags = keep_flags;
        if (rc != T3_OK) {
            apply_choice(plan, keep);
            return rc;
        }
        apply_choice(plan, best);
        {
            std::lock_guard<std::mutex> lk(mu);
            cache[key] = best;
        }
        if (best_ms) *best_ms = best_t;
        return T3_OK;
    } catch (...) {
        return fail(T3_EINVAL, "t3_autotune: exception");
    }
}

int t3_plan_settings(const t3_plan *plan, double *cell_arcmin, int32_t *scan_mode, double *lane_neighbours,
                     int32_t *tile_mode, int32_t *chunk_centres)
{
    if (!plan) return fail(T3_EINVAL, "t3_plan_settings: null plan");
    if (cell_arcmin) *cell_arcmin = plan->cell_arcmin;
    if (scan_mode) *scan_mode = plan->scan_mode;
    if (lane_neighbours) *lane_neighbours = plan->lane_neighbours;
    if (tile_mode) *tile_mode = plan->tile_mode;
    if (chunk_centres) *chunk_centres = plan->chunk_req;
    return T3_OK;
}

int t3_graph_stats(const t3_plan *plan, int64_t *captures, int64_t *launches)
{
    if (!plan) return fail(T3_EINVAL, "t3_graph_stats: null plan");
    if (captures) *captures = plan->graph_captures;
    if (launches) *launches = plan->graph_replays;
    return T3_OK;
}

int t3_workspace_bytes(const t3_plan *plan, int64_t *in_use, int64_t *peak)
{
    if (!plan) return fail(T3_EINVAL, "t3_workspace_bytes: null plan");
    if (in_use) *in_use = plan->budget.used;
    if (peak) *peak = plan->budget.peak;
    return T3_OK;
}

int t3_stage_times(const t3_plan *plan, double *ms, int64_t *launches)
{
    if (!plan || !ms) return fail(T3_EINVAL, "t3_stage_times: null argument");
    if (!(plan->flags & T3_FLAG_TIMING)) return fail(T3_EINVAL, "t3_stage_times: plan has no timing flag");
    for (int i = 0; i < 4; ++i) {
        ms[i] = plan->stage_ms[i];
        if (launches) launches[i] = plan->stage_launches[i];
    }
    return T3_OK;
}

int t3_backward(t3_plan *plan, const t3_catalog *cat, const int32_t *centres, int64_t n_centres,
                const double *grad_ups, float *grad_g1, float *grad_g2, float *grad_w, void *stream)
{
    try {
        if (!plan || !grad_ups || !grad_g1 || !grad_g2 || !grad_w)
            return fail(T3_EINVAL, "t3_backward: null argument");
        BudgetScope budget_scope(&plan->budget);
        if (plan->flags & T3_FLAG_EDGE_CORRECT)
            return fail(T3_EINVAL, "t3_backward: no adjoint for plans with T3_FLAG_EDGE_CORRECT");
        T3_TRY(check_catalog(cat, "t3_backward"));
        if (n_centres < 0 && centres)
            return fail(T3_EINVAL, "t3_backward: n_centres < 0 (all galaxies) needs centres == NULL");
        if (n_centres > 0 && !centres) return fail(T3_EINVAL, "t3_backward: null centre list");
        if (n_centres > (int64_t)0x7fffffff) return fail(T3_EINVAL, "t3_backward: bad centre count");
        return backward(plan, *cat, centres, n_centres, grad_ups, grad_g1, grad_g2, grad_w, (hipStream_t)stream);
    } catch (...) {
        return fail(T3_EINVAL, "t3_backward: exception");
    }
}

}  // extern "C"
