// C ABI of the t3pcf library (declared in include/t3pcf.h).
#include <cmath>
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

int DevBuf::reserve(size_t want)
{
    if (want <= bytes && ptr) return T3_OK;
    if (ptr) (void)hipDeviceSynchronize();  // earlier launches may still read the old buffer
    release();
    size_t b = want < 256 ? 256 : want;
    if (hipMalloc(&ptr, b) != hipSuccess) {
        (void)hipGetLastError();
        ptr = nullptr;
        bytes = 0;
        return fail(T3_ENOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
    }
    bytes = b;
    return T3_OK;
}

void DevBuf::release()
{
    if (ptr) (void)hipFree(ptr);
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
        // keep one chunk of planes near 128 MB (resident in the last-level cache)
        const double per_centre = (double)L.n_planes() * L.B * sizeof(float);
        K = (int)(128.0 * 1024 * 1024 / per_centre);
        if (K > 65536) K = 65536;
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
    L.B = plan->B;
    L.K = 0;
    L.K = choose_chunk(plan, L);
    return L;
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
        if (p->n_bins > 32) return fail(T3_ERANGE, "t3_plan_create: at most 32 radial bins");
        if (p->n_max < 0 || p->n_max > 64) return fail(T3_ERANGE, "t3_plan_create: n_max must be in [0, 64]");
        if (p->precision < T3_PREC_FP32 || p->precision > T3_PREC_FP16X3)
            return fail(T3_EINVAL, "t3_plan_create: unknown precision");
        if (p->flags & ~(T3_FLAG_KEEP_JK | T3_FLAG_TIMING))
            return fail(T3_EINVAL, "t3_plan_create: unknown flag");
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

        t3_plan *plan = new (std::nothrow) t3_plan();
        if (!plan) return fail(T3_ENOMEM, "t3_plan_create: host allocation failed");
        plan->B = p->n_bins;
        plan->n_max = p->n_max;
        plan->precision = p->precision;
        plan->flags = p->flags;
        plan->unit = unit;
        plan->box_lo_x = p->box_lo_x;
        plan->box_lo_y = p->box_lo_y;
        plan->box_size = p->box_size;
        plan->cell_arcmin = p->cell_arcmin;
        plan->chunk_req = p->chunk_centres;
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
    plan->partial.release();
    plan->diag.release();
    plan->flag.release();
    plan->dest.release();
    plan->scales.release();
    plan->counter.release();
    plan->misc.release();
    plan->misc2.release();
    for (auto e : plan->events) (void)hipEventDestroy(e);
    delete plan;
}

int t3_forward(t3_plan *plan, const t3_catalog *cat, const int32_t *centres, int64_t n_centres,
               double *ups_out, int64_t *n_pairs, void *stream)
{
    try {
        if (!plan || !ups_out) return fail(T3_EINVAL, "t3_forward: null argument");
        T3_TRY(check_catalog(cat, "t3_forward"));
        if (n_centres < 0 && centres)
            return fail(T3_EINVAL, "t3_forward: n_centres < 0 (all galaxies) needs centres == NULL");
        if (n_centres > 0 && !centres) return fail(T3_EINVAL, "t3_forward: null centre list");
        if (n_centres > (int64_t)0x7fffffff) return fail(T3_EINVAL, "t3_forward: bad centre count");
        hipStream_t s = (hipStream_t)stream;
        T3_TRY(timing_begin_call(plan));
        T3_TRY(prepare_small(plan, s));
        SortedCatalog &sc = plan->cats[0];
        T3_TRY(timing_mark(plan, 0, true, s));
        T3_TRY(build_cells(plan, sc, *cat, choose_grid(plan, cat->n), s));
        if (n_centres >= 0) T3_TRY(gather_centres(plan, *cat, centres, n_centres, plan->centres, s));
        else T3_TRY(gather_sorted_centres(plan, sc, plan->centres, s));
        T3_TRY(timing_mark(plan, 0, false, s));
        T3_TRY(check_flag(plan, s, "t3_forward"));
        const ChunkLayout L = layout_of(plan);
        const size_t n_out = (size_t)2 * 5 * (plan->n_max + 1) * plan->B * plan->B;
        T3_TRY(zero_doubles(ups_out, n_out, s));
        T3_TRY(plan->chunk.reserve(sizeof(float) * L.floats()));
        const int64_t nc = plan->centres.n;
        const bool jk = !(plan->flags & T3_FLAG_KEEP_JK);
        for (int64_t c0 = 0; c0 < nc; c0 += L.K) {
            const int n = (int)((nc - c0) < L.K ? (nc - c0) : L.K);
            T3_TRY(timing_mark(plan, 1, true, s));
            T3_TRY(scan_chunk(plan, sc, plan->centres, c0, n, L, plan->chunk.as<float>(),
                              plan->counter.as<unsigned long long>(), s));
            T3_TRY(timing_mark(plan, 1, false, s));
            T3_TRY(timing_mark(plan, 2, true, s));
            T3_TRY(contract_chunk(plan, plan->centres, c0, n, L, plan->chunk.as<float>(),
                                  plan->chunk.as<float>(), jk, ups_out, s));
            T3_TRY(timing_mark(plan, 2, false, s));
        }
        unsigned long long pairs = 0;
        T3_HIP_CHECK(hipMemcpyAsync(&pairs, plan->counter.ptr, sizeof(pairs), hipMemcpyDeviceToHost, s));
        T3_HIP_CHECK(hipStreamSynchronize(s));
        T3_TRY(timing_end_call(plan));
        if (n_pairs) *n_pairs = (int64_t)pairs;
        return T3_OK;
    } catch (...) {
        return fail(T3_EINVAL, "t3_forward: exception");
    }
}

int t3_forward_tomo(t3_plan *plan, const t3_catalog *cats, int32_t n_z, const int32_t *const *centres,
                    const int64_t *n_centres, double *ups_out, int64_t *n_pairs, void *stream)
{
    try {
        if (!plan || !cats || !ups_out) return fail(T3_EINVAL, "t3_forward_tomo: null argument");
        if (n_z < 1 || n_z > 8) return fail(T3_ERANGE, "t3_forward_tomo: n_z must be in [1, 8]");
        for (int z = 0; z < n_z; ++z) T3_TRY(check_catalog(&cats[z], "t3_forward_tomo"));
        if (centres && !n_centres) return fail(T3_EINVAL, "t3_forward_tomo: centres without counts");
        hipStream_t s = (hipStream_t)stream;
        T3_TRY(timing_begin_call(plan));
        T3_TRY(prepare_small(plan, s));
        int64_t n_all = 0;
        for (int z = 0; z < n_z; ++z) n_all += cats[z].n;
        const CellGrid grid = choose_grid(plan, n_all > 0 ? n_all / n_z : 0);
        T3_TRY(timing_mark(plan, 0, true, s));
        for (int z = 0; z < n_z; ++z) T3_TRY(build_cells(plan, plan->cats[z], cats[z], grid, s));
        T3_TRY(timing_mark(plan, 0, false, s));
        T3_TRY(check_flag(plan, s, "t3_forward_tomo"));
        ChunkLayout L = layout_of(plan);
        // n_z chunk buffers at once: shrink K so that they stay near 128 MB x 2
        if (plan->chunk_req <= 0) {
            int K = L.K / n_z * 2;
            K = K < 256 ? 256 : (K & ~255);
            L.K = K;
        }
        const size_t per_set = (size_t)2 * 5 * (plan->n_max + 1) * plan->B * plan->B;
        T3_TRY(zero_doubles(ups_out, per_set * (size_t)n_z * n_z * n_z, s));
        T3_TRY(plan->chunk.reserve(sizeof(float) * L.floats() * (size_t)n_z));
        float *planes = plan->chunk.as<float>();
        const bool jk = !(plan->flags & T3_FLAG_KEEP_JK);
        for (int z1 = 0; z1 < n_z; ++z1) {
            const int32_t *idx = centres ? centres[z1] : nullptr;
            const int64_t ncz = centres ? n_centres[z1] : -1;
            if (ncz < 0 && idx) return fail(T3_EINVAL, "t3_forward_tomo: count < 0 needs a NULL list");
            if (ncz > 0 && !idx) return fail(T3_EINVAL, "t3_forward_tomo: null centre list");
            if (ncz >= 0) {
                if (ncz > (int64_t)0x7fffffff) return fail(T3_EINVAL, "t3_forward_tomo: bad centre count");
                T3_TRY(gather_centres(plan, cats[z1], idx, ncz, plan->centres, s));
                T3_TRY(check_flag(plan, s, "t3_forward_tomo"));
            } else {
                T3_TRY(gather_sorted_centres(plan, plan->cats[z1], plan->centres, s));
            }
            const int64_t nc = plan->centres.n;
            for (int64_t c0 = 0; c0 < nc; c0 += L.K) {
                const int n = (int)((nc - c0) < L.K ? (nc - c0) : L.K);
                T3_TRY(timing_mark(plan, 1, true, s));
                for (int z = 0; z < n_z; ++z)
                    T3_TRY(scan_chunk(plan, plan->cats[z], plan->centres, c0, n, L,
                                      planes + (size_t)z * L.floats(),
                                      plan->counter.as<unsigned long long>(), s));
                T3_TRY(timing_mark(plan, 1, false, s));
                T3_TRY(timing_mark(plan, 2, true, s));
                for (int z2 = 0; z2 < n_z; ++z2)
                    for (int z3 = 0; z3 < n_z; ++z3) {
                        double *dst = ups_out + per_set * (((size_t)z1 * n_z + z2) * n_z + z3);
                        T3_TRY(contract_chunk(plan, plan->centres, c0, n, L,
                                              planes + (size_t)z2 * L.floats(),
                                              planes + (size_t)z3 * L.floats(), jk && z2 == z3,
                                              dst, s));
                    }
                T3_TRY(timing_mark(plan, 2, false, s));
            }
        }
        unsigned long long pairs = 0;
        T3_HIP_CHECK(hipMemcpyAsync(&pairs, plan->counter.ptr, sizeof(pairs), hipMemcpyDeviceToHost, s));
        T3_HIP_CHECK(hipStreamSynchronize(s));
        T3_TRY(timing_end_call(plan));
        if (n_pairs) *n_pairs = (int64_t)pairs;
        return T3_OK;
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
        T3_TRY(check_catalog(cat, "t3_harmonics"));
        if (n_centres < 0 || n_centres > (int64_t)0x7fffffff)
            return fail(T3_EINVAL, "t3_harmonics: bad centre count");
        hipStream_t s = (hipStream_t)stream;
        T3_TRY(prepare_small(plan, s));
        SortedCatalog &sc = plan->cats[0];
        T3_TRY(build_cells(plan, sc, *cat, choose_grid(plan, cat->n), s));
        T3_TRY(gather_centres(plan, *cat, centres, n_centres, plan->centres, s));
        T3_TRY(check_flag(plan, s, "t3_harmonics"));
        const ChunkLayout L = layout_of(plan);
        T3_TRY(plan->chunk.reserve(sizeof(float) * L.floats()));
        for (int64_t c0 = 0; c0 < n_centres; c0 += L.K) {
            const int n = (int)((n_centres - c0) < L.K ? (n_centres - c0) : L.K);
            T3_TRY(scan_chunk(plan, sc, plan->centres, c0, n, L, plan->chunk.as<float>(),
                              plan->counter.as<unsigned long long>(), s));
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
    if (n_sets < 1) return fail(T3_EINVAL, "t3_normalise_resum: n_sets must be >= 1");
    int n_z = 1;
    while (n_z * n_z * n_z < n_sets) ++n_z;
    if (n_z * n_z * n_z != n_sets) return fail(T3_EINVAL, "t3_normalise_resum: n_sets must be a cube");
    if (gamma_phi && (n_phi < 1 || n_phi > 4096))
        return fail(T3_ERANGE, "t3_normalise_resum: n_phi must be in [1, 4096]");
    return normalise_resum(plan, ups, n_sets, n_z, n_phi, gamma_n, gamma_phi, (hipStream_t)stream);
}

int t3_normalise_backward(t3_plan *plan, const double *ups, int32_t n_sets, const double *grad_gamma_n,
                          double *grad_ups, void *stream)
{
    if (!plan || !ups || !grad_gamma_n || !grad_ups)
        return fail(T3_EINVAL, "t3_normalise_backward: null argument");
    if (n_sets < 1) return fail(T3_EINVAL, "t3_normalise_backward: n_sets must be >= 1");
    return normalise_backward(plan, ups, grad_gamma_n, n_sets, grad_ups, (hipStream_t)stream);
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

int t3_backward(t3_plan *plan, const t3_catalog *cat, const double *grad_ups, float *grad_g1,
                float *grad_g2, float *grad_w, void *stream)
{
    try {
        if (!plan || !grad_ups || !grad_g1 || !grad_g2 || !grad_w)
            return fail(T3_EINVAL, "t3_backward: null argument");
        T3_TRY(check_catalog(cat, "t3_backward"));
        return backward(plan, *cat, grad_ups, grad_g1, grad_g2, grad_w, (hipStream_t)stream);
    } catch (...) {
        return fail(T3_EINVAL, "t3_backward: exception");
    }
}

}  // extern "C"
