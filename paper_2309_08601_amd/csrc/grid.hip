// Grid-based and combined multipole estimators (Porth et al. 2023,
// Sect. 3.2 and 3.3, Appendix A).
//
// Every radial bin has a level: 0 = discrete (galaxy pairs), l >= 1 = a grid
// of square pixels of side Delta_1 2^(l-1) lattice steps anchored at the plan
// box corner (nested resolutions).  For each grid level:
//  1. pixelisation: the galaxies are counting-sorted by pixel (the cell-list
//     builder with cell = pixel); every non-empty pixel gets the FP64 sums
//     of w gamma and w of its galaxies (summed in the sorted order, so the
//     result is deterministic) and its lower-left corner as position (only
//     differences of positions enter, so corners and centres are the same);
//  2. G_m^Delta, W_m^Delta and the j = k sums of the level's bins at every
//     non-empty pixel, i.e. the convolution of the gridded w gamma and w with
//     the bin kernels e^{i m phi} 1(theta in Theta), by one of two routes:
//     the stage-1 pair sums run on the pixel catalog (visits non-empty
//     pixels only), or FFTs on the dense grid of the occupied pixels
//     (fft.hip); a cost model picks one per level unless the caller does.
// Then, per chunk of galaxy centres: stage 1 for the discrete bins, a gather
// that copies every grid bin's planes from the pixel holding the galaxy,
// and the ordinary stage 2 over galaxies.  A sum over galaxies of
// c_i X(i; b1) Y(i; b2) with a grid bin's harmonics taken at the galaxy's
// pixel equals the regridded form of eq. (CombinedEstimatorRegridding): the
// finer side's products summed into the coarser pixel and contracted with
// the coarse harmonics; for two bins of one level it is the grid estimator
// (eq. UpsilonmuGrid) with the pixel factor c_P = sum of its galaxies' c.
// The j = k sums of a grid bin are those of the pixel catalog (degenerate
// pairs of one neighbour pixel), taken with the centre factor of each galaxy,
// whose sum over a pixel is the pixel's factor.
#include "t3_internal.h"

#include <algorithm>
#include <cmath>

namespace t3 {

void GridLevel::release()
{
    for (SortedCatalog *sc : {&by_pix, &pix}) {
        sc->pos.release();
        sc->cw.release();
        sc->cell_start.release();
        sc->perm.release();
        sc->keys.release();
        sc->counts.release();
        sc->scan_tmp.release();
    }
    pix_id.release();
    pix_xy.release();
    pix_sum.release();
    pix_gw.release();
    gal_pix.release();
    pix_centres.pos.release();
    pix_centres.cw.release();
    slot_of_pix.release();
    cen_slot.release();
    planes.release();
    fft_misc.release();
    fft_buf.release();
    fft_spec.release();
    for (auto &k : spec_key) k = -1;
}

namespace {

inline unsigned blocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// AUTO route: pixel weight peak-to-mean above which a level keeps the pair sums
constexpr double kFftPeakRatio = 100.0;

// 1 for non-empty cells, 0 for empty ones and for the extra entry [ncells]
__global__ void k_pix_flags(const int *__restrict__ start, int64_t ncells, int *__restrict__ flags)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > ncells) return;
    flags[c] = c < ncells && start[c + 1] > start[c] ? 1 : 0;
}

struct PixArgs {
    const int *start;     // cell_start of the galaxies sorted by pixel
    const int *perm;      // sorted slot -> galaxy
    const int *pix_id;    // exclusive scan of the non-empty flags
    int64_t ncells;
    CellGrid g;           // cell = pixel
    const float *g1, *g2, *w;  // input catalog
    int32_t *px, *py;
    double *sum;          // [n_pix][3]
    float *fg1, *fg2, *fw;
    int *gal_pix;
};

// One thread per cell: sums over the pixel's galaxies in FP64 (products of
// the FP32 inputs are exact in FP64), corner position, galaxy -> pixel.
__global__ void k_pix_build(PixArgs a)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.ncells) return;
    const int lo = a.start[c], hi = a.start[c + 1];
    if (lo == hi) return;
    const int P = a.pix_id[c];
    double s1 = 0.0, s2 = 0.0, sw = 0.0;
    for (int k = lo; k < hi; ++k) {
        const int i = a.perm[k];
        const double wi = (double)a.w[i];
        s1 += wi * (double)a.g1[i];
        s2 += wi * (double)a.g2[i];
        sw += wi;
        a.gal_pix[i] = P;
    }
    const int64_t cx = c % a.g.ncx, cy = c / a.g.ncx;
    a.px[P] = (int32_t)((int64_t)a.g.ox + cx * a.g.cell);
    a.py[P] = (int32_t)((int64_t)a.g.oy + cy * a.g.cell);
    a.sum[3 * (int64_t)P] = s1;
    a.sum[3 * (int64_t)P + 1] = s2;
    a.sum[3 * (int64_t)P + 2] = sw;
    a.fg1[P] = sw != 0.0 ? (float)(s1 / sw) : 0.0f;
    a.fg2[P] = sw != 0.0 ? (float)(s2 / sw) : 0.0f;
    a.fw[P] = (float)sw;
}

// Factors of the cell-sorted pixel catalog from the FP64 sums (one rounding).
__global__ void k_pix_factors(const int *__restrict__ perm, int64_t n, const double *__restrict__ sum,
                              float4 *__restrict__ cw, int *__restrict__ slot_of_pix)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int P = perm[s];
    cw[s] = make_float4((float)sum[3 * (int64_t)P], (float)sum[3 * (int64_t)P + 1],
                        (float)sum[3 * (int64_t)P + 2], 0.0f);
    slot_of_pix[P] = (int)s;
}

// Galaxy centre (sorted slot of the main catalog) -> plane slot of its pixel
// (slot_of_pix null: the pixel index itself).
__global__ void k_cen_slot(const int *__restrict__ perm, int64_t n, const int *__restrict__ gal_pix,
                           const int *__restrict__ slot_of_pix, int *__restrict__ out)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int P = gal_pix[perm[g]];
    out[g] = slot_of_pix ? slot_of_pix[P] : P;
}

// Copy the planes of one level's bins from each centre's pixel into the
// chunk layout.  One thread per (centre quad, bin) and group of
// kGatherPlanes planes (grid.y): the four centres' pixel offsets are found
// once, then each plane takes four gathered loads and one 16-byte store
// (threads in output order, so the stores of a wavefront are contiguous per
// quad).
constexpr int kGatherPlanes = 8;

struct GatherArgs {
    const float *src;     // pixel planes, layout (Kp, nb)
    float *dst;           // chunk planes, layout (K, B)
    const int *slot;      // [n_c] sorted pixel slot of each centre of the chunk
    int n_c, K, B, Kp, nb, b_lo, n_planes;
};

__global__ void k_grid_gather(GatherArgs a)
{
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned nb = (unsigned)a.nb;
    if (t >= (unsigned)(a.K >> 2) * nb) return;
    const int bb = (int)(t % nb);
    const int q = (int)(t / nb);
    const int i0 = 4 * q;
    if (i0 >= a.n_c) return;
    const int nv = min(4, a.n_c - i0);
    size_t so[4];  // offset of (pixel, bin bb) in a pixel plane
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int sl = a.slot[min(i0 + r, a.n_c - 1)];
        so[r] = ((size_t)(sl >> 2) * nb + bb) * 4 + (sl & 3);
    }
    const size_t sp = (size_t)(a.Kp >> 2) * nb * 4;  // floats per pixel plane
    const size_t dp = (size_t)(a.K >> 2) * a.B * 4;  // floats per chunk plane
    const size_t d0 = ((size_t)q * a.B + a.b_lo + bb) * 4;
    const int p0 = (int)blockIdx.y * kGatherPlanes, p1 = min(p0 + kGatherPlanes, a.n_planes);
#pragma unroll 4
    for (int p = p0; p < p1; ++p) {
        const float *src = a.src + (size_t)p * sp;
        float *dst = a.dst + (size_t)p * dp + d0;
        const float4 v = make_float4(src[so[0]], src[so[1]], src[so[2]], src[so[3]]);
        if (nv == 4) {
            *reinterpret_cast<float4 *>(dst) = v;
        } else {
            dst[0] = v.x;
            if (nv > 1) dst[1] = v.y;
            if (nv > 2) dst[2] = v.z;
        }
    }
}

int prepare_counters(t3_plan *plan, hipStream_t s)
{
    T3_TRY(plan->flag.reserve(sizeof(int) * 4));
    T3_TRY(plan->counter.reserve(sizeof(unsigned long long) * 4));
    T3_HIP_CHECK(hipMemsetAsync(plan->flag.ptr, 0, sizeof(int) * 4, s));
    T3_HIP_CHECK(hipMemsetAsync(plan->counter.ptr, 0, sizeof(unsigned long long) * 4, s));
    return T3_OK;
}

// Pixel catalog of one level and the stage-1 planes of its bins at every pixel.
int build_level(t3_plan *plan, GridLevel &lv, const t3_catalog &cat, int method, hipStream_t s)
{
    CellGrid pg;
    pg.cell = (int)lv.side;
    pg.ncx = pg.ncy = (int)((plan->box_size + lv.side - 1) / lv.side);
    pg.ox = plan->box_lo_x;
    pg.oy = plan->box_lo_y;
    const int64_t nc = pg.ncells();
    T3_TRY(build_cells(plan, lv.by_pix, cat, pg, s));
    T3_TRY(lv.pix_id.reserve(sizeof(int) * (size_t)(nc + 1)));
    hipLaunchKernelGGL(k_pix_flags, dim3(blocks(nc + 1, 256)), dim3(256), 0, s,
                       (const int *)lv.by_pix.cell_start.as<int>(), nc, lv.pix_id.as<int>());
    T3_HIP_CHECK(hipGetLastError());
    T3_TRY(exclusive_scan(lv.pix_id.as<int>(), nc + 1, lv.by_pix.scan_tmp, s));
    int n_pix = 0;
    T3_HIP_CHECK(hipMemcpyAsync(&n_pix, lv.pix_id.as<int>() + nc, sizeof(int), hipMemcpyDeviceToHost, s));
    T3_HIP_CHECK(hipStreamSynchronize(s));
    lv.n_pix = n_pix;
    const size_t np1 = (size_t)(n_pix > 0 ? n_pix : 1);
    T3_TRY(lv.pix_xy.reserve(sizeof(int32_t) * 2 * np1));
    T3_TRY(lv.pix_sum.reserve(sizeof(double) * 3 * np1));
    T3_TRY(lv.pix_gw.reserve(sizeof(float) * 3 * np1));
    T3_TRY(lv.gal_pix.reserve(sizeof(int) * (size_t)(cat.n > 0 ? cat.n : 1)));
    T3_TRY(lv.slot_of_pix.reserve(sizeof(int) * np1));
    T3_TRY(lv.cen_slot.reserve(sizeof(int) * (size_t)(cat.n > 0 ? cat.n : 1)));
    PixArgs a;
    a.start = lv.by_pix.cell_start.as<int>();
    a.perm = lv.by_pix.perm.as<int>();
    a.pix_id = lv.pix_id.as<int>();
    a.ncells = nc;
    a.g = pg;
    a.g1 = cat.g1;
    a.g2 = cat.g2;
    a.w = cat.w;
    a.px = lv.pix_xy.as<int32_t>();
    a.py = a.px + np1;
    a.sum = lv.pix_sum.as<double>();
    a.fg1 = lv.pix_gw.as<float>();
    a.fg2 = a.fg1 + np1;
    a.fw = a.fg2 + np1;
    a.gal_pix = lv.gal_pix.as<int>();
    if (cat.n > 0) {
        hipLaunchKernelGGL(k_pix_build, dim3(blocks(nc, 256)), dim3(256), 0, s, a);
        T3_HIP_CHECK(hipGetLastError());
    }
    // harmonics of the level's bins at every pixel
    lv.L.n_max = plan->n_max;
    lv.L.w_max = plan->w_max;
    lv.L.B = lv.nb;
    lv.L.K = (int)(((int64_t)n_pix + 255) & ~(int64_t)255);
    if (lv.L.K < 256) lv.L.K = 256;
    if (lv.L.floats() * sizeof(float) > ((size_t)64 << 30))
        return fail(T3_ERANGE, "t3_forward_grid: pixel planes of a level above 64 GiB (coarser Delta_1)");
    T3_TRY(lv.planes.reserve(sizeof(float) * lv.L.floats()));
    lv.method = T3_GRID_DIRECT;
    if (n_pix == 0) return T3_OK;
    // route: pair sums over the pixel catalog, or FFT convolution on the
    // dense grid of the occupied pixels (modelled cost decides for AUTO)
    T3_TRY(level_bbox(lv, a.px, a.py, a.sum, s));
    int m = method;
    if (m == T3_GRID_AUTO) {
        const double area = (double)lv.nx_occ * lv.ny_occ;  // pixels^2
        const double e_lo = std::sqrt(plan->e2[lv.b_lo]) / (double)lv.side;
        const double e_hi = std::sqrt(plan->e2[lv.b_lo + lv.nb]) / (double)lv.side;
        const double pairs = (double)n_pix * (double)n_pix / area * M_PI * (e_hi * e_hi - e_lo * e_lo);
        // measured stage 1: about 7e12 pair-orders per second plus about
        // 7 ns per (centre, bin) of fixed cost (batch, reduction, row set-up)
        const double direct_ms =
            1e3 * pairs * (3.0 * plan->n_max + 4.0) / 7.0e12 + 7e-6 * (double)n_pix * lv.nb;
        m = fft_cost_ms(plan, lv) < direct_ms ? T3_GRID_FFT : T3_GRID_DIRECT;
        // FFT rounding scales with the field's largest values: a pixel far
        // heavier than the mean (strong clustering) keeps the pair sums
        if (lv.w_peak > kFftPeakRatio) m = T3_GRID_DIRECT;
    }
    lv.method = m;
    // the FFT route indexes planes by pixel (row-major over the box: rows of
    // the grid are runs of consecutive pixels); the pair sums sweep the
    // cell-sorted pixel catalog and index planes by its sorted slot
    if (m == T3_GRID_FFT) return fft_level(plan, lv, s);
    const t3_catalog pc{n_pix, a.px, a.py, a.fg1, a.fg2, a.fw};
    T3_TRY(build_cells(plan, lv.pix, pc, choose_grid(plan, n_pix), s));
    hipLaunchKernelGGL(k_pix_factors, dim3(blocks(n_pix, 256)), dim3(256), 0, s, (const int *)lv.pix.perm.as<int>(),
                       (int64_t)n_pix, (const double *)a.sum, lv.pix.cw.as<float4>(), lv.slot_of_pix.as<int>());
    T3_HIP_CHECK(hipGetLastError());
    T3_TRY(gather_sorted_centres(plan, lv.pix, lv.pix_centres, s));
    const SortedCatalog *cl[1] = {&lv.pix};
    T3_TRY(scan_chunk(plan, cl, nullptr, 1, lv.pix_centres, 0, n_pix, lv.L, lv.planes.as<float>(), lv.L.floats(),
                      plan->counter.as<unsigned long long>(), plan->scan_mode, s, lv.b_lo, lv.nb));
    return T3_OK;
}

}  // namespace

int forward_grid(t3_plan *plan, const t3_catalog &cat, int64_t delta, const int32_t *levels, int method,
                 double *ups_out, int64_t *n_pairs, hipStream_t s)
{
    T3_TRY(timing_begin_call(plan));
    T3_TRY(prepare_counters(plan, s));
    if (plan->scan_var < 0) T3_TRY(scan_prepare(plan));
    const int B = plan->B;
    int b_disc = 0;
    while (b_disc < B && levels[b_disc] == 0) ++b_disc;
    for (int l = 1; l <= kMaxGridLevels; ++l) {
        GridLevel &lv = plan->grid[l - 1];
        lv.nb = 0;
        lv.b_lo = 0;
        for (int b = 0; b < B; ++b)
            if (levels[b] == l) {
                if (lv.nb == 0) lv.b_lo = b;
                ++lv.nb;
            }
        lv.side = delta << (l - 1);
    }

    // galaxies: cell list (centres in cell order), then every grid level
    T3_TRY(timing_mark(plan, 0, true, s));
    T3_TRY(build_cells(plan, plan->cats[0], cat, choose_grid(plan, cat.n), s));
    T3_TRY(gather_sorted_centres(plan, plan->cats[0], plan->csets[0], s));
    T3_TRY(check_flag(plan, s, "t3_forward_grid"));
    T3_TRY(timing_mark(plan, 0, false, s));
    T3_TRY(timing_mark(plan, 1, true, s));
    for (int l = 1; l <= kMaxGridLevels; ++l) {
        GridLevel &lv = plan->grid[l - 1];
        if (lv.nb == 0) continue;
        T3_TRY(build_level(plan, lv, cat, method, s));
        if (cat.n > 0) {
            hipLaunchKernelGGL(k_cen_slot, dim3(blocks(cat.n, 256)), dim3(256), 0, s,
                               (const int *)plan->cats[0].perm.as<int>(), cat.n,
                               (const int *)lv.gal_pix.as<int>(),
                               lv.method == T3_GRID_FFT ? nullptr : (const int *)lv.slot_of_pix.as<int>(),
                               lv.cen_slot.as<int>());
            T3_HIP_CHECK(hipGetLastError());
        }
    }
    T3_TRY(timing_mark(plan, 1, false, s));

    ChunkLayout L;
    L.n_max = plan->n_max;
    L.w_max = plan->w_max;
    L.B = B;
    L.K = choose_chunk(plan, L);
    const CentreSet &cs = plan->csets[0];
    if (plan->chunk_req <= 0 && (int64_t)L.K > cs.n) {
        int K = (int)std::min<int64_t>(L.K, (cs.n + 255) & ~(int64_t)255);
        L.K = K < 256 ? 256 : (K & ~255);
    }
    const size_t zstride = L.floats();
    T3_TRY(plan->chunk.reserve(sizeof(float) * zstride));
    T3_TRY(reserve_contract(plan, L, 1));
    const size_t n_out = (size_t)2 * L.out_blocks() * B * B;
    T3_TRY(zero_doubles(ups_out, n_out, s));
    const SortedCatalog *cl[1] = {&plan->cats[0]};
    const bool jk = !(plan->flags & T3_FLAG_KEEP_JK);
    int n_lane = 0;
    T3_TRY(lane_bins(plan, plan->cats[0], 0, b_disc, plan->lane_neighbours, s, &n_lane));
    for (int64_t c0 = 0; c0 < cs.n; c0 += L.K) {
        const int n = (int)((cs.n - c0) < L.K ? (cs.n - c0) : L.K);
        T3_TRY(timing_mark(plan, 1, true, s));
        if (b_disc > 0)
            T3_TRY(scan_chunk(plan, cl, nullptr, 1, cs, c0, n, L, plan->chunk.as<float>(), zstride,
                              plan->counter.as<unsigned long long>(), plan->scan_mode, s, 0, b_disc, n_lane));
        for (int l = 1; l <= kMaxGridLevels; ++l) {
            const GridLevel &lv = plan->grid[l - 1];
            if (lv.nb == 0) continue;
            GatherArgs g;
            g.src = lv.planes.as<float>();
            g.dst = plan->chunk.as<float>();
            g.slot = lv.cen_slot.as<int>() + c0;
            g.n_c = n;
            g.K = L.K;
            g.B = B;
            g.Kp = lv.L.K;
            g.nb = lv.nb;
            g.b_lo = lv.b_lo;
            g.n_planes = L.n_planes();
            const size_t per_group = (size_t)(L.K >> 2) * g.nb;
            hipLaunchKernelGGL(k_grid_gather,
                               dim3((unsigned)((per_group + 255) / 256),
                                    (unsigned)((g.n_planes + kGatherPlanes - 1) / kGatherPlanes)),
                               dim3(256), 0, s, g);
            T3_HIP_CHECK(hipGetLastError());
        }
        T3_TRY(timing_mark(plan, 1, false, s));
        T3_TRY(timing_mark(plan, 2, true, s));
        T3_TRY(contract_chunk(plan, cs, c0, n, L, plan->chunk.as<float>(), zstride, 1, jk, ups_out, s));
        T3_TRY(timing_mark(plan, 2, false, s));
    }
    unsigned long long pairs = 0;
    T3_HIP_CHECK(hipMemcpyAsync(&pairs, plan->counter.ptr, sizeof(pairs), hipMemcpyDeviceToHost, s));
    T3_HIP_CHECK(hipStreamSynchronize(s));
    T3_TRY(timing_end_call(plan));
    if (n_pairs) *n_pairs = (int64_t)pairs;
    return T3_OK;
}

}  // namespace t3
