// Spatial hash (cell list) for the neighbour search of the multipole
// estimator: a counting sort of the catalog by cell, row-major cells, so that
// any run of cells along one row is one contiguous range of galaxies.  The
// paper uses spatial hashing for O(1) neighbour lookup (Sect. 3.1, complexity
// paragraph); this is its GPU form.  Within a cell galaxies keep their
// original order, so the result is deterministic.
#include "t3_internal.h"

namespace t3 {
namespace {

constexpr int kScanBlock = 1024;

__global__ void k_cell_keys(const int32_t *__restrict__ x, const int32_t *__restrict__ y,
                            int64_t n, CellGrid g, int64_t box_size, int *__restrict__ keys,
                            int *__restrict__ counts, int *__restrict__ flag)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t rx = (int64_t)x[i] - g.ox;
    int64_t ry = (int64_t)y[i] - g.oy;
    if (rx < 0 || ry < 0 || rx >= box_size || ry >= box_size) {
        atomicOr(flag, 1);
        rx = rx < 0 ? 0 : (rx >= box_size ? box_size - 1 : rx);
        ry = ry < 0 ? 0 : (ry >= box_size ? box_size - 1 : ry);
    }
    int cx = (int)(rx / g.cell);
    int cy = (int)(ry / g.cell);
    cx = cx >= g.ncx ? g.ncx - 1 : cx;
    cy = cy >= g.ncy ? g.ncy - 1 : cy;
    int key = cy * g.ncx + cx;
    keys[i] = key;
    atomicAdd(&counts[key], 1);
}

// Exclusive scan, phase 1: per-block scan in place, block totals out.
__global__ __launch_bounds__(kScanBlock) void k_scan_block(int *__restrict__ data, int64_t n,
                                                           int *__restrict__ block_sums)
{
    __shared__ int s[kScanBlock];
    int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    int v = i < n ? data[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        int t = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) data[i] = s[threadIdx.x] - v;
    if (threadIdx.x == kScanBlock - 1) block_sums[blockIdx.x] = s[threadIdx.x];
}

// Phase 2: exclusive scan of the block totals by one block.
__global__ __launch_bounds__(kScanBlock) void k_scan_sums(int *__restrict__ sums, int nb)
{
    __shared__ int s[kScanBlock];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += kScanBlock) {
        int i = base + threadIdx.x;
        int v = i < nb ? sums[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kScanBlock; off <<= 1) {
            int t = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) sums[i] = s[threadIdx.x] - v + carry;
        __syncthreads();
        if (threadIdx.x == kScanBlock - 1) carry += s[threadIdx.x];
        __syncthreads();
    }
}

__global__ void k_scan_add(int *__restrict__ data, int64_t n, const int *__restrict__ sums)
{
    int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    if (i < n) data[i] += sums[blockIdx.x];
}

// Scatter: slot = start[key] + running count (order within a cell is fixed
// afterwards by k_sort_cells).
__global__ void k_scatter(const int *__restrict__ keys, int64_t n, const int *__restrict__ start,
                          int *__restrict__ fill, int *__restrict__ perm)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int k = keys[i];
    int slot = start[k] + atomicAdd(&fill[k], 1);
    perm[slot] = (int)i;
}

// Insertion sort of each cell's (short) index list: deterministic order.
__global__ void k_sort_cells(const int *__restrict__ start, int64_t ncells, int *__restrict__ perm)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    int a = start[c], b = start[c + 1];
    for (int i = a + 1; i < b; ++i) {
        int v = perm[i];
        int j = i - 1;
        while (j >= a && perm[j] > v) {
            perm[j + 1] = perm[j];
            --j;
        }
        perm[j + 1] = v;
    }
}

__global__ void k_gather_sorted(const int *__restrict__ perm, int64_t n, const int32_t *__restrict__ x,
                                const int32_t *__restrict__ y, const float *__restrict__ g1,
                                const float *__restrict__ g2, const float *__restrict__ w,
                                int2 *__restrict__ pos, float4 *__restrict__ cw)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int i = perm[s];
    float wi = w[i];
    pos[s] = make_int2(x[i], y[i]);
    cw[s] = make_float4(wi * g1[i], wi * g2[i], wi, 0.0f);
}

__global__ void k_gather_centres(const int32_t *__restrict__ idx, int64_t n, int64_t n_cat,
                                 const int32_t *__restrict__ x, const int32_t *__restrict__ y,
                                 const float *__restrict__ g1, const float *__restrict__ g2,
                                 const float *__restrict__ w, int2 *__restrict__ pos,
                                 float4 *__restrict__ cw, int *__restrict__ flag)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int64_t i = idx[s];
    if (i < 0 || i >= n_cat) {
        atomicOr(flag, 2);
        pos[s] = make_int2(0, 0);
        cw[s] = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    float wi = w[i];
    pos[s] = make_int2(x[i], y[i]);
    cw[s] = make_float4(wi * g1[i], wi * g2[i], wi, 0.0f);
}

__global__ void k_fill_int(int *__restrict__ p, int64_t n, int v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int fill_int(int *p, int64_t n, int v, hipStream_t s)
{
    if (n <= 0) return T3_OK;
    hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
    T3_HIP_CHECK(hipGetLastError());
    return T3_OK;
}

// Exclusive scan of data[0..n) in place (n <= 2^30).
int exclusive_scan(int *data, int64_t n, DevBuf &tmp, hipStream_t s)
{
    int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    T3_TRY(tmp.reserve(sizeof(int) * (size_t)(nb + 1)));
    hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(kScanBlock), 0, s, data, n,
                       tmp.as<int>());
    T3_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, s, tmp.as<int>(), (int)nb);
    T3_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanBlock), 0, s, data, n,
                       (const int *)tmp.as<int>());
    T3_HIP_CHECK(hipGetLastError());
    return T3_OK;
}

size_t cells_arena_bytes(int64_t n, const CellGrid &g)
{
    const int64_t nc = g.ncells();
    const size_t m = (size_t)(n > 0 ? n : 1);
    const int64_t nb = (nc + 1 + kScanBlock - 1) / kScanBlock;
    return 2 * arena_bytes(sizeof(int) * (size_t)(nc + 1))                       // cell starts, counts
           + arena_bytes(sizeof(int2) * m) + arena_bytes(sizeof(float4) * m)      // sorted positions, factors
           + 2 * arena_bytes(sizeof(int) * m)                                     // permutation, keys
           + arena_bytes(sizeof(int) * (size_t)(nb + 1));                         // block sums of the scan
}

CellGrid choose_grid(const t3_plan *plan, int64_t n_gal)
{
    CellGrid g;
    double side_lat;
    if (plan->cell_arcmin > 0) {
        side_lat = plan->cell_arcmin / plan->unit;
    } else {
        // about 8 galaxies per cell on average, never finer than 1/256 of the
        // largest separation, never more than 2^22 cells
        double area = (double)plan->box_size * (double)plan->box_size;
        double per = n_gal > 0 ? area / (double)n_gal : area;
        side_lat = sqrt(8.0 * per);
        side_lat = fmax(side_lat, plan->edges_lat.back() / 256.0);
    }
    double min_side = (double)plan->box_size / 2048.0;
    side_lat = fmax(side_lat, fmax(min_side, 1.0));
    side_lat = fmin(side_lat, (double)plan->box_size);
    g.cell = (int)fmin(side_lat, 1073741823.0);
    if (g.cell < 1) g.cell = 1;
    g.ncx = (int)((plan->box_size + g.cell - 1) / g.cell);
    g.ncy = g.ncx;
    g.ox = plan->box_lo_x;
    g.oy = plan->box_lo_y;
    return g;
}

int build_cells(t3_plan *plan, SortedCatalog &sc, const t3_catalog &cat, const CellGrid &g,
                hipStream_t s)
{
    ++plan->cells_seq;  // invalidates planes kept by an earlier forward
    sc.n = cat.n;
    sc.grid = g;
    const int64_t n = cat.n;
    const int64_t nc = g.ncells();
    T3_TRY(sc.cell_start.reserve(sizeof(int) * (size_t)(nc + 1)));
    T3_TRY(sc.counts.reserve(sizeof(int) * (size_t)(nc + 1)));
    T3_TRY(sc.pos.reserve(sizeof(int2) * (size_t)(n > 0 ? n : 1)));
    T3_TRY(sc.cw.reserve(sizeof(float4) * (size_t)(n > 0 ? n : 1)));
    T3_TRY(sc.perm.reserve(sizeof(int) * (size_t)(n > 0 ? n : 1)));
    T3_TRY(sc.keys.reserve(sizeof(int) * (size_t)(n > 0 ? n : 1)));
    int *start = sc.cell_start.as<int>();
    int *counts = sc.counts.as<int>();
    T3_TRY(fill_int(start, nc + 1, 0, s));
    if (n > 0) {
        hipLaunchKernelGGL(k_cell_keys, dim3(blocks_for(n, 256)), dim3(256), 0, s, cat.x, cat.y, n,
                           g, plan->box_size, sc.keys.as<int>(), start, plan->flag.as<int>());
        T3_HIP_CHECK(hipGetLastError());
    }
    T3_TRY(exclusive_scan(start, nc + 1, sc.scan_tmp, s));
    if (n > 0) {
        T3_TRY(fill_int(counts, nc, 0, s));
        hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                           (const int *)sc.keys.as<int>(), n, (const int *)start, counts,
                           sc.perm.as<int>());
        T3_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(k_sort_cells, dim3(blocks_for(nc, 256)), dim3(256), 0, s,
                           (const int *)start, nc, sc.perm.as<int>());
        T3_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(k_gather_sorted, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                           (const int *)sc.perm.as<int>(), n, cat.x, cat.y, cat.g1, cat.g2, cat.w,
                           sc.pos.as<int2>(), sc.cw.as<float4>());
        T3_HIP_CHECK(hipGetLastError());
    }
    return T3_OK;
}

namespace {
// number of non-empty cells (one atomic per wavefront)
__global__ void k_count_nonempty(const int *__restrict__ start, int64_t ncells, unsigned *__restrict__ out)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned v = c < ncells && start[c + 1] > start[c] ? 1u : 0u;
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(out, v);
}
}  // namespace

int lane_bins(t3_plan *plan, const SortedCatalog &sc, int b0, int nb, double most, hipStream_t s, int *n_lane)
{
    *n_lane = 0;
    if (sc.n == 0 || nb <= 0 || (plan->flags & T3_FLAG_NO_LANE)) return T3_OK;
    const int64_t nc = sc.grid.ncells();
    T3_TRY(plan->misc2.reserve(sizeof(unsigned) * 4));
    T3_HIP_CHECK(hipMemsetAsync(plan->misc2.ptr, 0, sizeof(unsigned), s));
    hipLaunchKernelGGL(k_count_nonempty, dim3(blocks_for(nc, 256)), dim3(256), 0, s, (const int *)sc.cell_start.as<int>(),
                       nc, plan->misc2.as<unsigned>());
    T3_HIP_CHECK(hipGetLastError());
    unsigned occupied = 0;
    T3_HIP_CHECK(hipMemcpyAsync(&occupied, plan->misc2.ptr, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    T3_HIP_CHECK(hipStreamSynchronize(s));
    if (occupied == 0) return T3_OK;
    // galaxies per lattice step^2 over the occupied cells
    const double density = (double)sc.n / ((double)occupied * (double)sc.grid.cell * (double)sc.grid.cell);
    int k = 0;
    while (k < nb && density * 3.14159265358979323846 * (plan->e2[b0 + k + 1] - plan->e2[b0 + k]) <= most) ++k;
    *n_lane = k;
    return T3_OK;
}

int gather_centres(t3_plan *plan, const t3_catalog &cat, const int32_t *idx, int64_t n,
                   CentreSet &cs, hipStream_t s)
{
    cs.n = n;
    T3_TRY(cs.pos.reserve(sizeof(int2) * (size_t)(n > 0 ? n : 1)));
    T3_TRY(cs.cw.reserve(sizeof(float4) * (size_t)(n > 0 ? n : 1)));
    if (n > 0) {
        hipLaunchKernelGGL(k_gather_centres, dim3(blocks_for(n, 256)), dim3(256), 0, s, idx, n,
                           cat.n, cat.x, cat.y, cat.g1, cat.g2, cat.w, cs.pos.as<int2>(),
                           cs.cw.as<float4>(), plan->flag.as<int>());
        T3_HIP_CHECK(hipGetLastError());
    }
    return T3_OK;
}

int gather_sorted_centres(t3_plan *plan, const SortedCatalog &sc, CentreSet &cs, hipStream_t s)
{
    (void)plan;
    cs.n = sc.n;
    T3_TRY(cs.pos.reserve(sizeof(int2) * (size_t)(sc.n > 0 ? sc.n : 1)));
    T3_TRY(cs.cw.reserve(sizeof(float4) * (size_t)(sc.n > 0 ? sc.n : 1)));
    if (sc.n > 0) {
        T3_HIP_CHECK(hipMemcpyAsync(cs.pos.ptr, sc.pos.ptr, sizeof(int2) * (size_t)sc.n,
                                    hipMemcpyDeviceToDevice, s));
        T3_HIP_CHECK(hipMemcpyAsync(cs.cw.ptr, sc.cw.ptr, sizeof(float4) * (size_t)sc.n,
                                    hipMemcpyDeviceToDevice, s));
    }
    return T3_OK;
}

int check_flag(t3_plan *plan, hipStream_t s, const char *what)
{
    int h = 0;
    T3_HIP_CHECK(hipMemcpyAsync(&h, plan->flag.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
    T3_HIP_CHECK(hipStreamSynchronize(s));
    if (h & 1) return fail(T3_ELATTICE, std::string(what) + ": a position lies outside the plan box");
    if (h & 2) return fail(T3_EINVAL, std::string(what) + ": a centre index is out of range");
    return T3_OK;
}

}  // namespace t3
