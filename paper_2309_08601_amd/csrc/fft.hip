// Grid harmonics by FFT convolution (Porth et al. 2023, Sect. 3.2: the
// G_n^Delta and W_n^Delta of a grid are convolutions of the gridded w gamma
// and w with the bin kernels g_{n;Theta}, computed with FFTs).
//
// One level of the combined estimator: the non-empty pixels' values are
// placed on a dense grid covering the occupied pixels plus a zero margin of
// the largest separation R (in pixels) of the level's bins (R clamped to the
// occupied extent), so that the
// circular convolution equals the linear one on the occupied part; the grid
// sides are products of 2, 3 and 5 (at most 8192).  Fields: c = sum w gamma,
// w, c^2, |c|^2, w^2 (the last three for the j = k sums).  For each bin and
// order m the kernel K(d) = e^{i m phi(d)} [|d| in bin] (d the offset from the
// centre pixel to the neighbour pixel, bin membership from the same FP64
// squared separations as the pair sums) is placed at -d (a correlation),
// transformed, multiplied with each field's spectrum that needs order m, and
// transformed back; the values at the non-empty pixels are written into the
// level's stage-1 planes.
//
// 2-D transforms: rows by a Stockham FFT in LDS (one workgroup per row, radix
// 2, 3, 4, 5 or 8 per stage, twiddles from an FP64-computed table), then a
// tiled transpose, then rows again; the spectrum stays transposed, and the
// inverse runs the same three steps back.  FP32 arithmetic.  Transforms run
// in batches (one launch per step for many fields, orders or outputs, the
// batch index on the grid's y axis) so that the coarse levels' small grids
// still fill the chip.  The kernel spectra depend only on the plan and the
// grid geometry; a level keeps them between calls while those are unchanged.
#include "t3_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace t3 {
namespace {

constexpr int kFftThreads = 256;
constexpr int kFftMax = 8192;   // largest side (64 KiB of LDS per row)
constexpr int kMaxStages = 16;

struct RowPlan {
    int n = 0;                  // transform length
    int ns = 0;                 // stages
    int radix[kMaxStages];
    unsigned magic[kMaxStages]; // ceil(2^32 / sub-transform size) of each stage (size >= 2)
    const float2 *tw = nullptr; // e^{-2 pi i k / n}, k < n
};

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// (s i) z for s = +-1
__device__ __forceinline__ float2 rot_i(float2 z, float s) { return make_float2(-s * z.y, s * z.x); }

// In-register DFT of size R: X_k = sum_j v_j e^{s 2 pi i j k / R} (s = -1
// forward, +1 inverse), written out from the definition.
template <int R> struct Dft;
template <> struct Dft<2> {
    __device__ static void run(float2 *v, float)
    {
        const float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};
template <> struct Dft<3> {
    __device__ static void run(float2 *v, float s)
    {
        const float c = -0.5f, sn = 0.86602540378443864676f;  // cos, sin of 2 pi / 3
        const float2 b = cadd(v[1], v[2]), d = csub(v[1], v[2]);
        const float2 t = make_float2(v[0].x + c * b.x, v[0].y + c * b.y);
        const float2 u = rot_i(cscale(d, sn), s);
        v[0] = cadd(v[0], b);
        v[1] = cadd(t, u);
        v[2] = csub(t, u);
    }
};
template <> struct Dft<4> {
    __device__ static void run(float2 *v, float s)
    {
        const float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
        const float2 a2 = cadd(v[1], v[3]), a3 = rot_i(csub(v[1], v[3]), s);
        v[0] = cadd(a0, a2);
        v[2] = csub(a0, a2);
        v[1] = cadd(a1, a3);
        v[3] = csub(a1, a3);
    }
};
template <> struct Dft<5> {
    __device__ static void run(float2 *v, float s)
    {
        const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;  // cos 2pi/5, 4pi/5
        const float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;   // sin 2pi/5, 4pi/5
        const float2 b1 = cadd(v[1], v[4]), b2 = cadd(v[2], v[3]);
        const float2 d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
        const float2 t1 = make_float2(v[0].x + c1 * b1.x + c2 * b2.x, v[0].y + c1 * b1.y + c2 * b2.y);
        const float2 t2 = make_float2(v[0].x + c2 * b1.x + c1 * b2.x, v[0].y + c2 * b1.y + c1 * b2.y);
        const float2 u1 = rot_i(make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y), s);
        const float2 u2 = rot_i(make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y), s);
        v[0] = cadd(v[0], cadd(b1, b2));
        v[1] = cadd(t1, u1);
        v[4] = csub(t1, u1);
        v[2] = cadd(t2, u2);
        v[3] = csub(t2, u2);
    }
};
template <> struct Dft<8> {
    __device__ static void run(float2 *v, float s)
    {
        float2 e[4] = {v[0], v[2], v[4], v[6]};
        float2 o[4] = {v[1], v[3], v[5], v[7]};
        Dft<4>::run(e, s);
        Dft<4>::run(o, s);
        const float h = 0.70710678118654752440f;
        // o_k times e^{s 2 pi i k / 8}
        o[1] = make_float2(h * (o[1].x - s * o[1].y), h * (o[1].y + s * o[1].x));
        o[2] = rot_i(o[2], s);
        o[3] = make_float2(h * (-o[3].x - s * o[3].y), h * (-o[3].y + s * o[3].x));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = cadd(e[k], o[k]);
            v[k + 4] = csub(e[k], o[k]);
        }
    }
};

// One Stockham stage of radix R over buf[0, n) (sub-transforms of size ns
// so far): butterfly j takes buf[j + r n/R], twiddles by
// e^{s 2 pi i r (j mod ns) / (ns R)}, and writes buf[(j / ns) ns R + j mod ns + r ns].
// Every thread first loads all of its butterflies, then the workgroup
// synchronises and stores (one buffer serves as source and destination).
// j / ns is a multiply-high by ceil(2^32 / ns): exact for j, ns <= 2^13.
template <int R, int NMAX>
__device__ __forceinline__ void stage(float2 *buf, const RowPlan &p, int ns, unsigned magic, float s)
{
    constexpr int MB = (NMAX / R + kFftThreads - 1) / kFftThreads;  // butterflies per thread
    const int nb = p.n / R;
    float2 v[MB][R];
#pragma unroll
    for (int q = 0; q < MB; ++q) {
        const int j = threadIdx.x + q * kFftThreads;
        if (j < nb) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[j + r * nb];
        }
    }
    __syncthreads();
    const int tw_step = p.n / (ns * R);
#pragma unroll
    for (int q = 0; q < MB; ++q) {
        const int j = threadIdx.x + q * kFftThreads;
        if (j < nb) {
            const int jq = ns == 1 ? j : (int)__umulhi((unsigned)j, magic);
            const int k = j - jq * ns;
            if (k != 0) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 w = p.tw[r * k * tw_step];
                    w.y *= -s;  // table holds e^{-2 pi i t / n}; s = +1 conjugates
                    v[q][r] = cmul(v[q][r], w);
                }
            }
            Dft<R>::run(v[q], s);
            const int base = jq * ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[base + r * ns] = v[q][r];
        }
    }
    __syncthreads();
}

// NMAX: largest row length of the instantiation (sizes the per-thread
// butterfly registers: rows up to 1024 or 4096 points keep fewer registers
// live than 8192-point rows, so more wavefronts fit per SIMD)
template <int NMAX>
__device__ void fft_lds(float2 *buf, const RowPlan &p, float s)
{
    int ns = 1;
    for (int st = 0; st < p.ns; ++st) {
        const int R = p.radix[st];
        const unsigned mg = p.magic[st];
        switch (R) {
            case 2: stage<2, NMAX>(buf, p, ns, mg, s); break;
            case 3: stage<3, NMAX>(buf, p, ns, mg, s); break;
            case 4: stage<4, NMAX>(buf, p, ns, mg, s); break;
            case 5: stage<5, NMAX>(buf, p, ns, mg, s); break;
            default: stage<8, NMAX>(buf, p, ns, mg, s); break;
        }
        ns *= R;
    }
}

// ---------------------------------------------------------------- loaders / storers
// (batch index t = blockIdx.y; grids of one batch entry are `stride` apart)
struct LoadGrid {
    const float2 *src;
    size_t stride;
    __device__ float2 operator()(int t, int row, int i, int n) const
    {
        return src[t * stride + (size_t)row * n + i];
    }
};
// Spectrum of field f[job] times kernel spectrum k[job].
struct LoadProduct {
    const float2 *F, *K;
    size_t stride;
    const int *f, *k;
    int job0;
    __device__ float2 operator()(int t, int row, int i, int n) const
    {
        const size_t o = (size_t)row * n + i;
        return cmul(F[(size_t)f[job0 + t] * stride + o], K[(size_t)k[job0 + t] * stride + o]);
    }
};
// Kernel of order m0 + t and bin [e2lo, e2hi) on a grid of nx x ny pixels of
// side `side` lattice steps; grid point (x, y) holds K(-signed(x), -signed(y)).
struct LoadKernel {
    int nx, ny, rx, ry, m0;
    double side, e2lo, e2hi;
    __device__ float2 operator()(int t, int row, int i, int) const
    {
        const int m = m0 + t;
        const int sx = i <= nx / 2 ? i : i - nx;
        const int sy = row <= ny / 2 ? row : row - ny;
        const int dx = -sx, dy = -sy;
        if (dx > rx || dx < -rx || dy > ry || dy < -ry) return make_float2(0.f, 0.f);
        const double ddx = (double)dx * side, ddy = (double)dy * side;
        const double r2 = fma(ddx, ddx, ddy * ddy);
        if (!(r2 >= e2lo && r2 < e2hi)) return make_float2(0.f, 0.f);
        const double r = sqrt((double)dx * dx + (double)dy * dy);
        double zr = dx / r, zi = m < 0 ? -dy / r : dy / r;
        double pr = 1.0, pi = 0.0;
        for (int e = m < 0 ? -m : m; e > 0; e >>= 1) {  // z^|m| by squaring, FP64
            if (e & 1) {
                const double u = pr * zr - pi * zi;
                pi = pr * zi + pi * zr;
                pr = u;
            }
            const double u = zr * zr - zi * zi;
            zi = 2.0 * zr * zi;
            zr = u;
        }
        return make_float2((float)pr, (float)pi);
    }
};
struct StoreGrid {
    float2 *dst;
    size_t stride;
    __device__ void operator()(int t, int row, int i, int n, float2 v) const
    {
        dst[t * stride + (size_t)row * n + i] = v;
    }
};
// Values at the non-empty pixels into stage-1 planes (layout K, nb) of
// local bin b: planes re[job], im[job] (im < 0: real part only).
struct StorePlanes {
    const int *slot;   // [ny_occ][nx_occ] pixel index or -1
    int nx_occ, ny_occ;
    float *planes;
    const int *p_re, *p_im;
    int job0, K, nb, b;
    float scale;
    __device__ void operator()(int t, int row, int i, int, float2 v) const
    {
        if (row >= ny_occ || i >= nx_occ) return;
        const int sl = slot[(size_t)row * nx_occ + i];
        if (sl < 0) return;
        const int pr = p_re[job0 + t], pi = p_im[job0 + t];
        planes[chunk_offset(pr, sl, b, K, nb)] = v.x * scale;
        if (pi >= 0) planes[chunk_offset(pi, sl, b, K, nb)] = v.y * scale;
    }
};

// One workgroup per (row, batch entry): load, transform in LDS, store.
// Blocks x >= row_gap skip gap_len rows (kernel generation touches only the
// rows that can be non-zero).
template <int NMAX, class Load, class Store>
__global__ __launch_bounds__(kFftThreads) void k_fft_rows(RowPlan p, float s, Load ld, Store st, int row_gap,
                                                          int gap_len)
{
    extern __shared__ float2 lds[];
    int row = (int)blockIdx.x;
    if (gap_len > 0 && row >= row_gap) row += gap_len;
    const int t = (int)blockIdx.y;
    for (int i = threadIdx.x; i < p.n; i += kFftThreads) lds[i] = ld(t, row, i, p.n);
    __syncthreads();
    fft_lds<NMAX>(lds, p, s);
    for (int i = threadIdx.x; i < p.n; i += kFftThreads) st(t, row, i, p.n, lds[i]);
}

// dst[z][c][r] = src[z][r][c] for grids of rows x cols, `stride` apart
constexpr int kTile = 32;
__global__ __launch_bounds__(256) void k_transpose(const float2 *__restrict__ src, float2 *__restrict__ dst,
                                                   int rows, int cols, size_t stride)
{
    __shared__ float2 t[kTile][kTile + 1];
    src += blockIdx.z * stride;
    dst += blockIdx.z * stride;
    const int c0 = blockIdx.x * kTile, r0 = blockIdx.y * kTile;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int k = ty; k < kTile; k += 8) {
        const int r = r0 + k, c = c0 + tx;
        if (r < rows && c < cols) t[k][tx] = src[(size_t)r * cols + c];
    }
    __syncthreads();
    for (int k = ty; k < kTile; k += 8) {
        const int c = c0 + k, r = r0 + tx;
        if (r < rows && c < cols) dst[(size_t)c * rows + r] = t[tx][k];
    }
}

__global__ void k_zero_c(float2 *p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = make_float2(0.f, 0.f);
}

// occupied pixel range (min/max corner) and the largest and total pixel
// weight: wave reduction, then a workgroup reduction in LDS, then one set of
// atomics per workgroup (weights >= 0, so their bit patterns order like the
// values)
constexpr int kBoxBlock = 1024;
__global__ __launch_bounds__(kBoxBlock) void k_bbox(const int32_t *__restrict__ px, const int32_t *__restrict__ py,
                                                    const double *__restrict__ sum, int64_t n, int *__restrict__ box,
                                                    float *__restrict__ wsum)
{
    __shared__ int s_i[kBoxBlock / 64][5];
    __shared__ float s_w[kBoxBlock / 64];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int x0 = 0x7fffffff, y0 = 0x7fffffff, x1 = (int)0x80000000, y1 = (int)0x80000000;
    float w = 0.0f;
    if (i < n) {
        x0 = x1 = px[i];
        y0 = y1 = py[i];
        w = fmaxf((float)sum[3 * i + 2], 0.0f);
    }
    float wmax = w;
    for (int d = 32; d > 0; d >>= 1) {
        x0 = min(x0, __shfl_xor(x0, d, 64));
        y0 = min(y0, __shfl_xor(y0, d, 64));
        x1 = max(x1, __shfl_xor(x1, d, 64));
        y1 = max(y1, __shfl_xor(y1, d, 64));
        wmax = fmaxf(wmax, __shfl_xor(wmax, d, 64));
        w += __shfl_xor(w, d, 64);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_i[wv][0] = x0;
        s_i[wv][1] = y0;
        s_i[wv][2] = x1;
        s_i[wv][3] = y1;
        s_i[wv][4] = __float_as_int(wmax);
        s_w[wv] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kBoxBlock / 64; ++k) {
            s_i[0][0] = min(s_i[0][0], s_i[k][0]);
            s_i[0][1] = min(s_i[0][1], s_i[k][1]);
            s_i[0][2] = max(s_i[0][2], s_i[k][2]);
            s_i[0][3] = max(s_i[0][3], s_i[k][3]);
            s_i[0][4] = max(s_i[0][4], s_i[k][4]);
            s_w[0] += s_w[k];
        }
        atomicMin(&box[0], s_i[0][0]);
        atomicMin(&box[1], s_i[0][1]);
        atomicMax(&box[2], s_i[0][2]);
        atomicMax(&box[3], s_i[0][3]);
        atomicMax(&box[4], s_i[0][4]);
        atomicAdd(wsum, s_w[0]);
    }
}

// five field grids ([ny][nx] complex, N apart) and the slot map (pixel index)
struct ScatterArgs {
    const int32_t *px, *py;  // corners, by pixel index
    const double *sum;       // [pixel][3]
    int64_t n;
    int x0, y0;
    int64_t side;
    int nx, nx_occ;
    size_t N;
    float2 *f;
    int *slot;
};
__global__ void k_scatter_fields(ScatterArgs a)
{
    const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= a.n) return;
    const int x = (int)(((int64_t)a.px[P] - a.x0) / a.side), y = (int)(((int64_t)a.py[P] - a.y0) / a.side);
    const double c1 = a.sum[3 * (int64_t)P], c2 = a.sum[3 * (int64_t)P + 1], w = a.sum[3 * (int64_t)P + 2];
    const size_t o = (size_t)y * a.nx + x;
    a.f[o] = make_float2((float)c1, (float)c2);
    a.f[a.N + o] = make_float2((float)w, 0.f);
    a.f[2 * a.N + o] = make_float2((float)(c1 * c1 - c2 * c2), (float)(2.0 * c1 * c2));
    a.f[3 * a.N + o] = make_float2((float)(c1 * c1 + c2 * c2), 0.f);
    a.f[4 * a.N + o] = make_float2((float)(w * w), 0.f);
    a.slot[(size_t)y * a.nx_occ + x] = (int)P;
}

inline unsigned nblk(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

bool smooth(int n)
{
    for (int f : {2, 3, 5})
        while (n % f == 0) n /= f;
    return n == 1;
}

int nice_size(int n)
{
    for (int k = std::max(n, 1); k <= kFftMax; ++k)
        if (smooth(k)) return k;
    return -1;
}

void factor(int n, RowPlan &p)
{
    p.n = n;
    p.ns = 0;
    int ns = 1;
    for (int r : {8, 4, 2, 5, 3})
        while (n % r == 0 && p.ns < kMaxStages) {
            p.magic[p.ns] = ns >= 2 ? (unsigned)(((1ull << 32) + ns - 1) / ns) : 0u;
            p.radix[p.ns++] = r;
            ns *= r;
            n /= r;
        }
}

template <class Load, class Store>
int rows_launch(const RowPlan &p, float s, Load ld, Store st, int n_rows, int batch, hipStream_t q, int row_gap = 0,
                int gap_len = 0)
{
    if (n_rows <= 0 || batch <= 0) return T3_OK;
    const dim3 grid((unsigned)n_rows, (unsigned)batch), block(kFftThreads);
    const size_t lds = sizeof(float2) * p.n;
    if (p.n <= 1024)
        hipLaunchKernelGGL((k_fft_rows<1024, Load, Store>), grid, block, lds, q, p, s, ld, st, row_gap, gap_len);
    else if (p.n <= 4096)
        hipLaunchKernelGGL((k_fft_rows<4096, Load, Store>), grid, block, lds, q, p, s, ld, st, row_gap, gap_len);
    else
        hipLaunchKernelGGL((k_fft_rows<kFftMax, Load, Store>), grid, block, lds, q, p, s, ld, st, row_gap, gap_len);
    T3_HIP_CHECK(hipGetLastError());
    return T3_OK;
}

int transpose(const float2 *src, float2 *dst, int rows, int cols, int batch, size_t stride, hipStream_t q)
{
    hipLaunchKernelGGL(k_transpose,
                       dim3((unsigned)((cols + kTile - 1) / kTile), (unsigned)((rows + kTile - 1) / kTile),
                            (unsigned)batch),
                       dim3(256), 0, q, src, dst, rows, cols, stride);
    T3_HIP_CHECK(hipGetLastError());
    return T3_OK;
}

// Orders and inverse transforms of one bin: kernel order m is needed by
// G (m <= n_max - 1), W (0 <= m <= w_max) and the j = k sums (m = -6, -2, 0).
struct Job {
    int f, m, p_re, p_im;
};
void jobs_of(const t3_plan *plan, const ChunkLayout &L, int *m_lo, int *m_hi, std::vector<Job> &jobs)
{
    *m_lo = -plan->n_max - 3;
    *m_hi = std::max(plan->n_max - 1, plan->w_max);
    jobs.clear();
    for (int m = *m_lo; m <= *m_hi; ++m) {
        if (m <= plan->n_max - 1) jobs.push_back({0, m, L.plane_G(m, 0), L.plane_G(m, 1)});
        if (m >= 0 && m <= plan->w_max) jobs.push_back({1, m, L.plane_W(m, 0), L.plane_W(m, 1)});
        if (m == -6) jobs.push_back({2, m, L.plane_D(0), L.plane_D(1)});
        if (m == -2) {
            jobs.push_back({2, m, L.plane_D(2), L.plane_D(3)});
            jobs.push_back({3, m, L.plane_D(4), L.plane_D(5)});
        }
        if (m == 0) jobs.push_back({4, m, L.plane_D(6), -1});
    }
}

constexpr double kBatchBytes = 2.0 * (1 << 30);    // work grids of one batch of inverse transforms
constexpr double kSpectraBytes = 24.0 * (1 << 30); // kernel spectra kept per level

}  // namespace

// Occupied pixel range of a level (corners px, py by pixel) and the ratio of
// its largest pixel weight to the mean, read back to the host.
int level_bbox(GridLevel &lv, const int32_t *px, const int32_t *py, const double *sum, hipStream_t s)
{
    lv.nx_occ = lv.ny_occ = 0;
    lv.w_peak = 0.0;
    if (lv.n_pix == 0) return T3_OK;
    T3_TRY(lv.fft_misc.reserve(sizeof(int) * 8));
    const int init[6] = {0x7fffffff, 0x7fffffff, (int)0x80000000, (int)0x80000000, 0, 0};
    T3_HIP_CHECK(hipMemcpyAsync(lv.fft_misc.ptr, init, sizeof(init), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_bbox, dim3(nblk(lv.n_pix, kBoxBlock)), dim3(kBoxBlock), 0, s, px, py, sum, lv.n_pix,
                       lv.fft_misc.as<int>(), reinterpret_cast<float *>(lv.fft_misc.as<int>() + 5));
    T3_HIP_CHECK(hipGetLastError());
    int h[6];
    T3_HIP_CHECK(hipMemcpyAsync(h, lv.fft_misc.ptr, sizeof(h), hipMemcpyDeviceToHost, s));
    T3_HIP_CHECK(hipStreamSynchronize(s));
    for (int k = 0; k < 4; ++k) lv.box[k] = h[k];
    lv.nx_occ = (int)(((int64_t)lv.box[2] - lv.box[0]) / lv.side) + 1;
    lv.ny_occ = (int)(((int64_t)lv.box[3] - lv.box[1]) / lv.side) + 1;
    float wmax, wsum;
    std::memcpy(&wmax, &h[4], sizeof(float));
    std::memcpy(&wsum, &h[5], sizeof(float));
    lv.w_peak = wsum > 0.0f ? (double)wmax * (double)lv.n_pix / (double)wsum : 0.0;
    return T3_OK;
}

// FFT grid of a level: sides >= occupied extent + kernel reach (the reach
// clamped to the extent - 1: larger offsets never meet data), so the
// circular correlation equals the linear one on the occupied pixels and
// kernel offsets are represented without overlap.  False above 8192.
bool fft_geometry(const t3_plan *plan, const GridLevel &lv, int *nx, int *ny, int *rx, int *ry)
{
    const double emax = std::sqrt(plan->e2[lv.b_lo + lv.nb]);
    const int64_t R = (int64_t)(emax / (double)lv.side) + 1;
    *rx = (int)std::min<int64_t>(R, lv.nx_occ - 1);
    *ry = (int)std::min<int64_t>(R, lv.ny_occ - 1);
    if ((int64_t)lv.nx_occ + *rx > kFftMax || (int64_t)lv.ny_occ + *ry > kFftMax) return false;
    *nx = nice_size(lv.nx_occ + *rx);
    *ny = nice_size(lv.ny_occ + *ry);
    return *nx > 0 && *ny > 0;
}

// Modelled time (ms) of the FFT route for a level: the inverse transforms
// (three passes over the grid each, the first reading two grids), plus the
// kernel transforms unless they are kept from an earlier call, at the
// effective rate measured for these kernels.
double fft_cost_ms(const t3_plan *plan, const GridLevel &lv)
{
    int nx, ny, rx, ry;
    if (lv.n_pix == 0 || !fft_geometry(plan, lv, &nx, &ny, &rx, &ry)) return 1e30;
    int m_lo, m_hi;
    std::vector<Job> jobs;
    ChunkLayout L = lv.L;
    jobs_of(plan, L, &m_lo, &m_hi, jobs);
    const double grid = sizeof(float2) * (double)nx * ny;
    double bytes = 7.0 * grid * (double)jobs.size() * lv.nb;
    const bool kept = lv.spec_key[0] == nx && lv.spec_key[1] == ny && lv.spec_key[2] == rx && lv.spec_key[3] == ry &&
                      lv.spec_key[4] == lv.side && lv.spec_key[5] == lv.b_lo && lv.spec_key[6] == lv.nb;
    if (!kept) bytes += 5.0 * grid * (double)(m_hi - m_lo + 1) * lv.nb;
    return 1e3 * bytes / 3.5e12 + 0.05 * lv.nb;  // about 3.5 TB/s measured on the 1M field's levels
}

int fft_level(t3_plan *plan, GridLevel &lv, hipStream_t s)
{
    const int64_t n_pix = lv.n_pix;
    if (n_pix == 0) return T3_OK;
    int nx, ny, Rx, Ry;
    if (!fft_geometry(plan, lv, &nx, &ny, &Rx, &Ry))
        return fail(T3_ERANGE, "t3_forward_grid: FFT grid above 8192 pixels per side");
    const int nx_occ = lv.nx_occ, ny_occ = lv.ny_occ;
    const ChunkLayout &L = lv.L;
    const size_t N = (size_t)nx * ny;
    int m_lo, m_hi;
    std::vector<Job> jobs;
    jobs_of(plan, L, &m_lo, &m_hi, jobs);
    const int n_ord = m_hi - m_lo + 1;
    const int n_jobs = (int)jobs.size();
    // kernel spectra of every (bin, order): kept between calls when they fit
    const double spec_bytes = sizeof(float2) * (double)N * n_ord * lv.nb;
    const bool keep = spec_bytes <= kSpectraBytes;
    const int64_t key[7] = {nx, ny, Rx, Ry, lv.side, lv.b_lo, lv.nb};
    bool have = keep;
    for (int i = 0; i < 7; ++i) have = have && lv.spec_key[i] == key[i];
    // batch of inverse transforms: two work grids per job
    const int jb = (int)std::max(1.0, std::min((double)n_jobs, kBatchBytes / (2.0 * sizeof(float2) * N)));
    const int kb = std::min(n_ord, jb);  // kernel orders per batch (when not kept)
    const size_t n_spec = keep ? (size_t)n_ord * lv.nb : (size_t)n_ord;
    T3_TRY(lv.fft_spec.reserve(sizeof(float2) * N * n_spec));
    T3_TRY(lv.fft_buf.reserve(sizeof(float2) * N * (5 + 2 * (size_t)jb) + sizeof(int) * (size_t)nx_occ * ny_occ +
                              sizeof(float2) * (size_t)(nx + ny) + sizeof(int) * 4 * (size_t)n_jobs));
    float2 *F = lv.fft_buf.as<float2>();  // five field spectra
    float2 *A = F + 5 * N, *Bw = A + (size_t)jb * N;
    int *slot = reinterpret_cast<int *>(Bw + (size_t)jb * N);
    float2 *twx = reinterpret_cast<float2 *>(slot + (size_t)nx_occ * ny_occ);
    float2 *twy = twx + nx;
    int *jf = reinterpret_cast<int *>(twy + ny), *jk = jf + n_jobs, *jre = jk + n_jobs, *jim = jre + n_jobs;
    float2 *Ks = lv.fft_spec.as<float2>();
    {
        std::vector<float2> h(nx + ny);
        for (int k = 0; k < nx; ++k) {
            const double a = -2.0 * M_PI * (double)k / nx;
            h[k] = make_float2((float)std::cos(a), (float)std::sin(a));
        }
        for (int k = 0; k < ny; ++k) {
            const double a = -2.0 * M_PI * (double)k / ny;
            h[nx + k] = make_float2((float)std::cos(a), (float)std::sin(a));
        }
        std::vector<int> jt(4 * (size_t)n_jobs);
        for (int j = 0; j < n_jobs; ++j) {
            jt[j] = jobs[j].f;
            jt[n_jobs + j] = jobs[j].m - m_lo;  // spectrum slot within the bin
            jt[2 * n_jobs + j] = jobs[j].p_re;
            jt[3 * n_jobs + j] = jobs[j].p_im;
        }
        T3_HIP_CHECK(hipMemcpyAsync(twx, h.data(), sizeof(float2) * h.size(), hipMemcpyHostToDevice, s));
        T3_HIP_CHECK(hipMemcpyAsync(jf, jt.data(), sizeof(int) * jt.size(), hipMemcpyHostToDevice, s));
        T3_HIP_CHECK(hipStreamSynchronize(s));  // h, jt leave scope
    }
    RowPlan px, py;
    factor(nx, px);
    factor(ny, py);
    px.tw = twx;
    py.tw = twy;

    // fields on the grid, slot map, forward transforms -> spectra [nx][ny]
    hipLaunchKernelGGL(k_zero_c, dim3(nblk(N * 5, 256)), dim3(256), 0, s, F, N * 5);
    T3_HIP_CHECK(hipGetLastError());
    T3_TRY(fill_int(slot, (int64_t)nx_occ * ny_occ, -1, s));
    const int32_t *pxa = lv.pix_xy.as<int32_t>();
    const size_t np1 = (size_t)(n_pix > 0 ? n_pix : 1);
    ScatterArgs sa{pxa, pxa + np1, lv.pix_sum.as<double>(), n_pix, lv.box[0], lv.box[1], lv.side, nx, nx_occ, N, F,
                   slot};
    hipLaunchKernelGGL(k_scatter_fields, dim3(nblk(n_pix, 256)), dim3(256), 0, s, sa);
    T3_HIP_CHECK(hipGetLastError());
    for (int f0 = 0; f0 < 5; f0 += jb) {
        const int nf = std::min(jb, 5 - f0);
        T3_TRY(rows_launch(px, -1.0f, LoadGrid{F + f0 * N, N}, StoreGrid{A, N}, ny, nf, s));
        T3_TRY(transpose(A, Bw, ny, nx, nf, N, s));
        T3_TRY(rows_launch(py, -1.0f, LoadGrid{Bw, N}, StoreGrid{F + f0 * N, N}, nx, nf, s));
    }

    const float scale = 1.0f / (float)N;
    for (int bl = 0; bl < lv.nb; ++bl) {
        const int b = lv.b_lo + bl;
        float2 *Kb = Ks + (keep ? (size_t)bl * n_ord * N : 0);  // spectra of this bin's orders
        if (!have) {
            // only the rows |dy| <= Ry of a kernel grid are non-zero (ny >= 2 Ry + 1)
            const int head = Ry + 1, tail = Ry;
            for (int m0 = 0; m0 < n_ord; m0 += kb) {
                const int nm = std::min(kb, n_ord - m0);
                hipLaunchKernelGGL(k_zero_c, dim3(nblk(N * nm, 256)), dim3(256), 0, s, A, N * nm);
                T3_HIP_CHECK(hipGetLastError());
                LoadKernel lk{nx, ny, Rx, Ry, m_lo + m0, (double)lv.side, plan->e2[b], plan->e2[b + 1]};
                T3_TRY(rows_launch(px, -1.0f, lk, StoreGrid{A, N}, head + tail, nm, s, head, ny - head - tail));
                T3_TRY(transpose(A, Bw, ny, nx, nm, N, s));
                T3_TRY(rows_launch(py, -1.0f, LoadGrid{Bw, N}, StoreGrid{Kb + (size_t)m0 * N, N}, nx, nm, s));
            }
        }
        // inverse transforms of field spectrum x kernel spectrum, values at the pixels
        for (int j0 = 0; j0 < n_jobs; j0 += jb) {
            const int nj = std::min(jb, n_jobs - j0);
            T3_TRY(rows_launch(py, 1.0f, LoadProduct{F, Kb, N, jf, jk, j0}, StoreGrid{A, N}, nx, nj, s));
            T3_TRY(transpose(A, Bw, nx, ny, nj, N, s));
            StorePlanes sp{slot, nx_occ, ny_occ, lv.planes.as<float>(), jre, jim, j0, L.K, L.B, bl, scale};
            T3_TRY(rows_launch(px, 1.0f, LoadGrid{Bw, N}, sp, ny, nj, s));
        }
    }
    for (int i = 0; i < 7; ++i) lv.spec_key[i] = keep ? key[i] : -1;
    return T3_OK;
}

}  // namespace t3
