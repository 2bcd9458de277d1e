// Stage 2 of the multipole estimator: the contraction over centres
//     Upsilon_{mu,n}(b1, b2) = sum_i alpha_i X_{mu,n}(i, b1) Y_{mu,n}(i, b2)
// (Porth et al. 2023, eqs. Upsilon0_Derivation, Upsilon1-3,
// 3PCF_Normalization), one small complex GEMM (B x B, K = centres) per
// (mu, n), run on MFMA:
//     mu = 0: alpha = -c,  X = G_{n-3},      Y = G_{-n-3}
//     mu = 1: alpha = -c*, X = G_{n-1},      Y = G_{-n-1}
//     mu = 2: alpha = -c,  X = G_{-n-1}*,    Y = G_{-n-3}
//     mu = 3: alpha = -c,  X = G_{n-3},      Y = G_{n-1}*
//     mu = 4: alpha =  w,  X = W_n,          Y = W_n*
// A complex product is four real MFMAs: Re += Xr Yr - Xi Yi, Im += Xr Yi + Xi Yr.
// Each wavefront owns one (mu, n) and one slice of centres; FP32 MFMA runs
// of at most 64 centres are promoted into FP64 accumulators, and the
// slices are summed in FP64 in a fixed order (deterministic).  The j = k
// terms (n-independent, diagonal only) are summed separately in FP64 and
// subtracted in the final reduction.
//
// Precision variants (same operands, same FP64 promotion):
//  * FP32:    v_mfma_f32_32x32x2_f32.
//  * BF16x3:  x = hi + lo with hi = bf16(x), lo = bf16(x - hi); each real
//             product is hi*hi + hi*lo + lo*hi on v_mfma_f32_32x32x16_bf16.
//             The normaliser N_n, which divides every Gamma, stays on the
//             FP32 path (hi + lo in bf16 keeps about 17 bits).
//  * FP16x3:  as BF16x3 in fp16 after scaling each (operand, bin) row by a
//             power of two so that its largest entry is near 2^12 (keeps lo
//             out of the subnormal range); the scales are divided out in FP64.
#include "t3_internal.h"

namespace t3 {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

constexpr int kRun = 64;   // centres per FP32 accumulation run before FP64 promotion

// One launch covers every ordered pair (Z2, Z3) of neighbour catalogs
// (grid.z = n_z^2; n_z = 1 outside tomography): the b1-side harmonics come
// from the planes of Z2, the b2-side ones from those of Z3.
struct ContractArgs {
    const float *planes; // planes of catalog 0; catalog z at planes + z * zstride
    size_t zstride;
    const float4 *ccw;   // centre factors (w g1, w g2, w, 0), chunk-relative
    const float *scale;  // fp16 row scales [pair][2][5][n_max+1][B] or null
    int n_c, K, B, n_max, n_z;
    int slice;           // centres per slice (multiple of 16)
    int S;               // slices
    int mu0;             // first component of this launch (grid.x covers mu >= mu0)
    double *partial;     // [pair][S][5][n_max+1][B][B][2]
};

__device__ __forceinline__ void pair_planes(const ContractArgs &a, int pair, const float *&px,
                                            const float *&py)
{
    px = a.planes + (size_t)(pair / a.n_z) * a.zstride;
    py = a.planes + (size_t)(pair % a.n_z) * a.zstride;
}

struct Operands {
    int xr, xi, yr, yi;  // plane indices
    float xs, ys;        // sign applied to the imaginary parts (conjugation)
};

__device__ __forceinline__ Operands operands(int mu, int n, int n_max)
{
    const int n_g = 2 * n_max + 3;
    auto pg = [&](int m) { return 2 * (m + n_max + 3); };
    Operands o;
    int xm, ym;
    o.xs = 1.0f;
    o.ys = 1.0f;
    switch (mu) {
        case 0: xm = n - 3; ym = -n - 3; break;
        case 1: xm = n - 1; ym = -n - 1; break;
        case 2: xm = -n - 1; ym = -n - 3; o.xs = -1.0f; break;
        case 3: xm = n - 3; ym = n - 1; o.ys = -1.0f; break;
        default: xm = 0; ym = 0; o.ys = -1.0f; break;
    }
    if (mu < 4) {
        o.xr = pg(xm);
        o.yr = pg(ym);
    } else {
        o.xr = 2 * n_g + 2 * n;
        o.yr = o.xr;
    }
    o.xi = o.xr + 1;
    o.yi = o.yr + 1;
    return o;
}

// alpha_i for component mu from (w g1, w g2, w).
__device__ __forceinline__ void alpha_of(int mu, float4 f, float &ar, float &ai)
{
    if (mu == 4) {
        ar = f.z;
        ai = 0.0f;
    } else if (mu == 1) {
        ar = -f.x;
        ai = f.y;
    } else {
        ar = -f.x;
        ai = -f.y;
    }
}

__device__ __forceinline__ void store_tile(double *dst, int B, int lane, const double (&dr)[16],
                                           const double (&di)[16], double sx = 1.0)
{
    const int col = lane & 31;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int row = 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
        if (row < B && col < B) {
            double2 v;
            v.x = dr[j] * sx;
            v.y = di[j] * sx;
            *reinterpret_cast<double2 *>(dst + 2 * ((size_t)row * B + col)) = v;
        }
    }
}

// Loads 4 consecutive centres (ib..ib+3) of bin b for one plane; zeros for
// bins >= B or centres >= i_end (select, never multiply: stale memory may
// hold non-finite values).
__device__ __forceinline__ float4 load4(const float *planes, int plane, int ib, int b, int K, int B,
                                        int i_end)
{
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (b < B && ib < i_end) {
        v = *reinterpret_cast<const float4 *>(planes + chunk_offset(plane, ib, b, K, B));
        if (ib + 1 >= i_end) v.y = 0.f;
        if (ib + 2 >= i_end) v.z = 0.f;
        if (ib + 3 >= i_end) v.w = 0.f;
    }
    return v;
}

__global__ __launch_bounds__(64) void k_contract_fp32(ContractArgs a)
{
    const int lane = threadIdx.x;
    const int mn = blockIdx.x + a.mu0 * (a.n_max + 1);
    const int mu = mn / (a.n_max + 1), n = mn % (a.n_max + 1);
    const int sl = blockIdx.y;
    const int pair = blockIdx.z;
    const float *px, *py;
    pair_planes(a, pair, px, py);
    const int i_begin = sl * a.slice;
    const int i_end = min(i_begin + a.slice, a.n_c);
    const Operands o = operands(mu, n, a.n_max);
    const int b = lane & 31, kq = lane >> 5;

    floatx16 cr = {}, ci = {};
    double dr[16], di[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) dr[j] = di[j] = 0.0;

    int run = 0;
    for (int i0 = i_begin; i0 < i_end; i0 += 8) {
        const int ib = i0 + 4 * kq;
        const float4 xr = load4(px, o.xr, ib, b, a.K, a.B, i_end);
        float4 xi = load4(px, o.xi, ib, b, a.K, a.B, i_end);
        const float4 yr = load4(py, o.yr, ib, b, a.K, a.B, i_end);
        float4 yi = load4(py, o.yi, ib, b, a.K, a.B, i_end);
        const float xa[4] = {xr.x, xr.y, xr.z, xr.w};
        const float xb[4] = {xi.x * o.xs, xi.y * o.xs, xi.z * o.xs, xi.w * o.xs};
        const float ya[4] = {yr.x, yr.y, yr.z, yr.w};
        const float yb[4] = {yi.x * o.ys, yi.y * o.ys, yi.z * o.ys, yi.w * o.ys};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            float al_r = 0.f, al_i = 0.f;
            if (ib + s < i_end) alpha_of(mu, a.ccw[ib + s], al_r, al_i);
            const float pr = fmaf(al_r, xa[s], -al_i * xb[s]);
            const float pi = fmaf(al_r, xb[s], al_i * xa[s]);
            cr = __builtin_amdgcn_mfma_f32_32x32x2f32(pr, ya[s], cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_32x32x2f32(-pi, yb[s], cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_32x32x2f32(pr, yb[s], ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_32x32x2f32(pi, ya[s], ci, 0, 0, 0);
        }
        run += 8;
        if (run >= kRun) {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                dr[j] += (double)cr[j];
                di[j] += (double)ci[j];
                cr[j] = 0.f;
                ci[j] = 0.f;
            }
            run = 0;
        }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        dr[j] += (double)cr[j];
        di[j] += (double)ci[j];
    }
    double *dst = a.partial + ((((size_t)pair * a.S + sl) * 5 + mu) * (a.n_max + 1) + n) * a.B * a.B * 2;
    store_tile(dst, a.B, lane, dr, di);
}

// hi/lo split of 8 values for the split-precision variants.
template <class T>
__device__ __forceinline__ void split8(const float (&x)[8], T (&hi)[8], T (&lo)[8])
{
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        hi[j] = (T)x[j];
        lo[j] = (T)(x[j] - (float)hi[j]);
    }
}

// Split-precision contraction: 16 centres per MFMA (8 per half-wave).
// Lane (b, kq) holds centres ib = i0 + 8 kq + (0..7).
template <bool FP16>
__global__ __launch_bounds__(64) void k_contract_split(ContractArgs a)
{
    using T = typename std::conditional<FP16, _Float16, __bf16>::type;
    using V8 = typename std::conditional<FP16, halfx8, bf16x8>::type;
    const int lane = threadIdx.x;
    const int mn = blockIdx.x + a.mu0 * (a.n_max + 1);
    const int mu = mn / (a.n_max + 1), n = mn % (a.n_max + 1);
    const int sl = blockIdx.y;
    const int pair = blockIdx.z;
    const float *px, *py;
    pair_planes(a, pair, px, py);
    const int i_begin = sl * a.slice;
    const int i_end = min(i_begin + a.slice, a.n_c);
    const Operands o = operands(mu, n, a.n_max);
    const int b = lane & 31, kq = lane >> 5;

    // power-of-two row scales (FP16 only): X row b1 by sx, Y row b2 by sy
    const size_t half = (size_t)5 * (a.n_max + 1) * a.B;
    const float *scale = a.scale ? a.scale + (size_t)pair * 2 * half : nullptr;
    float sx = 1.0f, sy = 1.0f;
    if (FP16 && scale) {
        const size_t base = ((size_t)mu * (a.n_max + 1) + n) * a.B;
        if (b < a.B) {
            sx = scale[base + b];
            sy = scale[half + base + b];
        }
    }

    floatx16 cr = {}, ci = {};
    double dr[16], di[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) dr[j] = di[j] = 0.0;
    int run = 0;
    for (int i0 = i_begin; i0 < i_end; i0 += 16) {
        const int ib = i0 + 8 * kq;
        float xa[8], xb[8], ya[8], yb[8];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float4 xr = load4(px, o.xr, ib + 4 * h, b, a.K, a.B, i_end);
            const float4 xi = load4(px, o.xi, ib + 4 * h, b, a.K, a.B, i_end);
            const float4 yr = load4(py, o.yr, ib + 4 * h, b, a.K, a.B, i_end);
            const float4 yi = load4(py, o.yi, ib + 4 * h, b, a.K, a.B, i_end);
            const float xr4[4] = {xr.x, xr.y, xr.z, xr.w}, xi4[4] = {xi.x, xi.y, xi.z, xi.w};
            const float yr4[4] = {yr.x, yr.y, yr.z, yr.w}, yi4[4] = {yi.x, yi.y, yi.z, yi.w};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int i = ib + 4 * h + s;
                float al_r = 0.f, al_i = 0.f;
                if (i < i_end) alpha_of(mu, a.ccw[i], al_r, al_i);
                const float x_r = xr4[s], x_i = xi4[s] * o.xs;
                xa[4 * h + s] = fmaf(al_r, x_r, -al_i * x_i) * sx;
                xb[4 * h + s] = fmaf(al_r, x_i, al_i * x_r) * sx;
                ya[4 * h + s] = yr4[s] * sy;
                yb[4 * h + s] = yi4[s] * o.ys * sy;
            }
        }
        T xah[8], xal[8], xbh[8], xbl[8], yah[8], yal[8], ybh[8], ybl[8];
        split8<T>(xa, xah, xal);
        split8<T>(xb, xbh, xbl);
        split8<T>(ya, yah, yal);
        split8<T>(yb, ybh, ybl);
        V8 XAH, XAL, XBH, XBL, YAH, YAL, YBH, YBL, NXBH, NXBL;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            XAH[j] = xah[j]; XAL[j] = xal[j]; XBH[j] = xbh[j]; XBL[j] = xbl[j];
            YAH[j] = yah[j]; YAL[j] = yal[j]; YBH[j] = ybh[j]; YBL[j] = ybl[j];
            NXBH[j] = -xbh[j]; NXBL[j] = -xbl[j];
        }
        // Re: xa*ya - xb*yb ; Im: xa*yb + xb*ya ; each as hi*hi + hi*lo + lo*hi
        if constexpr (FP16) {
            cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(XAH, YAH, cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(XAH, YAL, cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(XAL, YAH, cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(NXBH, YBH, cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(NXBH, YBL, cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(NXBL, YBH, cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(XAH, YBH, ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(XAH, YBL, ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(XAL, YBH, ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(XBH, YAH, ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(XBH, YAL, ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(XBL, YAH, ci, 0, 0, 0);
        } else {
            cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XAH, YAH, cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XAH, YAL, cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XAL, YAH, cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(NXBH, YBH, cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(NXBH, YBL, cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(NXBL, YBH, cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XAH, YBH, ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XAH, YBL, ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XAL, YBH, ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XBH, YAH, ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XBH, YAL, ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XBL, YAH, ci, 0, 0, 0);
        }
        run += 16;
        if (run >= kRun) {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                dr[j] += (double)cr[j];
                di[j] += (double)ci[j];
                cr[j] = 0.f;
                ci[j] = 0.f;
            }
            run = 0;
        }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        dr[j] += (double)cr[j];
        di[j] += (double)ci[j];
    }
    // undo the row scales: entry (row, col) carries sx(row) sy(col)
    double *dst = a.partial + ((((size_t)pair * a.S + sl) * 5 + mu) * (a.n_max + 1) + n) * a.B * a.B * 2;
    if (FP16 && scale) {
        const size_t base = ((size_t)mu * (a.n_max + 1) + n) * a.B;
        const int col = lane & 31;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int row = 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
            if (row < a.B && col < a.B) {
                const double f = 1.0 / ((double)scale[base + row] * (double)scale[half + base + col]);
                double2 v;
                v.x = dr[j] * f;
                v.y = di[j] * f;
                *reinterpret_cast<double2 *>(dst + 2 * ((size_t)row * a.B + col)) = v;
            }
        }
    } else {
        store_tile(dst, a.B, lane, dr, di);
    }
}

// Row scales for FP16x3: for every (mu, n) and bin, the power of two that
// brings max_i |alpha_i X(i, b)| (resp. max |Y(i, b)|) to [2^11, 2^12).
__global__ __launch_bounds__(256) void k_fp16_scales(ContractArgs a, float *scale_all)
{
    const int mn = blockIdx.x;
    const int mu = mn / (a.n_max + 1), n = mn % (a.n_max + 1);
    const int b = blockIdx.y;
    const int side = blockIdx.z & 1;  // 0: X (with alpha), 1: Y
    const int pair = blockIdx.z >> 1;
    const float *px, *py;
    pair_planes(a, pair, px, py);
    float *scale = scale_all + (size_t)pair * 2 * 5 * (a.n_max + 1) * a.B;
    const Operands o = operands(mu, n, a.n_max);
    float m = 0.0f;
    for (int i = threadIdx.x; i < a.n_c; i += blockDim.x) {
        const float *pl = side ? py : px;
        const int pr = side ? o.yr : o.xr;
        const float re = pl[chunk_offset(pr, i, b, a.K, a.B)];
        const float im = pl[chunk_offset(pr + 1, i, b, a.K, a.B)];
        float v = fmaxf(fabsf(re), fabsf(im));
        if (!side) {
            const float4 f = a.ccw[i];
            const float al = mu == 4 ? fabsf(f.z) : fmaxf(fabsf(f.x), fabsf(f.y));
            v *= 2.0f * al;
        }
        m = fmaxf(m, v);
    }
    __shared__ float sm[256];
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float sc = 1.0f;
        const float mx = sm[0];
        if (mx > 0.0f && isfinite(mx)) {
            const int e = ilogbf(mx);  // mx in [2^e, 2^{e+1})
            sc = ldexpf(1.0f, 11 - e);
        }
        scale[(size_t)side * 5 * (a.n_max + 1) * a.B + ((size_t)mu * (a.n_max + 1) + n) * a.B + b] = sc;
    }
}

// Diagonal (j = k) sums E_mu(b) = sum_i alpha_i D_mu(i, b) in FP64.
__global__ __launch_bounds__(256) void k_diag(const float *planes0, size_t zstride, const float4 *ccw,
                                              int n_c, int K, int B, int pD, double *E0)
{
    const int mu = blockIdx.x, b = blockIdx.y;
    const float *planes = planes0 + (size_t)blockIdx.z * zstride;
    double *E = E0 + (size_t)blockIdx.z * 10 * B;
    double sr = 0.0, si = 0.0;
    for (int i = threadIdx.x; i < n_c; i += blockDim.x) {
        float ar, ai;
        alpha_of(mu, ccw[i], ar, ai);
        float dr, di;
        if (mu == 4) {
            dr = planes[chunk_offset(pD + 6, i, b, K, B)];
            di = 0.0f;
        } else {
            const int d = mu == 0 ? 0 : (mu == 1 ? 2 : 4);
            dr = planes[chunk_offset(pD + d, i, b, K, B)];
            di = planes[chunk_offset(pD + d + 1, i, b, K, B)];
        }
        sr += (double)ar * dr - (double)ai * di;
        si += (double)ar * di + (double)ai * dr;
    }
    __shared__ double s_r[256], s_i[256];
    s_r[threadIdx.x] = sr;
    s_i[threadIdx.x] = si;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            s_r[threadIdx.x] += s_r[threadIdx.x + s];
            s_i[threadIdx.x] += s_i[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        E[2 * (mu * B + b)] = s_r[0];
        E[2 * (mu * B + b) + 1] = s_i[0];
    }
}

// out[pair][mu][n][b1][b2] += sum_s partial[pair][s][...] - [b1 == b2][Z2 == Z3] E_{Z2,mu}(b1)
__global__ void k_reduce(const double *partial, int S, int n_max, int B, int n_z, const double *E,
                         int jk, double *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)5 * (n_max + 1) * B * B;
    if (t >= per * n_z * n_z) return;
    const int pair = (int)(t / per);
    const int64_t e = t % per;
    const int b2 = (int)(e % B);
    const int b1 = (int)((e / B) % B);
    const int mu = (int)(e / ((int64_t)(n_max + 1) * B * B));
    const double *p = partial + 2 * ((int64_t)pair * S * per + e);
    double re = 0.0, im = 0.0;
    for (int s = 0; s < S; ++s) {
        re += p[2 * s * per];
        im += p[2 * s * per + 1];
    }
    const int z2 = pair / n_z, z3 = pair % n_z;
    if (jk && z2 == z3 && b1 == b2) {
        const double *Ez = E + (size_t)z2 * 10 * B;
        re -= Ez[2 * (mu * B + b1)];
        im -= Ez[2 * (mu * B + b1) + 1];
    }
    out[2 * t] += re;
    out[2 * t + 1] += im;
}

__global__ void k_zero(double *p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

}  // namespace

int zero_doubles(double *p, size_t n, hipStream_t s)
{
    if (n == 0) return T3_OK;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    T3_HIP_CHECK(hipGetLastError());
    return T3_OK;
}

// Centres per stage-2 slice: a function of the chunk capacity only, so that
// every chunk of a call fits the buffers reserved up front.
int contract_slice(const ChunkLayout &L, int n_z)
{
    const int nmn = 5 * (L.n_max + 1);
    int slice = 512;
    while (slice > 64 && (int64_t)nmn * n_z * n_z * ((L.K + slice - 1) / slice) < 2048) slice >>= 1;
    return slice;
}

int reserve_contract(t3_plan *plan, const ChunkLayout &L, int n_z)
{
    const int pairs = n_z * n_z;
    const int S = (L.K + contract_slice(L, n_z) - 1) / contract_slice(L, n_z);
    const size_t per = (size_t)5 * (L.n_max + 1) * L.B * L.B;
    T3_TRY(plan->partial.reserve(sizeof(double) * 2 * per * (size_t)S * pairs));
    T3_TRY(plan->diag.reserve(sizeof(double) * 2 * 5 * (size_t)L.B * n_z));
    if (plan->precision == T3_PREC_FP16X3)
        T3_TRY(plan->scales.reserve(sizeof(float) * 2 * 5 * (size_t)(L.n_max + 1) * L.B * pairs));
    return T3_OK;
}

int contract_chunk(t3_plan *plan, const CentreSet &cs, int64_t c0, int n_c, const ChunkLayout &L,
                   const float *planes, size_t zstride, int n_z, bool jk, double *ups_out, hipStream_t s)
{
    if (n_c <= 0) return T3_OK;
    const int nmn = 5 * (L.n_max + 1);
    const int pairs = n_z * n_z;
    const int slice = contract_slice(L, n_z);
    const int S = (n_c + slice - 1) / slice;
    const size_t per = (size_t)nmn * L.B * L.B;
    T3_TRY(reserve_contract(plan, L, n_z));  // no-op when reserved before a capture

    ContractArgs a{};
    a.planes = planes;
    a.zstride = zstride;
    a.ccw = cs.cw.as<float4>() + c0;
    a.scale = nullptr;
    a.n_c = n_c;
    a.K = L.K;
    a.B = L.B;
    a.n_max = L.n_max;
    a.n_z = n_z;
    a.slice = slice;
    a.S = S;
    a.mu0 = 0;
    a.partial = plan->partial.as<double>();
    if (plan->precision == T3_PREC_FP32) {
        hipLaunchKernelGGL(k_contract_fp32, dim3(nmn, S, pairs), dim3(64), 0, s, a);
    } else if (plan->precision == T3_PREC_BF16X3) {
        const int nu = 4 * (L.n_max + 1);
        hipLaunchKernelGGL(k_contract_split<false>, dim3(nu, S, pairs), dim3(64), 0, s, a);
        T3_HIP_CHECK(hipGetLastError());
        ContractArgs an = a;
        an.mu0 = 4;
        hipLaunchKernelGGL(k_contract_fp32, dim3(nmn - nu, S, pairs), dim3(64), 0, s, an);
    } else {
        hipLaunchKernelGGL(k_fp16_scales, dim3(nmn, L.B, 2 * pairs), dim3(256), 0, s, a,
                           plan->scales.as<float>());
        T3_HIP_CHECK(hipGetLastError());
        a.scale = plan->scales.as<float>();
        hipLaunchKernelGGL(k_contract_split<true>, dim3(nmn, S, pairs), dim3(64), 0, s, a);
    }
    T3_HIP_CHECK(hipGetLastError());
    if (jk) {
        hipLaunchKernelGGL(k_diag, dim3(5, L.B, n_z), dim3(256), 0, s, planes, zstride, a.ccw, n_c, L.K,
                           L.B, L.plane_D(0), plan->diag.as<double>());
        T3_HIP_CHECK(hipGetLastError());
    }
    const size_t tot = per * pairs;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       (const double *)plan->partial.as<double>(), S, L.n_max, L.B, n_z,
                       (const double *)plan->diag.as<double>(), jk ? 1 : 0, ups_out);
    T3_HIP_CHECK(hipGetLastError());
    return T3_OK;
}

}  // namespace t3
