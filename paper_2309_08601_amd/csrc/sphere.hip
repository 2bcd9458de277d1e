// Curved-sky catalogs in flat patches (Porth et al. 2023, Appendix B).
//
// Per patch (an RA/Dec rectangle, its centre c):
//  * the rotation R that takes c to (RA, Dec) = (0, 0): a rotation about the
//    polar axis by -RA_c, then about the new y axis by Dec_c;
//  * the sinusoidal projection of the rotated position (longitude lambda,
//    latitude beta): x = lambda cos(beta), y = beta, in arcmin, rounded to
//    the plan's lattice (x east, y north);
//  * shears (spin 2 in the local (east, north) frame) rotated by the change
//    of reference direction: with psi the angle, from north towards east, of
//    R(north at p) in the (east, north) basis at R p, gamma' = gamma e^{-2 i psi};
//  * flags: bit 0 = in the extended patch (the rectangle widened by theta_max
//    in Dec and theta_max / cos(Dec) in RA), bit 1 = in the core rectangle.
// The patch driver (t3_forward_sphere) compacts the extended galaxies and
// runs the flat estimator with the core galaxies as centres (eq. PatchGamma).
#include "t3_internal.h"

namespace t3 {
namespace {

struct SphArgs {
    const double *ra, *dec;   // degrees
    const float *g1, *g2, *w;
    int64_t n;
    double R[9];              // row-major rotation
    double ra_lo, ra_hi, dec_lo, dec_hi, tmax_deg;
    double inv_unit;          // lattice steps per arcmin
    int32_t *x, *y;
    float *h1, *h2;
    int32_t *flag;
};

__device__ __forceinline__ void basis(double vx, double vy, double vz, double (&e)[3], double (&nn)[3])
{
    // east = z x v / |z x v|, north = v x east
    const double ex = -vy, ey = vx;
    const double en = sqrt(ex * ex + ey * ey);
    e[0] = ex / en;
    e[1] = ey / en;
    e[2] = 0.0;
    nn[0] = vy * e[2] - vz * e[1];
    nn[1] = vz * e[0] - vx * e[2];
    nn[2] = vx * e[1] - vy * e[0];
}

__global__ void k_sphere_project(SphArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const double d2r = 3.14159265358979323846 / 180.0;
    const double ra = a.ra[i], dec = a.dec[i];
    double sr, cr, sd, cd;
    sincos(ra * d2r, &sr, &cr);
    sincos(dec * d2r, &sd, &cd);
    const double v[3] = {cd * cr, cd * sr, sd};
    double w[3];
    for (int r = 0; r < 3; ++r) w[r] = a.R[3 * r] * v[0] + a.R[3 * r + 1] * v[1] + a.R[3 * r + 2] * v[2];
    const double lam = atan2(w[1], w[0]);
    const double beta = asin(fmin(1.0, fmax(-1.0, w[2])));
    const double arcmin = 180.0 * 60.0 / 3.14159265358979323846;
    const double xl = rint(lam * cos(beta) * arcmin * a.inv_unit);
    const double yl = rint(beta * arcmin * a.inv_unit);
    // shear reference-direction change
    double e0[3], n0[3], e1[3], n1[3];
    basis(v[0], v[1], v[2], e0, n0);
    basis(w[0], w[1], w[2], e1, n1);
    double rn[3];
    for (int r = 0; r < 3; ++r) rn[r] = a.R[3 * r] * n0[0] + a.R[3 * r + 1] * n0[1] + a.R[3 * r + 2] * n0[2];
    const double psi = atan2(rn[0] * e1[0] + rn[1] * e1[1] + rn[2] * e1[2], rn[0] * n1[0] + rn[1] * n1[1] + rn[2] * n1[2]);
    double sp, cp;
    sincos(-2.0 * psi, &sp, &cp);
    const double gr = a.g1[i], gi = a.g2[i];
    a.h1[i] = (float)(gr * cp - gi * sp);
    a.h2[i] = (float)(gr * sp + gi * cp);
    int f = 0;
    const double dra = a.tmax_deg / cos(fmin(89.9, fmax(-89.9, dec)) * d2r);
    if (ra >= a.ra_lo - dra && ra < a.ra_hi + dra && dec >= a.dec_lo - a.tmax_deg && dec < a.dec_hi + a.tmax_deg)
        f |= 1;
    if (ra >= a.ra_lo && ra < a.ra_hi && dec >= a.dec_lo && dec < a.dec_hi) f |= 2;
    const bool fits = fabs(xl) < 2147483000.0 && fabs(yl) < 2147483000.0;
    if (!fits) f |= 4;  // outside the int32 lattice: reported as an error by the driver
    a.x[i] = fits ? (int32_t)xl : 0;
    a.y[i] = fits ? (int32_t)yl : 0;
    a.flag[i] = f;
}

constexpr int kCompactBlock = 256;

// per block: number of extended galaxies and of extended core galaxies
__global__ __launch_bounds__(kCompactBlock) void k_sph_count(const int32_t *flag, int64_t n, int32_t *counts)
{
    __shared__ int s_ext, s_core;
    if (threadIdx.x == 0) {
        s_ext = 0;
        s_core = 0;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kCompactBlock + threadIdx.x;
    const int f = i < n ? flag[i] : 0;
    if (f & 1) atomicAdd(&s_ext, 1);
    if ((f & 3) == 3) atomicAdd(&s_core, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        counts[2 * blockIdx.x] = s_ext;
        counts[2 * blockIdx.x + 1] = s_core;
    }
}

// scatter in original order within a block (deterministic): ranks from a
// block-wide prefix count of the flags
__global__ __launch_bounds__(kCompactBlock) void k_sph_scatter(SphArgs a, const int32_t *offs, int32_t *cx,
                                                               int32_t *cy, float *cg1, float *cg2, float *cw,
                                                               int32_t *core_idx)
{
    __shared__ int s_e[kCompactBlock], s_c[kCompactBlock];
    const int64_t i = (int64_t)blockIdx.x * kCompactBlock + threadIdx.x;
    const int f = i < a.n ? a.flag[i] : 0;
    s_e[threadIdx.x] = f & 1;
    s_c[threadIdx.x] = (f & 3) == 3;
    __syncthreads();
    for (int d = 1; d < kCompactBlock; d <<= 1) {  // inclusive scans
        const int ve = threadIdx.x >= (unsigned)d ? s_e[threadIdx.x - d] : 0;
        const int vc = threadIdx.x >= (unsigned)d ? s_c[threadIdx.x - d] : 0;
        __syncthreads();
        s_e[threadIdx.x] += ve;
        s_c[threadIdx.x] += vc;
        __syncthreads();
    }
    if (f & 1) {
        const int j = offs[2 * blockIdx.x] + s_e[threadIdx.x] - 1;
        cx[j] = a.x[i];
        cy[j] = a.y[i];
        cg1[j] = a.h1[i];
        cg2[j] = a.h2[i];
        cw[j] = a.w[i];
        if (f & 2) core_idx[offs[2 * blockIdx.x + 1] + s_c[threadIdx.x] - 1] = j;
    }
}

void rotation(double ra0, double dec0, double (&R)[9])
{
    const double cz = std::cos(-ra0), sz = std::sin(-ra0);
    const double cy = std::cos(dec0), sy = std::sin(dec0);
    const double Rz[9] = {cz, -sz, 0.0, sz, cz, 0.0, 0.0, 0.0, 1.0};
    const double Ry[9] = {cy, 0.0, sy, 0.0, 1.0, 0.0, -sy, 0.0, cy};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += Ry[3 * r + k] * Rz[3 * k + c];
            R[3 * r + c] = s;
        }
}

}  // namespace

// Project one patch and compact its extended galaxies into plan buffers.
// On return: *view is a catalog of the extended galaxies (device arrays owned
// by the plan), core points at the compacted indices of the core galaxies.
int sphere_patch(t3_plan *plan, const t3_sphere_catalog &cat, const t3_patch &p, double theta_max_arcmin,
                 t3_catalog *view, const int32_t **core, int64_t *n_core, hipStream_t s)
{
    const int64_t n = cat.n;
    const int64_t nb = (n + kCompactBlock - 1) / kCompactBlock;
    // workspace: x, y, flag (int32) and h1, h2 (float) per galaxy; compacted
    // x, y, g1, g2, w and core indices; block counts
    T3_TRY(plan->sph_a.reserve(sizeof(int32_t) * 5 * (size_t)n));
    T3_TRY(plan->sph_b.reserve(sizeof(int32_t) * 6 * (size_t)n + sizeof(int32_t) * 4 * (size_t)nb + 64));
    int32_t *px = plan->sph_a.as<int32_t>(), *py = px + n, *pf = py + n;
    float *ph1 = reinterpret_cast<float *>(pf + n), *ph2 = ph1 + n;
    int32_t *cx = plan->sph_b.as<int32_t>(), *cy = cx + n;
    float *cg1 = reinterpret_cast<float *>(cy + n), *cg2 = cg1 + n, *cw = cg2 + n;
    int32_t *cidx = reinterpret_cast<int32_t *>(cw + n);
    int32_t *counts = cidx + n, *offs = counts + 2 * nb;

    SphArgs a{};
    a.ra = cat.ra;
    a.dec = cat.dec;
    a.g1 = cat.g1;
    a.g2 = cat.g2;
    a.w = cat.w;
    a.n = n;
    const double d2r = 3.14159265358979323846 / 180.0;
    rotation(0.5 * (p.ra_lo + p.ra_hi) * d2r, 0.5 * (p.dec_lo + p.dec_hi) * d2r, a.R);
    a.ra_lo = p.ra_lo;
    a.ra_hi = p.ra_hi;
    a.dec_lo = p.dec_lo;
    a.dec_hi = p.dec_hi;
    a.tmax_deg = theta_max_arcmin / 60.0;
    a.inv_unit = 1.0 / plan->unit;
    a.x = px;
    a.y = py;
    a.h1 = ph1;
    a.h2 = ph2;
    a.flag = pf;
    if (n > 0) {
        hipLaunchKernelGGL(k_sphere_project, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
        T3_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(k_sph_count, dim3((unsigned)nb), dim3(kCompactBlock), 0, s, (const int32_t *)pf, n,
                           counts);
        T3_HIP_CHECK(hipGetLastError());
    }
    std::vector<int32_t> hc(2 * (size_t)nb), ho(2 * (size_t)nb);
    if (nb > 0) {
        T3_HIP_CHECK(hipMemcpyAsync(hc.data(), counts, sizeof(int32_t) * hc.size(), hipMemcpyDeviceToHost, s));
        T3_HIP_CHECK(hipStreamSynchronize(s));
    }
    int64_t ne = 0, nc = 0;
    for (int64_t b = 0; b < nb; ++b) {
        ho[2 * b] = (int32_t)ne;
        ho[2 * b + 1] = (int32_t)nc;
        ne += hc[2 * b];
        nc += hc[2 * b + 1];
    }
    if (nb > 0) {
        T3_HIP_CHECK(hipMemcpyAsync(offs, ho.data(), sizeof(int32_t) * ho.size(), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_sph_scatter, dim3((unsigned)nb), dim3(kCompactBlock), 0, s, a, (const int32_t *)offs,
                           cx, cy, cg1, cg2, cw, cidx);
        T3_HIP_CHECK(hipGetLastError());
        // hc/ho must outlive the copy: wait before they go out of scope
        T3_HIP_CHECK(hipStreamSynchronize(s));
    }
    view->n = ne;
    view->x = cx;
    view->y = cy;
    view->g1 = cg1;
    view->g2 = cg2;
    view->w = cw;
    *core = cidx;
    *n_core = nc;
    return T3_OK;
}

}  // namespace t3

namespace t3 {
namespace {
__global__ void k_add(double *dst, const double *src, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] += src[i];
}
}  // namespace

int add_doubles(double *dst, const double *src, size_t n, hipStream_t s)
{
    if (n == 0) return T3_OK;
    hipLaunchKernelGGL(k_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, src, n);
    T3_HIP_CHECK(hipGetLastError());
    return T3_OK;
}

}  // namespace t3
