// Third-order aperture statistics from the centroid-projected 3PCF
// (Porth et al. 2023, Sect. 4 and Appendix C), FP64.
//
// For aperture radii (theta_1, theta_2, theta_3) the four complex correlators
//     C_mu = int dvartheta_1 dvartheta_2 dphi  Gamma_mu^cent F_mu,
// C_0 = <M^3>, C_1 = <M* M^2>, C_2 = <M M* M>, C_3 = <M^2 M*>
// (eqs. MFrom3pcfTheory, MFrom3pcfTheoryb), are evaluated by the midpoint
// rule on the estimator's bins (radial bin centres and widths, angular bin
// centres), and the eight real statistics follow from eqs. MapTrafo8_1-8.
//
// Filters (Appendix C): with q_k the centroid-to-vertex vectors of the
// triangle (vertex 1 at the origin, vertex 2 at vartheta_1 on the x axis,
// vertex 3 at vartheta_2 e^{i phi}), Theta^2, S, M, Z, f_k, g_k as defined
// there, F_0 as printed, and the filter of component mu (conjugate at
// vertex mu) the printed F_1 with its indices rotated so that its
// distinguished index (printed 2) is mu -- the assignment that a direct
// integration of a single triangle against three apertures gives.
#include "t3_internal.h"

namespace t3 {
namespace {

struct cd {
    double x, y;
};
__device__ __forceinline__ cd operator+(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cd operator*(cd a, cd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cd operator*(double s, cd a) { return {s * a.x, s * a.y}; }
__device__ __forceinline__ cd cj(cd a) { return {a.x, -a.y}; }
__device__ __forceinline__ double n2(cd a) { return a.x * a.x + a.y * a.y; }

constexpr int kApPerLaunch = 64;  // aperture triples passed by value per launch

struct ApArgs {
    const double *gam;   // [n_sets][4][B][B][K][2]
    double *corr;        // [n_sets][n_ap][4][2]
    double *stats;       // [n_sets][n_ap][8] or null
    int B, K, n_ap, ap0;  // ap0: index of this launch's first triple
    double centre[kMaxRadialBins], width[kMaxRadialBins];  // radial bins, arcmin
    double ap[kApPerLaunch][3];    // aperture radii, arcmin
};

constexpr int kApThreads = 256;

// F_0..F_3 at one triangle for aperture radii th[3]; false for a
// degenerate triangle (a vanishing centroid-to-vertex vector).
__device__ bool ap_filters(double t1, double t2, double phi, const double (&th)[3], cd (&F)[4])
{
    double s, c;
    sincos(phi, &s, &c);
    const cd v1{t1, 0.0}, v2{t2 * c, t2 * s};
    const cd q[3] = {(-1.0 / 3.0) * (v1 + v2), (1.0 / 3.0) * (2.0 * v1 - v2), (1.0 / 3.0) * (2.0 * v2 - v1)};
    double aq[3];
    for (int k = 0; k < 3; ++k) aq[k] = n2(q[k]);
    if (aq[0] == 0.0 || aq[1] == 0.0 || aq[2] == 0.0) return false;
    double t2s[3];
    for (int k = 0; k < 3; ++k) t2s[k] = th[k] * th[k];
    const double T2 = sqrt((t2s[0] * t2s[1] + t2s[0] * t2s[2] + t2s[1] * t2s[2]) / 3.0);  // Theta^2
    const double T4 = T2 * T2, T6 = T4 * T2;
    const double S = t2s[0] * t2s[1] * t2s[2] / T6;
    const double Mf = S * t1 * t2 / (2.0 * 3.14159265358979323846 * T4);
    double Z = 0.0;
    cd f[3], g[3];
    for (int k = 0; k < 3; ++k) {
        const int a = (k + 1) % 3, b = (k + 2) % 3;
        Z += (-t2s[k] + 2.0 * t2s[a] + 2.0 * t2s[b]) * aq[k];
        const cd r = (1.0 / aq[k]) * (cj(q[k]) * (q[a] - q[b]));
        f[k] = cd{(t2s[a] + t2s[b]) / (2.0 * T2), 0.0} + ((t2s[a] - t2s[b]) / (6.0 * T2)) * r;
        g[k] = cd{t2s[a] * t2s[b] / T4, 0.0} + (t2s[k] * (t2s[b] - t2s[a]) / (3.0 * T4)) * r;
    }
    Z /= 6.0 * T4;
    const double ez = exp(-Z);
    const double P = aq[0] * aq[1] * aq[2];
    const cd cf0 = cj(f[0]), cf1 = cj(f[1]), cf2 = cj(f[2]);
    F[0] = (Mf / 24.0 * P / T6 * ez) * (cf0 * cf0 * cf1 * cf1 * cf2 * cf2);
    for (int mu = 1; mu <= 3; ++mu) {
        const int b = mu - 1, a = (b + 2) % 3, cc = (b + 1) % 3;  // slots 1, 2, 3 of the printed F_1
        const cd fa = cj(f[a]), fc = cj(f[cc]), fb = f[b], gb = cj(g[b]);
        const cd qb2 = cj(q[b]) * cj(q[b]);
        const cd qcqa = q[cc] * q[a];
        cd term = (P / (24.0 * T6)) * (fc * fc * fa * fa * fb * fb);
        term = term - (1.0 / (9.0 * T4)) * (qcqa * qb2 * fc * fa * fb * gb);
        const cd inner = (1.0 / (P * T2)) * (qcqa * qcqa * qb2 * qb2 * gb * gb) +
                         (2.0 * t2s[cc] * t2s[a] / (T4 * aq[b] * T2)) * (qcqa * qb2 * fc * fa);
        term = term + (1.0 / 27.0) * inner;
        F[mu] = (Mf * ez) * term;
    }
    return true;
}

__global__ __launch_bounds__(kApThreads) void k_aperture(ApArgs a)
{
    const int il = blockIdx.x, set = blockIdx.y;
    const int ia = a.ap0 + il;
    const double th[3] = {a.ap[il][0], a.ap[il][1], a.ap[il][2]};
    const int B = a.B, K = a.K;
    const double dphi = 6.283185307179586476925286766559 / K;
    const int64_t per_mu = (int64_t)B * B * K;
    const double *g = a.gam + 2 * (int64_t)set * 4 * per_mu;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t t = threadIdx.x; t < per_mu; t += kApThreads) {
        const int k = (int)(t % K);
        const int b2 = (int)((t / K) % B), b1 = (int)(t / ((int64_t)K * B));
        cd F[4];
        if (!ap_filters(a.centre[b1], a.centre[b2], (k + 0.5) * dphi, th, F)) continue;
        const double w = a.width[b1] * a.width[b2] * dphi;
        for (int mu = 0; mu < 4; ++mu) {
            const cd v{g[2 * (mu * per_mu + t)], g[2 * (mu * per_mu + t) + 1]};
            const cd p = v * F[mu];
            acc[2 * mu] += w * p.x;
            acc[2 * mu + 1] += w * p.y;
        }
    }
    __shared__ double red[8][kApThreads];
    for (int j = 0; j < 8; ++j) red[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int s = kApThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int j = 0; j < 8; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *o = a.corr + 8 * ((int64_t)set * a.n_ap + ia);
        for (int j = 0; j < 8; ++j) o[j] = red[j][0];
        if (a.stats) {
            // C_0 = <M^3>, C_1 = <M* M^2>, C_2 = <M M* M>, C_3 = <M^2 M*>
            const double r0 = red[0][0], i0 = red[1][0], r1 = red[2][0], i1 = red[3][0];
            const double r2 = red[4][0], i2 = red[5][0], r3 = red[6][0], i3 = red[7][0];
            double *st = a.stats + 8 * ((int64_t)set * a.n_ap + ia);
            st[0] = (r3 + r2 + r1 + r0) / 4;   // <Map^3>
            st[1] = (i3 + i2 - i1 + i0) / 4;   // <Mx Map^2>
            st[2] = (i3 - i2 + i1 + i0) / 4;   // <Map Mx Map>
            st[3] = (-i3 + i2 + i1 + i0) / 4;  // <Map^2 Mx>
            st[4] = (r3 + r2 - r1 - r0) / 4;   // <Map Mx^2>
            st[5] = (r3 - r2 + r1 - r0) / 4;   // <Mx Map Mx>
            st[6] = (-r3 + r2 + r1 - r0) / 4;  // <Mx^2 Map>
            st[7] = (i3 + i2 + i1 - i0) / 4;   // <Mx^3>
        }
    }
}

}  // namespace

int aperture_stats(t3_plan *plan, const double *gamma_cent, int n_sets, int n_phi, const double *apertures,
                   int n_ap, double *corr, double *stats, hipStream_t s)
{
    ApArgs a{};
    a.gam = gamma_cent;
    a.corr = corr;
    a.stats = stats;
    a.B = plan->B;
    a.K = n_phi;
    a.n_ap = n_ap;
    for (int b = 0; b < plan->B; ++b) {
        const double lo = plan->edges_lat[b] * plan->unit, hi = plan->edges_lat[b + 1] * plan->unit;
        a.centre[b] = 0.5 * (lo + hi);
        a.width[b] = hi - lo;
    }
    for (int a0 = 0; a0 < n_ap; a0 += kApPerLaunch) {
        const int cnt = n_ap - a0 < kApPerLaunch ? n_ap - a0 : kApPerLaunch;
        a.ap0 = a0;
        for (int j = 0; j < cnt; ++j)
            for (int k = 0; k < 3; ++k) a.ap[j][k] = apertures[3 * (a0 + j) + k];
        hipLaunchKernelGGL(k_aperture, dim3((unsigned)cnt, (unsigned)n_sets), dim3(kApThreads), 0, s, a);
        T3_HIP_CHECK(hipGetLastError());
    }
    return T3_OK;
}

}  // namespace t3
