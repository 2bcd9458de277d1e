// FP64 post-processing of the multipoles.
//  * Normalisation Gamma_{mu,n} = Upsilon_{mu,n} / N_0 (Porth et al. 2023,
//    Sect. 3.4: the mode-coupling matrix is the identity for uniformly
//    distributed tracers).  Bin pairs with N_0 = 0 give 0.
//  * Resummation onto angular bins (eq. Gamma0_binned applied to
//    Gamma(phi) = sum_n Gamma_n e^{i n phi}):
//        Gamma(b1, b2, Phi_k) = sum_{|n| <= n_max} Gamma_n(b1, b2) s_n(Phi_k),
//        s_0 = 1,  s_n = (e^{i n Phi_up} - e^{i n Phi_lo}) / (i n dPhi),
//    negative n from the Appendix A symmetries.
// Also the export of stage-1 chunk planes into a per-centre layout.
#include "t3_internal.h"

namespace t3 {
namespace {

__global__ void k_normalise(const double *ups, int n_sets, int n_max, int B, double *gamma_n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per_mu = (int64_t)(n_max + 1) * B * B;
    const int64_t total = (int64_t)n_sets * 4 * per_mu;
    if (t >= total) return;
    const int64_t set = t / (4 * per_mu);
    const int64_t r = t % (4 * per_mu);
    const int mu = (int)(r / per_mu);
    const int64_t e = r % per_mu;  // n * B * B + b1 * B + b2
    const int64_t bb = e % ((int64_t)B * B);
    const double *u = ups + 2 * (set * 5 * per_mu);
    const double n0 = u[2 * (4 * per_mu + bb)];
    double re = 0.0, im = 0.0;
    if (n0 != 0.0) {
        re = u[2 * (mu * per_mu + e)] / n0;
        im = u[2 * (mu * per_mu + e) + 1] / n0;
    }
    gamma_n[2 * t] = re;
    gamma_n[2 * t + 1] = im;
}

__global__ void k_resum(const double *gamma_n, int n_sets, int n_z, int n_max, int B, int n_phi,
                        double *gamma_phi)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)n_sets * 4 * B * B * n_phi;
    if (t >= total) return;
    const int k = (int)(t % n_phi);
    const int b2 = (int)((t / n_phi) % B);
    const int b1 = (int)((t / ((int64_t)n_phi * B)) % B);
    const int mu = (int)((t / ((int64_t)n_phi * B * B)) % 4);
    const int64_t set = t / ((int64_t)n_phi * B * B * 4);
    const int z3 = (int)(set % n_z), z2 = (int)((set / n_z) % n_z), z1 = (int)(set / ((int64_t)n_z * n_z));
    const int64_t swp = ((int64_t)z1 * n_z + z3) * n_z + z2;
    const int mus = mu == 2 ? 3 : (mu == 3 ? 2 : mu);
    const int64_t per_mu = (int64_t)(n_max + 1) * B * B;
    const double *g = gamma_n + 2 * (set * 4 * per_mu + mu * per_mu);
    const double *gs = gamma_n + 2 * (swp * 4 * per_mu + mus * per_mu);
    const double two_pi = 6.283185307179586476925286766559;
    const double lo = two_pi * k / n_phi, hi = two_pi * (k + 1) / n_phi, d = hi - lo;
    // n = 0
    double re = g[2 * ((int64_t)b1 * B + b2)], im = g[2 * ((int64_t)b1 * B + b2) + 1];
    for (int n = 1; n <= n_max; ++n) {
        for (int sg = -1; sg <= 1; sg += 2) {
            const int nn = sg * n;
            double sh, ch, sl, cl;
            sincos(nn * hi, &sh, &ch);
            sincos(nn * lo, &sl, &cl);
            // s = (e^{i nn hi} - e^{i nn lo}) / (i nn d) = ((sh - sl) - i (ch - cl)) / (nn d)
            const double sr = (sh - sl) / (nn * d), si = -(ch - cl) / (nn * d);
            double gr, gi;
            if (sg > 0) {
                gr = g[2 * ((int64_t)n * B * B + (int64_t)b1 * B + b2)];
                gi = g[2 * ((int64_t)n * B * B + (int64_t)b1 * B + b2) + 1];
            } else {
                gr = gs[2 * ((int64_t)n * B * B + (int64_t)b2 * B + b1)];
                gi = gs[2 * ((int64_t)n * B * B + (int64_t)b2 * B + b1) + 1];
            }
            re += gr * sr - gi * si;
            im += gr * si + gi * sr;
        }
    }
    gamma_phi[2 * t] = re;
    gamma_phi[2 * t + 1] = im;
}

// chunk planes -> G[i][b][m][2], W[i][b][m][2], D[i][b][4][2]
__global__ void k_export(const float *planes, int n_c, int K, int B, int n_max, float *G, float *W,
                         float *D)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n_g = 2 * n_max + 3;
    const int per = n_g + (n_max + 1) + 4;  // complex entries per (i, b)
    if (t >= (int64_t)n_c * B * per) return;
    const int q = (int)(t % per);
    const int b = (int)((t / per) % B);
    const int i = (int)(t / ((int64_t)per * B));
    const int pW = 2 * n_g, pD = 2 * n_g + 2 * (n_max + 1);
    float re, im;
    if (q < n_g) {
        re = planes[chunk_offset(2 * q, i, b, K, B)];
        im = planes[chunk_offset(2 * q + 1, i, b, K, B)];
        float *o = G + 2 * (((int64_t)i * B + b) * n_g + q);
        o[0] = re;
        o[1] = im;
    } else if (q < n_g + n_max + 1) {
        const int m = q - n_g;
        re = planes[chunk_offset(pW + 2 * m, i, b, K, B)];
        im = planes[chunk_offset(pW + 2 * m + 1, i, b, K, B)];
        float *o = W + 2 * (((int64_t)i * B + b) * (n_max + 1) + m);
        o[0] = re;
        o[1] = im;
    } else {
        const int d = q - n_g - (n_max + 1);
        re = planes[chunk_offset(pD + 2 * d, i, b, K, B)];
        im = d < 3 ? planes[chunk_offset(pD + 2 * d + 1, i, b, K, B)] : 0.0f;
        float *o = D + 2 * (((int64_t)i * B + b) * 4 + d);
        o[0] = re;
        o[1] = im;
    }
}

}  // namespace

int normalise_resum(t3_plan *plan, const double *ups, int n_sets, int n_z, int n_phi,
                    double *gamma_n, double *gamma_phi, hipStream_t s)
{
    const int B = plan->B, nm = plan->n_max;
    const int64_t tot = (int64_t)n_sets * 4 * (nm + 1) * B * B;
    hipLaunchKernelGGL(k_normalise, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, ups,
                       n_sets, nm, B, gamma_n);
    T3_HIP_CHECK(hipGetLastError());
    if (gamma_phi) {
        const int64_t tp = (int64_t)n_sets * 4 * B * B * n_phi;
        hipLaunchKernelGGL(k_resum, dim3((unsigned)((tp + 255) / 256)), dim3(256), 0, s,
                           (const double *)gamma_n, n_sets, n_z, nm, B, n_phi, gamma_phi);
        T3_HIP_CHECK(hipGetLastError());
    }
    return T3_OK;
}

int harmonics_export(t3_plan *plan, const CentreSet &cs, const ChunkLayout &L, const float *planes,
                     int64_t c0, int n_c, float *G, float *W, float *D, hipStream_t s)
{
    (void)plan;
    (void)cs;
    if (n_c <= 0) return T3_OK;
    const int n_g = 2 * L.n_max + 3;
    const int per = n_g + (L.n_max + 1) + 4;
    const int64_t tot = (int64_t)n_c * L.B * per;
    hipLaunchKernelGGL(k_export, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, planes, n_c,
                       L.K, L.B, L.n_max, G + 2 * c0 * L.B * n_g, W + 2 * c0 * L.B * (L.n_max + 1),
                       D + 2 * c0 * L.B * 4);
    T3_HIP_CHECK(hipGetLastError());
    return T3_OK;
}

}  // namespace t3
