// FP64 post-processing of the multipoles.
//  * Normalisation Gamma_{mu,n} = Upsilon_{mu,n} / N_0 (Porth et al. 2023,
//    Sect. 3.4: the mode-coupling matrix is the identity for uniformly
//    distributed tracers).  Bin pairs with N_0 = 0 give 0.
//  * Resummation onto angular bins (eq. Gamma0_binned applied to
//    Gamma(phi) = sum_n Gamma_n e^{i n phi}):
//        Gamma(b1, b2, Phi_k) = sum_{|n| <= n_max} Gamma_n(b1, b2) s_n(Phi_k),
//        s_0 = 1,  s_n = (e^{i n Phi_up} - e^{i n Phi_lo}) / (i n dPhi),
//    negative n from the Appendix A symmetries.
//  * Edge correction (eqs. ModeCoupling, GammaMultipolesWithEC): per bin pair
//    the Hermitian Toeplitz system sum_n N_{l-n} Gamma_n = Upsilon_l,
//    |l|, |n| <= n_max, solved by the Levinson recursion in FP64.
//  * x -> centroid projection (eqs. X2Centroid0-3).
// Also the export of stage-1 chunk planes into a per-centre layout.
#include "t3_internal.h"

namespace t3 {
namespace {

// ups: sets of 4 (n_max+1) + w_max + 1 blocks of B x B (Upsilon, then N_n)
__global__ void k_normalise(const double *ups, int n_sets, int n_max, int w_max, int B, double *gamma_n)
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
    const double *u = ups + 2 * (set * (4 * per_mu + (int64_t)(w_max + 1) * B * B));
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

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ double2 cinv(double2 a)
{
    const double d = a.x * a.x + a.y * a.y;
    return make_double2(a.x / d, -a.y / d);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kMCWaves = 4;  // systems (wavefronts) per workgroup

// Edge-corrected multipoles, one wavefront per (set, b1, b2).  With
// L = 2 n_max + 1, indices i = l + n_max, and t_k = N_k(b1, b2) (t_{-k} = t_k^*,
// so T_ij = t_{i-j} is Hermitian Toeplitz), solve T x_mu = y_mu for the four
// components, y_mu[i] = Upsilon_{mu, i - n_max}(b1, b2) (negative orders from
// the swapped set and bins).  Levinson recursion: forward / backward vectors
// f, b of the leading n x n block (T f = e_first, T b = e_last) grow one
// order at a time,
//   ef = sum_{j<n} t_{n-j} f_j,  eb = sum_{j<n} t_{-(j+1)} b_j,
//   f' = ([f;0] - ef [0;b]) / (1 - ef eb),  b' = ([0;b] - eb [f;0]) / (1 - ef eb),
//   x' = [x;0] + (y_n - sum_{j<n} t_{n-j} x_j) b'.
// Dynamic LDS per wavefront: f, b, x[4] of L entries and t_k, k = 0..L-1.
__global__ __launch_bounds__(64 * kMCWaves) void k_mode_couple(const double *ups, int n_sets, int n_z, int n_max,
                                                               int w_max, int B, double *gamma_n)
{
    extern __shared__ double2 mc_lds[];
    const int L = 2 * n_max + 1;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t sys = (int64_t)blockIdx.x * kMCWaves + wv;
    if (sys >= (int64_t)n_sets * B * B) return;  // whole wavefront
    double2 *f = mc_lds + (size_t)wv * 7 * L;
    double2 *bv = f + L;
    double2 *x = bv + L;  // [4][L]
    double2 *tk = x + 4 * L;
    const int b2 = (int)(sys % B), b1 = (int)((sys / B) % B);
    const int64_t set = sys / ((int64_t)B * B);
    const int z3 = (int)(set % n_z), z2 = (int)((set / n_z) % n_z), z1 = (int)(set / ((int64_t)n_z * n_z));
    const int64_t swp = ((int64_t)z1 * n_z + z3) * n_z + z2;
    const int64_t bb = (int64_t)B * B;
    const int64_t per_set = (int64_t)(4 * (n_max + 1) + w_max + 1) * bb;
    const double *u = ups + 2 * set * per_set;
    const double *us = ups + 2 * swp * per_set;
    const double *nb = u + 2 * (4 * (int64_t)(n_max + 1) * bb);  // N blocks of this set
    for (int k = lane; k < L; k += 64) {
        const double *p = nb + 2 * ((int64_t)k * bb + (int64_t)b1 * B + b2);
        tk[k] = make_double2(p[0], p[1]);
    }
    wave_sync();
    auto t_at = [&](int k) -> double2 {  // t_k for |k| <= L - 1
        const double2 v = tk[k < 0 ? -k : k];
        return k < 0 ? make_double2(v.x, -v.y) : v;
    };
    auto y_at = [&](int mu, int i) -> double2 {  // Upsilon_{mu, i - n_max}(b1, b2)
        const int l = i - n_max;
        if (l >= 0) {
            const double *p = u + 2 * (((int64_t)mu * (n_max + 1) + l) * bb + (int64_t)b1 * B + b2);
            return make_double2(p[0], p[1]);
        }
        const int mus = mu == 2 ? 3 : (mu == 3 ? 2 : mu);
        const double *p = us + 2 * (((int64_t)mus * (n_max + 1) - l) * bb + (int64_t)b2 * B + b1);
        return make_double2(p[0], p[1]);
    };
    const double t0 = tk[0].x;
    double *g = gamma_n + 2 * set * 4 * (int64_t)(n_max + 1) * bb;
    if (!(t0 != 0.0)) {
        for (int e = lane; e < 4 * (n_max + 1); e += 64) {
            double *o = g + 2 * ((int64_t)e * bb + (int64_t)b1 * B + b2);
            o[0] = 0.0;
            o[1] = 0.0;
        }
        return;
    }
    if (lane == 0) {
        f[0] = make_double2(1.0 / t0, 0.0);
        bv[0] = f[0];
        for (int mu = 0; mu < 4; ++mu) {
            const double2 y0 = y_at(mu, 0);
            x[mu * L] = make_double2(y0.x / t0, y0.y / t0);
        }
    }
    wave_sync();
    for (int n = 1; n < L; ++n) {
        // inner products over j < n (each lane a strided share, then a wave sum)
        double2 ef = make_double2(0, 0), eb = make_double2(0, 0), ex[4];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) ex[mu] = make_double2(0, 0);
        for (int j = lane; j < n; j += 64) {
            const double2 tn = t_at(n - j);
            const double2 a = cmul(tn, f[j]), c = cmul(t_at(-(j + 1)), bv[j]);
            ef.x += a.x;
            ef.y += a.y;
            eb.x += c.x;
            eb.y += c.y;
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) {
                const double2 d = cmul(tn, x[mu * L + j]);
                ex[mu].x += d.x;
                ex[mu].y += d.y;
            }
        }
        ef = make_double2(wave_sum(ef.x), wave_sum(ef.y));
        eb = make_double2(wave_sum(eb.x), wave_sum(eb.y));
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) ex[mu] = make_double2(wave_sum(ex[mu].x), wave_sum(ex[mu].y));
        const double2 efeb = cmul(ef, eb);
        const double2 inv = cinv(make_double2(1.0 - efeb.x, -efeb.y));
        double2 r[4];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const double2 y = y_at(mu, n);
            r[mu] = make_double2(y.x - ex[mu].x, y.y - ex[mu].y);
        }
        // new f, b of length n + 1: read every old entry before any write
        double2 nf[3], nbv[3];
        int cnt = 0;
        for (int j = lane; j <= n; j += 64, ++cnt) {
            const double2 fo = j < n ? f[j] : make_double2(0, 0);
            const double2 bo = j >= 1 ? bv[j - 1] : make_double2(0, 0);
            const double2 p = cmul(ef, bo), q = cmul(eb, fo);
            nf[cnt] = cmul(make_double2(fo.x - p.x, fo.y - p.y), inv);
            nbv[cnt] = cmul(make_double2(bo.x - q.x, bo.y - q.y), inv);
        }
        wave_sync();
        cnt = 0;
        for (int j = lane; j <= n; j += 64, ++cnt) {
            f[j] = nf[cnt];
            bv[j] = nbv[cnt];
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) {
                const double2 xo = j < n ? x[mu * L + j] : make_double2(0, 0);
                const double2 d = cmul(r[mu], nbv[cnt]);
                x[mu * L + j] = make_double2(xo.x + d.x, xo.y + d.y);
            }
        }
        wave_sync();
    }
    // Gamma_{mu,n} for n = 0..n_max (index i = n + n_max)
    for (int e = lane; e < 4 * (n_max + 1); e += 64) {
        const int mu = e / (n_max + 1), nn = e % (n_max + 1);
        const double2 v = x[mu * L + nn + n_max];
        double *o = g + 2 * ((int64_t)e * bb + (int64_t)b1 * B + b2);
        o[0] = v.x;
        o[1] = v.y;
    }
}

struct CentroidArgs {
    double theta[kMaxRadialBins];  // representative radius per bin (any unit: only ratios matter)
    int B, n_phi;
    int64_t total;     // n_sets * 4 * B * B * n_phi
};

// x -> centroid projection of Gamma(b1, b2, Phi_k) at (theta[b1], theta[b2],
// phi_k = 2 pi (k + 1/2) / n_phi):
//   A1 = (t1 + t2 e^{-i phi}) / (t1 + t2 e^{i phi})
//   A2 = (t2 e^{-i phi} - 2 t1) / (t2 e^{i phi} - 2 t1)
//   A3 = (t1 - 2 t2 e^{-i phi}) / (t1 - 2 t2 e^{i phi})
//   factors: mu = 0: A1 A2 A3 e^{3i phi}, 1: A2 A3 / A1 e^{i phi},
//            2: A1 A3 / A2 e^{3i phi}, 3: A1 A2 / A3 e^{-i phi};
// 0 where a denominator is exactly zero.
__global__ void k_centroid(const double *in, double *out, CentroidArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.total) return;
    const int k = (int)(t % a.n_phi);
    const int b2 = (int)((t / a.n_phi) % a.B);
    const int b1 = (int)((t / ((int64_t)a.n_phi * a.B)) % a.B);
    const int mu = (int)((t / ((int64_t)a.n_phi * a.B * a.B)) % 4);
    const double t1 = a.theta[b1], t2 = a.theta[b2];
    const double two_pi = 6.283185307179586476925286766559;
    double s, c;
    sincos(two_pi * (k + 0.5) / a.n_phi, &s, &c);
    const double2 e = make_double2(c, s), ec = make_double2(c, -s);
    const double2 n1 = make_double2(t1 + t2 * ec.x, t2 * ec.y), d1 = make_double2(t1 + t2 * e.x, t2 * e.y);
    const double2 n2 = make_double2(t2 * ec.x - 2.0 * t1, t2 * ec.y), d2 = make_double2(t2 * e.x - 2.0 * t1, t2 * e.y);
    const double2 n3 = make_double2(t1 - 2.0 * t2 * ec.x, -2.0 * t2 * ec.y),
                  d3 = make_double2(t1 - 2.0 * t2 * e.x, -2.0 * t2 * e.y);
    const bool bad = (d1.x == 0.0 && d1.y == 0.0) || (d2.x == 0.0 && d2.y == 0.0) || (d3.x == 0.0 && d3.y == 0.0);
    double2 fac = make_double2(0.0, 0.0);
    if (!bad) {
        const double2 A1 = cmul(n1, cinv(d1)), A2 = cmul(n2, cinv(d2)), A3 = cmul(n3, cinv(d3));
        const double2 e2 = cmul(e, e), e3 = cmul(e2, e);
        switch (mu) {
            case 0: fac = cmul(cmul(cmul(A1, A2), A3), e3); break;
            case 1: fac = cmul(cmul(cmul(A2, A3), cinv(A1)), e); break;
            case 2: fac = cmul(cmul(cmul(A1, A3), cinv(A2)), e3); break;
            default: fac = cmul(cmul(cmul(A1, A2), cinv(A3)), ec); break;
        }
    }
    const double2 v = make_double2(in[2 * t], in[2 * t + 1]);
    const double2 r = cmul(v, fac);
    out[2 * t] = r.x;
    out[2 * t + 1] = r.y;
}

// chunk planes -> G[i][b][m][2], W[i][b][m][2], D[i][b][4][2]
__global__ void k_export(const float *planes, int n_c, int K, int B, int n_max, int w_max, float *G, float *W,
                         float *D)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n_g = 2 * n_max + 3;
    const int per = n_g + (n_max + 1) + 4;  // complex entries per (i, b)
    if (t >= (int64_t)n_c * B * per) return;
    const int q = (int)(t % per);
    const int b = (int)((t / per) % B);
    const int i = (int)(t / ((int64_t)per * B));
    const int pW = 2 * n_g, pD = 2 * n_g + 2 * (w_max + 1);
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
    if (plan->flags & T3_FLAG_EDGE_CORRECT) {
        const int64_t systems = (int64_t)n_sets * B * B;
        const size_t lds = sizeof(double2) * 7 * (size_t)(2 * nm + 1) * kMCWaves;
        hipLaunchKernelGGL(k_mode_couple, dim3((unsigned)((systems + kMCWaves - 1) / kMCWaves)),
                           dim3(64 * kMCWaves), lds, s, ups, n_sets, n_z, nm, plan->w_max, B, gamma_n);
    } else {
        const int64_t tot = (int64_t)n_sets * 4 * (nm + 1) * B * B;
        hipLaunchKernelGGL(k_normalise, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, ups,
                           n_sets, nm, plan->w_max, B, gamma_n);
    }
    T3_HIP_CHECK(hipGetLastError());
    if (gamma_phi) {
        const int64_t tp = (int64_t)n_sets * 4 * B * B * n_phi;
        hipLaunchKernelGGL(k_resum, dim3((unsigned)((tp + 255) / 256)), dim3(256), 0, s,
                           (const double *)gamma_n, n_sets, n_z, nm, B, n_phi, gamma_phi);
        T3_HIP_CHECK(hipGetLastError());
    }
    return T3_OK;
}

int x_to_centroid(t3_plan *plan, const double *in, int n_sets, int n_phi, const double *theta, double *out,
                  hipStream_t s)
{
    CentroidArgs a{};
    a.B = plan->B;
    a.n_phi = n_phi;
    a.total = (int64_t)n_sets * 4 * plan->B * plan->B * n_phi;
    for (int b = 0; b < plan->B; ++b)
        a.theta[b] = theta ? theta[b] : 0.5 * (plan->edges_lat[b] + plan->edges_lat[b + 1]);
    if (a.total == 0) return T3_OK;
    hipLaunchKernelGGL(k_centroid, dim3((unsigned)((a.total + 255) / 256)), dim3(256), 0, s, in, out, a);
    T3_HIP_CHECK(hipGetLastError());
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
                       L.K, L.B, L.n_max, L.w_max, G + 2 * c0 * L.B * n_g, W + 2 * c0 * L.B * (L.n_max + 1),
                       D + 2 * c0 * L.B * 4);
    T3_HIP_CHECK(hipGetLastError());
    return T3_OK;
}

}  // namespace t3
