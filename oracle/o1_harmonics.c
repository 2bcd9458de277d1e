/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code with the HIP path.
 *
 * Plain FP64 per-centre harmonic sums of the discrete multipole estimator
 * of the shear three-point function (Porth et al. 2023, Sect. 3.1):
 *
 *   G_m(i; b) = sum_k w_k gamma_k e^{i m phi_ik} B(theta_ik in bin b)   (eq. Gn_disc)
 *   W_m(i; b) = sum_k w_k         e^{i m phi_ik} B(theta_ik in bin b)   (W_n^disc, eq. 3PCF_Normalization)
 *
 * plus the four sums over single neighbours that the product of two G's
 * (or two W's) contains when both neighbours are the same galaxy (j = k):
 *
 *   D6 = sum_k c_k^2  e^{-6 i phi}    (enters Upsilon_0)
 *   D2 = sum_k c_k^2  e^{-2 i phi}    (enters Upsilon_1)
 *   DA = sum_k |c_k|^2 e^{-2 i phi}   (enters Upsilon_2 and Upsilon_3)
 *   DW = sum_k w_k^2                  (enters N)
 * with c_k = w_k gamma_k.
 *
 * Neighbour search is a plain loop over every galaxy (no spatial index).
 * Bin membership is half-open: e_b <= theta < e_{b+1}, decided by
 * comparing the exact squared separation (positions are lattice integers
 * held in doubles, so dx*dx + dy*dy is exact below 2^53) with the squared
 * edges given in the same lattice units.
 * e^{i m phi} is the m-th power of the unit vector z = (dx + i dy)/r,
 * formed by repeated multiplication; negative powers are conjugates.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Number of OpenMP threads the oracle uses. */
int o1_threads(void)
{
    return omp_get_max_threads();
}

/* Threads for later calls from the calling thread (n >= 1). */
void o1_set_threads(int n)
{
    if (n >= 1) omp_set_num_threads(n);
}

static int find_bin(double r2, int n_bins, const double *e2)
{
    if (!(r2 >= e2[0]) || !(r2 < e2[n_bins]))
        return -1;
    for (int b = 0; b < n_bins; ++b)
        if (r2 >= e2[b] && r2 < e2[b + 1])
            return b;
    return -1;
}

/*
 * Centres (cx, cy) against a neighbour catalog (nx, ny, g1, g2, w).
 * Orders: G for m in [m_lo, m_hi]; W for m in [-w_max, w_max].
 * Output layouts (row-major, complex as interleaved re/im doubles):
 *   G[n_c][n_bins][m_hi - m_lo + 1][2]
 *   W[n_c][n_bins][2 w_max + 1][2]
 *   D[n_c][n_bins][4][2]   (D6, D2, DA, DW)
 *   npairs[n_c]            in-range (centre, neighbour) pairs
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int o1_harmonics(int64_t n_c, const double *cx, const double *cy,
                 int64_t n_nb, const double *nx, const double *ny,
                 const double *g1, const double *g2, const double *w,
                 int n_bins, const double *e2,
                 int m_lo, int m_hi, int w_max,
                 double *G, double *W, double *D, int64_t *npairs)
{
    if (n_c < 0 || n_nb < 0 || n_bins < 1 || m_hi < m_lo || w_max < 0)
        return -1;
    const int n_g = m_hi - m_lo + 1;
    const int n_w = 2 * w_max + 1;
    int p_max = w_max;
    if (-m_lo > p_max) p_max = -m_lo;
    if (m_hi > p_max) p_max = m_hi;
    if (6 > p_max) p_max = 6;
    int fail = 0;

#pragma omp parallel
    {
        double complex *zp = malloc(sizeof(double complex) * (size_t)(2 * p_max + 1));
        double complex *Gi = malloc(sizeof(double complex) * (size_t)n_bins * n_g);
        double complex *Wi = malloc(sizeof(double complex) * (size_t)n_bins * n_w);
        double complex *Di = malloc(sizeof(double complex) * (size_t)n_bins * 4);
        if (!zp || !Gi || !Wi || !Di) {
#pragma omp atomic write
            fail = 1;
        } else {
            double complex *zpow = zp + p_max; /* zpow[m], m in [-p_max, p_max] */
#pragma omp for schedule(dynamic, 4)
            for (int64_t i = 0; i < n_c; ++i) {
                memset(Gi, 0, sizeof(double complex) * (size_t)n_bins * n_g);
                memset(Wi, 0, sizeof(double complex) * (size_t)n_bins * n_w);
                memset(Di, 0, sizeof(double complex) * (size_t)n_bins * 4);
                int64_t np = 0;
                for (int64_t k = 0; k < n_nb; ++k) {
                    double dx = nx[k] - cx[i];
                    double dy = ny[k] - cy[i];
                    double r2 = dx * dx + dy * dy;
                    int b = find_bin(r2, n_bins, e2);
                    if (b < 0)
                        continue;
                    ++np;
                    double r = sqrt(r2);
                    double complex z = dx / r + I * (dy / r);
                    zpow[0] = 1.0;
                    for (int m = 1; m <= p_max; ++m) {
                        zpow[m] = zpow[m - 1] * z;
                        zpow[-m] = conj(zpow[m]);
                    }
                    double complex c = w[k] * (g1[k] + I * g2[k]);
                    double complex *Gb = Gi + (size_t)b * n_g;
                    double complex *Wb = Wi + (size_t)b * n_w;
                    for (int m = m_lo; m <= m_hi; ++m)
                        Gb[m - m_lo] += c * zpow[m];
                    for (int m = -w_max; m <= w_max; ++m)
                        Wb[m + w_max] += w[k] * zpow[m];
                    double complex *Db = Di + (size_t)b * 4;
                    Db[0] += c * c * zpow[-6];
                    Db[1] += c * c * zpow[-2];
                    Db[2] += (creal(c) * creal(c) + cimag(c) * cimag(c)) * zpow[-2];
                    Db[3] += w[k] * w[k];
                }
                double *Go = G + (size_t)i * n_bins * n_g * 2;
                double *Wo = W + (size_t)i * n_bins * n_w * 2;
                double *Do = D + (size_t)i * n_bins * 4 * 2;
                for (size_t t = 0; t < (size_t)n_bins * n_g; ++t) {
                    Go[2 * t] = creal(Gi[t]);
                    Go[2 * t + 1] = cimag(Gi[t]);
                }
                for (size_t t = 0; t < (size_t)n_bins * n_w; ++t) {
                    Wo[2 * t] = creal(Wi[t]);
                    Wo[2 * t + 1] = cimag(Wi[t]);
                }
                for (size_t t = 0; t < (size_t)n_bins * 4; ++t) {
                    Do[2 * t] = creal(Di[t]);
                    Do[2 * t + 1] = cimag(Di[t]);
                }
                npairs[i] = np;
            }
        }
        free(zp);
        free(Gi);
        free(Wi);
        free(Di);
    }
    return fail ? -1 : 0;
}
