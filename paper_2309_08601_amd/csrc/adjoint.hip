// Hand-written adjoint of the multipole estimator (reverse mode through
// stage 2 and stage 1, recomputing the harmonic sums instead of storing them).
//
// Gradient convention for a real loss L and a complex quantity u = a + i b:
//     grad u = dL/da + i dL/db.
// Then a holomorphic map v = f(u) gives grad u = conj(f'(u)) grad v, and
// v = conj(u) gives grad u = conj(grad v).
//
// Forward (Porth et al. 2023, eqs. Upsilon0_Derivation, Upsilon1-3,
// 3PCF_Normalization): for each (mu, n),
//     Upsilon(b1, b2) = sum_i alpha_i [X_i(b1) Y_i(b2) - [b1 == b2] D_i(b1)]
// with (alpha, X, Y, D) = (-c, G_{n-3}, G_{-n-3}, D6), (-c*, G_{n-1}, G_{-n-1}, D2),
// (-c, G*_{-n-1}, G_{-n-3}, DA), (-c, G_{n-3}, G*_{n-1}, DA), (w, W_n, W_n*, DW).
// Reverse, per centre i (given Ub = grad Upsilon):
//     grad X(b1)  = conj(alpha) sum_b2 Ub(b1, b2) conj(Y(b2))
//     grad Y(b2)  = conj(alpha) sum_b1 Ub(b1, b2) conj(X(b1))
//     grad alpha  = sum_b1 conj(X(b1)) sum_b2 Ub conj(Y(b2)) - sum_b conj(D(b)) Ub(b, b)
//     grad D(b)   = -conj(alpha) Ub(b, b)
// accumulated over (mu, n) into Gb_m(i, b), Wb_m(i, b) and the j = k sums.
// Then every neighbour j of i in bin b (z = e^{i phi_ij}, p_m = z^m):
//     G_m  = sum_j c_j p_m       ->  grad c_j += sum_m conj(p_m) Gb_m
//     W_m  = sum_j w_j p_m       ->  grad w_j += sum_m Re(conj(p_m) Wb_m)
//     D6   = sum_j c_j^2 conj(p_6)  ->  grad c_j += 2 conj(c_j) p_6 D6b
//     D2   = sum_j c_j^2 conj(p_2)  ->  grad c_j += 2 conj(c_j) p_2 D2b
//     DA   = sum_j |c_j|^2 conj(p_2) -> grad c_j += 2 c_j Re(DAb p_2)
//     DW   = sum_j w_j^2            ->  grad w_j += 2 w_j Re(DWb)
// The +-m orders share p_m: conj(p) a + p b = Re p (a + b) + Im p i (b - a),
// so each lane needs 4 FMAs per order pair with per-(centre, bin)
// coefficients s_m = Gb_m + Gb_{-m}, d_m = i (Gb_{-m} - Gb_m) that are uniform
// across the wavefront (read from LDS).  The centre factors give
//     grad c_i += -grad alpha_0 - conj(grad alpha_1) - grad alpha_2 - grad alpha_3,
//     grad w_i += Re grad alpha_4,
// and finally c = w gamma: grad gamma = w grad c, grad w += Re(conj(gamma) grad c).
//
// The transpose scan walks the same annuli as the forward scan (sweep.h),
// every lane one neighbour, and adds its three gradient terms with
// hardware FP32 atomics into per-galaxy buffers (summation order therefore
// varies between runs at the level of FP32 rounding).  In deterministic mode
// the terms are rounded to 64-bit fixed point instead -- scale 2^e per
// centre chunk with e set from a bound on the chunk's largest term, so that
// no sum can overflow -- and added with integer atomics, which are
// associative; the chunks are then summed in FP64 in chunk order.
#include "sweep.h"

namespace t3 {
namespace {

constexpr int kWaves = 4;

// Coefficient block of one (centre, bin) for a compiled order capacity C:
//   [0, 4M)       m = 1..M (M = C + 3): s_m re, s_m im, d_m re, d_m im
//   [4M, 4M+2)    Gb_0
//   next 2(C+1)   Wb_m, m = 0..C
//   next 7        D6b (2), D2b (2), DAb (2), DWb (1)
__host__ __device__ constexpr int coef_size(int C) { return 4 * (C + 3) + 2 + 2 * (C + 1) + 7; }

struct CoefArgs {
    const float *planes;   // stage-1 chunk planes
    const float4 *ccw;     // centre factors (chunk-relative)
    const double *gups;    // grad Upsilon [5][n_max+1][B][B][2]
    int n_c, K, B, n_max, cap, jk;
    float *coef;           // [n_c][B][coef_size(cap)]
    float2 *cen_gc;        // [n_c] centre part of grad c (chunk-relative)
    float *cen_gw;         // [n_c] centre part of grad w
    unsigned *coef_max;    // deterministic mode: largest |coefficient| of the chunk (float bits); else null
};

// Deterministic mode: exponent e of the fixed-point scale 2^e of one chunk.
// A pair's three terms are each at most (1 + 4 cmax) times the sum of the
// absolute entries of the centre's coefficient block (|z^m| = 1, cmax =
// max(1, |Re c| + |Im c|, w) over the catalog), a galaxy receives at most one
// pair term per centre, so every per-galaxy sum is below
// n_c * coef_size * max|coef| * 8 cmax = bound < 2^ex, and with e = 61 - ex
// the scaled sums stay below 2^61.
__device__ __forceinline__ int det_exponent(const unsigned *hdr, int n_c, int cs)
{
    const double mc = (double)__uint_as_float(hdr[0]);
    const double cm = (double)__uint_as_float(hdr[1]);
    const double bound = mc * (double)cs * 8.0 * cm * (double)n_c;
    if (!(bound > 0.0)) return 0;
    int ex = 0;
    (void)frexp(bound, &ex);
    return 61 - ex;
}

// One wavefront per centre.  The operands (FP32 planes) and the gradient
// accumulators of the harmonics (a few terms each, stored as FP32
// coefficients) are FP32 in LDS, 8 B (3 n_max + 8) per bin, so that LDS
// leaves about four workgroups per SIMD; products and the sums over bins are
// FP64.
__global__ __launch_bounds__(64) void k_adj_coef(CoefArgs a)
{
    extern __shared__ float2 sm[];
    const int B = a.B, nm = a.n_max;
    const int n_g = 2 * nm + 3;
    float2 *Gb = sm;                      // [B][n_g]   index m + nm + 3
    float2 *Wb = Gb + B * n_g;            // [B][nm+1]
    float2 *Db = Wb + B * (nm + 1);       // [B][4]
    float2 *Xs = Db + B * 4;              // [kMaxRadialBins]
    float2 *Ys = Xs + kMaxRadialBins;     // [kMaxRadialBins]
    const int lane = threadIdx.x;
    const int i = blockIdx.x;
    if (i >= a.n_c) return;
    const int K = a.K;
    for (int t = lane; t < B * (n_g + nm + 1 + 4); t += 64) sm[t] = make_float2(0.0f, 0.0f);

    const float4 f = a.ccw[i];
    const double cr = f.x, ci = f.y, w = f.z;
    // alpha per mu
    const double al_r[5] = {-cr, -cr, -cr, -cr, w};
    const double al_i[5] = {-ci, ci, -ci, -ci, 0.0};
    double ga_r[5] = {0, 0, 0, 0, 0}, ga_i[5] = {0, 0, 0, 0, 0};  // grad alpha (lanes 0..B-1 partials)
    __syncthreads();

    const bool side_y = lane >= 32;   // lanes 32.. compute grad Y, bins (lane & 31) + 32 g
    const size_t pstr = (size_t)(nm + 1) * B * B;
    // (mu, n) -> operand orders and planes; xs/ys = 1 when the operand is conjugated
    auto orders = [&](int it, int &mu, int &n, int &xm, int &ym, int &xs, int &ys, int &pxr, int &pyr) {
        mu = it / (nm + 1);
        n = it - mu * (nm + 1);
        xs = 0;
        ys = 0;
        switch (mu) {
            case 0: xm = n - 3; ym = -n - 3; break;
            case 1: xm = n - 1; ym = -n - 1; break;
            case 2: xm = -n - 1; ym = -n - 3; xs = 1; break;
            case 3: xm = n - 3; ym = n - 1; ys = 1; break;
            default: xm = n; ym = n; ys = 1; break;
        }
        pxr = mu < 4 ? 2 * (xm + nm + 3) : 2 * n_g + 2 * n;
        pyr = mu < 4 ? 2 * (ym + nm + 3) : 2 * n_g + 2 * n;
    };
    // operands of one iteration: slot t < B is X(b = t), t >= B is Y(b = t - B);
    // lane holds slots lane and lane + 64.  Loaded one iteration ahead.
    float pre[2][2];
    auto fetch = [&](int it) {
        int mu_, n_, xm_, ym_, xs_, ys_, pxr_, pyr_;
        orders(it, mu_, n_, xm_, ym_, xs_, ys_, pxr_, pyr_);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int t = lane + 64 * r;
            pre[r][0] = pre[r][1] = 0.0f;
            if (t < 2 * B) {
                const bool ty_side = t >= B;
                const int bt = ty_side ? t - B : t;
                const int pl = ty_side ? pyr_ : pxr_;
                pre[r][0] = a.planes[chunk_offset(pl, i, bt, K, B)];
                const float im = a.planes[chunk_offset(pl + 1, i, bt, K, B)];
                pre[r][1] = (ty_side ? ys_ : xs_) ? -im : im;
            }
        }
    };
    const int n_it = 5 * (nm + 1);
    fetch(0);
    for (int it = 0; it < n_it; ++it) {
        int mu, n, xm, ym, xs, ys, pxr, pyr;
        orders(it, mu, n, xm, ym, xs, ys, pxr, pyr);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int t = lane + 64 * r;
            if (t < 2 * B) {
                const bool ty_side = t >= B;
                (ty_side ? Ys : Xs)[ty_side ? t - B : t] = make_float2(pre[r][0], pre[r][1]);
            }
        }
        if (it + 1 < n_it) fetch(it + 1);  // in flight during this iteration
        __syncthreads();
        const double *U = a.gups + 2 * ((size_t)mu * pstr + (size_t)n * B * B);
        double2 gops[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
        for (int g = 0; g < 2; ++g) {
            const int b = (lane & 31) + 32 * g;
            if (b >= B) break;
            // side X: u(b1) = sum_b2 Ub(b1, b2) conj(Y(b2)); side Y: v(b2) = sum_b1 Ub(b1, b2) conj(X(b1))
            double ur = 0.0, ui = 0.0;
            for (int k0 = 0; k0 < B; k0 += 8) {
                // eight independent loads of Ub in flight, then the products
                double ugr[8], ugi[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int k = min(k0 + q, B - 1);
                    const size_t idx = side_y ? ((size_t)k * B + b) : ((size_t)b * B + k);
                    ugr[q] = U[2 * idx];
                    ugi[q] = U[2 * idx + 1];
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if (k0 + q < B) {
                        const float2 of = side_y ? Xs[k0 + q] : Ys[k0 + q];
                        const double2 o = make_double2(of.x, of.y);
                        ur += ugr[q] * o.x + ugi[q] * o.y;  // Ub * conj(o)
                        ui += ugi[q] * o.x - ugr[q] * o.y;
                    }
                }
            }
            // grad operand = conj(alpha) * u
            const double ar = al_r[mu], ai = al_i[mu];
            double gr = ar * ur + ai * ui, gi = ar * ui - ai * ur;
            if (!side_y) {
                // grad alpha += conj(X(b1)) u(b1)
                const double2 x = make_double2(Xs[b].x, Xs[b].y);
                ga_r[mu] += x.x * ur + x.y * ui;
                ga_i[mu] += x.x * ui - x.y * ur;
            }
            const int cj = side_y ? ys : xs;
            if (cj) gi = -gi;  // operand was conj(G): grad G = conj(grad operand)
            gops[g] = make_double2(gr, gi);
        }
        // the two sides may update the same (b, order): one side at a time
        for (int side = 0; side < 2; ++side) {
            if (side_y == (side == 1)) {
                for (int g = 0; g < 2; ++g) {
                    const int b = (lane & 31) + 32 * g;
                    if (b >= B) break;
                    const int m = side ? ym : xm;
                    float2 *t = mu < 4 ? &Gb[b * n_g + (m + nm + 3)] : &Wb[b * (nm + 1) + n];
                    *t = make_float2((float)(t->x + gops[g].x), (float)(t->y + gops[g].y));
                }
            }
            __syncthreads();
        }
    }
    // j = k terms
    if (a.jk && lane < B) {
        const int bb = lane;
        const int pD = 2 * n_g + 2 * (nm + 1);
        double dsum_r[5], dsum_i[5];
        for (int mu = 0; mu < 5; ++mu) {
            double sr = 0.0, si = 0.0;
            const double *U = a.gups + 2 * ((size_t)mu * pstr);
            for (int n = 0; n <= nm; ++n) {
                const size_t idx = (size_t)n * B * B + (size_t)bb * B + bb;
                sr += U[2 * idx];
                si += U[2 * idx + 1];
            }
            dsum_r[mu] = sr;
            dsum_i[mu] = si;
        }
        // D values of this centre
        const double d6r = a.planes[chunk_offset(pD + 0, i, bb, K, B)];
        const double d6i = a.planes[chunk_offset(pD + 1, i, bb, K, B)];
        const double d2r = a.planes[chunk_offset(pD + 2, i, bb, K, B)];
        const double d2i = a.planes[chunk_offset(pD + 3, i, bb, K, B)];
        const double dar = a.planes[chunk_offset(pD + 4, i, bb, K, B)];
        const double dai = a.planes[chunk_offset(pD + 5, i, bb, K, B)];
        const double dw = a.planes[chunk_offset(pD + 6, i, bb, K, B)];
        // grad D = -conj(alpha) sum_n Ub(b, b); grad alpha -= conj(D) sum_n Ub(b, b)
        auto gD = [&](int mu, double &gr, double &gi) {
            const double ar = al_r[mu], ai = al_i[mu], ur = dsum_r[mu], ui = dsum_i[mu];
            gr = -(ar * ur + ai * ui);
            gi = -(ar * ui - ai * ur);
        };
        double r0, i0, r1, i1, r2, i2, r3, i3, r4, i4;
        gD(0, r0, i0);
        gD(1, r1, i1);
        gD(2, r2, i2);
        gD(3, r3, i3);
        gD(4, r4, i4);
        Db[bb * 4 + 0] = make_float2((float)r0, (float)i0);
        Db[bb * 4 + 1] = make_float2((float)r1, (float)i1);
        Db[bb * 4 + 2] = make_float2((float)(r2 + r3), (float)(i2 + i3));
        Db[bb * 4 + 3] = make_float2((float)r4, (float)i4);
        auto sub = [&](int mu, double dr, double di) {
            ga_r[mu] -= dr * dsum_r[mu] + di * dsum_i[mu];
            ga_i[mu] -= dr * dsum_i[mu] - di * dsum_r[mu];
        };
        sub(0, d6r, d6i);
        sub(1, d2r, d2i);
        sub(2, dar, dai);
        sub(3, dar, dai);
        sub(4, dw, 0.0);
    }
    __syncthreads();
    // centre gradient: reduce grad alpha over the wavefront (the X-side
    // lanes hold the operand terms, lanes 0..B-1 the j = k terms, others 0)
    double gcr = 0.0, gci = 0.0, gw = 0.0;
    {
        double vr = -ga_r[0] - ga_r[1] - ga_r[2] - ga_r[3];
        double vi = -ga_i[0] + ga_i[1] - ga_i[2] - ga_i[3];
        double vw = ga_r[4];
        for (int d = 32; d > 0; d >>= 1) {
            vr += __shfl_xor(vr, d, 64);
            vi += __shfl_xor(vi, d, 64);
            vw += __shfl_xor(vw, d, 64);
        }
        gcr = vr;
        gci = vi;
        gw = vw;
    }
    if (lane == 0) {
        a.cen_gc[i] = make_float2((float)gcr, (float)gci);
        a.cen_gw[i] = (float)gw;
    }
    // coefficient blocks
    const int C = a.cap, M = C + 3, CS = coef_size(C);
    float vmax = 0.0f;
    for (int t = lane; t < B * CS; t += 64) {
        const int bb = t / CS, k = t % CS;
        float v = 0.0f;
        if (k < 4 * M) {
            const int m = k / 4 + 1, q = k % 4;
            double2 gp = make_double2(0.0, 0.0), gm = make_double2(0.0, 0.0);
            if (m <= nm - 1) gp = make_double2(Gb[bb * n_g + (m + nm + 3)].x, Gb[bb * n_g + (m + nm + 3)].y);
            if (m <= nm + 3) gm = make_double2(Gb[bb * n_g + (-m + nm + 3)].x, Gb[bb * n_g + (-m + nm + 3)].y);
            // s = gp + gm ; d = i (gm - gp) = (-(gm.y - gp.y), gm.x - gp.x)
            const double val = q == 0 ? gp.x + gm.x : q == 1 ? gp.y + gm.y
                             : q == 2 ? -(gm.y - gp.y) : (gm.x - gp.x);
            v = (float)val;
        } else if (k < 4 * M + 2) {
            if (nm >= 1) {
                const float2 g0 = Gb[bb * n_g + (nm + 3)];
                v = (float)(k == 4 * M ? g0.x : g0.y);
            }
        } else if (k < 4 * M + 2 + 2 * (C + 1)) {
            const int kk = k - 4 * M - 2, m = kk / 2;
            if (m <= nm) {
                const float2 wv = Wb[bb * (nm + 1) + m];
                v = (float)(kk % 2 == 0 ? wv.x : wv.y);
            }
        } else {
            const int kk = k - 4 * M - 2 - 2 * (C + 1);  // 0..6
            const float2 d = Db[bb * 4 + (kk < 6 ? kk / 2 : 3)];
            v = (float)(kk == 6 ? d.x : (kk % 2 == 0 ? d.x : d.y));
        }
        a.coef[((size_t)i * B + bb) * CS + k] = v;
        vmax = fmaxf(vmax, fabsf(v));
    }
    if (a.coef_max) {
        // an integer maximum of non-negative float bits: order-independent
        for (int d = 32; d > 0; d >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, d, 64));
        if (lane == 0) atomicMax(a.coef_max, __float_as_uint(vmax));
    }
}

struct ScatterArgs {
    SweepArgs sw;
    const int2 *cpos;     // centre positions (chunk-relative)
    const float *coef;    // [n_c][B][coef_size(cap)]
    int n_c, B, jk;
    float *nb_gc;         // [2][n] grad c of neighbours (sorted index): real parts, then imaginary
    float *nb_gw;         // [n]
    unsigned long long *det_acc;  // deterministic mode: [3][n] fixed-point sums (else null)
    const unsigned *det_hdr;      // deterministic mode: max |coef| and cmax (float bits)
    int64_t n_nb;         // neighbours n
    double e2[65];
};

// Gradient terms of one (centre, neighbour) pair: the transposed
// recurrence against the centre's coefficient block c (LDS, uniform across
// the wavefront), added to (gr, gim, gw).
template <int C>
__device__ __forceinline__ void pair_grad(const float *c, int dx, int dy, float cr, float cim, float wt, int jk,
                                          float &gr_out, float &gim_out, float &gw_out)
{
    constexpr int M = C + 3;
    const double xd = (double)dx, yd = (double)dy;
    const double r2 = fma(xd, xd, yd * yd);
    double s = (double)__builtin_amdgcn_rsqf((float)r2);
    s = s * fma(-0.5 * r2 * s, s, 1.5);
    const double zr = xd * s, zi = yd * s;
    const float fzr = (float)zr, fzi = (float)zi;
    const double z2r = fma(zr, zr, -zi * zi), z2i = 2.0 * zr * zi;
    const double z4r = fma(z2r, z2r, -z2i * z2i), z4i = 2.0 * z2r * z2i;
    float gr = c[4 * M], gim = c[4 * M + 1];  // Gb_0
    float gw = c[4 * M + 2];                   // Re Wb_0
    // the terms of order m with the power (pr, pi) = z^m
    auto term = [&](int m, float pr, float pi) {
        if (m < 1 || m > M) return;
        const float4 sd = *reinterpret_cast<const float4 *>(c + 4 * (m - 1));
        gr = fmaf(pr, sd.x, fmaf(pi, sd.z, gr));
        gim = fmaf(pr, sd.y, fmaf(pi, sd.w, gim));
        if (m <= C) {
            const float2 wb = *reinterpret_cast<const float2 *>(c + 4 * M + 2 + 2 * m);
            gw = fmaf(pr, wb.x, fmaf(pi, wb.y, gw));
        }
    };
    // Powers as in the forward scan: FP64 anchors Z_k = z^{4k} (z^4 by
    // squaring, then Z_{k+1} = 2 cos(4 phi) Z_k - Z_{k-1}) rounded once to
    // FP32; around an anchor z^a, z^{a+1} = z^a z by one FP32 complex
    // multiplication and z^{a-1}, z^{a+2} from z^{k+1} + z^{k-1} = 2 cos(phi) z^k.
    const float tc = 2.0f * fzr;
    const double t4 = 2.0 * z4r;
    double cr0 = 1.0, ci0 = 0.0, pr0 = 0.0, pi0 = 0.0;
#pragma unroll
    for (int k = 0; 4 * k <= M + 1; ++k) {
        const int a0 = 4 * k;
        float fr = (float)cr0, fi = (float)ci0, ur = fzr, ui = fzi;
        if (k == 0) {
            fr = 1.0f;
            fi = 0.0f;
        } else {
            ur = fmaf(fr, fzr, -fi * fzi);
            ui = fmaf(fr, fzi, fi * fzr);
        }
        term(a0 - 1, fmaf(tc, fr, -ur), fmaf(tc, fi, -ui));
        term(a0, fr, fi);
        term(a0 + 1, ur, ui);
        if (k == 0)
            term(2, (float)z2r, (float)z2i);
        else
            term(a0 + 2, fmaf(tc, ur, -fr), fmaf(tc, ui, -fi));
        if (a0 + 3 > M) break;
        double nr, ni;
        if (k == 0) {
            nr = z4r;
            ni = z4i;
        } else {
            nr = fma(t4, cr0, -pr0);
            ni = fma(t4, ci0, -pi0);
        }
        pr0 = cr0;
        pi0 = ci0;
        cr0 = nr;
        ci0 = ni;
    }
    if (jk) {
        const int o = 4 * M + 2 + 2 * (C + 1);
        const float p2r = (float)z2r, p2i = (float)z2i;
        const double z6r = fma(z4r, z2r, -z4i * z2i), z6i = fma(z4r, z2i, z4i * z2r);
        const float p6r = (float)z6r, p6i = (float)z6i;
        // 2 conj(c) p6 D6b + 2 conj(c) p2 D2b
        const float q6r = fmaf(p6r, c[o + 0], -p6i * c[o + 1]);
        const float q6i = fmaf(p6r, c[o + 1], p6i * c[o + 0]);
        const float q2r = fmaf(p2r, c[o + 2], -p2i * c[o + 3]);
        const float q2i = fmaf(p2r, c[o + 3], p2i * c[o + 2]);
        const float qr = q6r + q2r, qi = q6i + q2i;
        gr = fmaf(2.0f * cr, qr, fmaf(2.0f * cim, qi, gr));
        gim = fmaf(2.0f * cr, qi, fmaf(-2.0f * cim, qr, gim));
        // 2 c Re(DAb p2)
        const float ra = fmaf(c[o + 4], p2r, -c[o + 5] * p2i);
        gr = fmaf(2.0f * cr, ra, gr);
        gim = fmaf(2.0f * cim, ra, gim);
        // 2 w Re(DWb)
        gw = fmaf(2.0f * wt, c[o + 6], gw);
    }
    gr_out += gr;
    gim_out += gim;
    gw_out += gw;
}

// Transpose scan.  A workgroup owns four consecutive centres of the
// cell-sorted order (nearby on the sky).  Per bin its four wavefronts split
// the cell rows (every fourth row) of one annulus around centre 0, widened
// by the largest centre offset D so that it holds the four centres' annuli;
// each lane takes one candidate through the transposed recurrences of the
// centres in whose bin it lies and adds the summed terms with three
// atomics: a quarter of the atomics of one centre per wavefront.  Where the
// widening D exceeds the bin width (narrow bins, or a group that straddles
// the end of a cell row) the group sweeps each centre's own annulus in turn
// instead.  (Measured on 500k galaxies, 15 bins 1'-60': joint sweeps where
// D <= width/8: 26 ms per 65k-centre chunk, D <= width/4: 21 ms,
// D <= width/2: 19.7 ms, D <= width: 19.5 ms; one centre per wavefront:
// 35 ms.)
template <int C>
__global__ __launch_bounds__(64 * kWaves) void k_adj_scatter(ScatterArgs a)
{
    constexpr int CS = coef_size(C);
    __shared__ int4 q_xyc[kWaves][kRing];
    __shared__ int2 q_wi[kWaves][kRing];
    __shared__ int2 spans[kWaves][2 * kRowsPerBlock + 1];
    constexpr int CSP = (CS + 3) & ~3;  // 16-byte aligned rows
    __shared__ __align__(16) float cf[kWaves][CSP];  // coefficient block of centre k of the group
    __shared__ int2 cpk[kWaves];                       // positions of the group's centres

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    // groups in launch order: the round-robin dispatch over the 8 XCDs keeps
    // every XCD on neighbouring groups, which share neighbours in the
    // Infinity Cache (2% faster kept-plane backward than contiguous ranges
    // of groups per XCD)
    const int c0 = blockIdx.x * kWaves;  // first centre of the group
    if (c0 >= a.n_c) return;     // the whole workgroup leaves together
    const int nk = min(kWaves, a.n_c - c0);
    double dmax = 0.0;
    const int2 p0 = a.cpos[c0];
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
        const int2 pk = a.cpos[c0 + min(k, nk - 1)];
        const double ox = (double)((long long)pk.x - p0.x), oy = (double)((long long)pk.y - p0.y);
        dmax = fmax(dmax, sqrt(fma(ox, ox, oy * oy)));
    }
    if (threadIdx.x < kWaves) cpk[threadIdx.x] = a.cpos[c0 + min((int)threadIdx.x, nk - 1)];
    const double D = ceil(dmax) + 2.0;  // covers the roundings of the square roots below
    const SweepLDS lds{q_xyc[wv], q_wi[wv], spans[wv]};
    const double det_scale = a.det_acc ? ldexp(1.0, det_exponent(a.det_hdr, a.n_c, CS)) : 0.0;

    for (int b = 0; b < a.B; ++b) {
        __syncthreads();
        for (int t = threadIdx.x; t < kWaves * CS; t += 64 * kWaves) {
            const int k = t / CS, e = t - k * CS;
            cf[k][e] = k < nk ? a.coef[((size_t)(c0 + k) * a.B + b) * CS + e] : 0.0f;
        }
        __syncthreads();
        const double e2lo = a.e2[b], e2hi = a.e2[b + 1];
        const double elo = sqrt(e2lo), ehi = sqrt(e2hi);
        const bool joint = nk > 1 && D <= ehi - elo;
        // joint: one sweep for every centre; else one sweep per centre
        const int n_sweeps = joint ? 1 : nk;
        for (int q = 0; q < n_sweeps; ++q) {
            const int2 sc = cpk[q];
            const int k_lo = joint ? 0 : q, k_hi = joint ? nk : q + 1;
            const double wlo = joint ? fmax(elo - D, 0.0) : 0.0;
            const double s2lo = joint ? wlo * wlo : e2lo;
            const double s2hi = joint ? (ehi + D) * (ehi + D) : e2hi;
            sweep_annulus(
                a.sw, sc, s2lo, s2hi, lane, lds,
                [&](const int4 &e, float wt, int gi, bool act) {
                    const float cr = __int_as_float(e.z), cim = __int_as_float(e.w);
                    float gr = 0.0f, gim = 0.0f, gw = 0.0f;
                    bool any_in = false;
#pragma unroll 1
                    for (int k = k_lo; k < k_hi; ++k) {
                        const int dx = e.x + (sc.x - cpk[k].x), dy = e.y + (sc.y - cpk[k].y);
                        const double r2 = fma((double)dx, (double)dx, (double)dy * (double)dy);
                        const bool in = act && r2 >= e2lo && r2 < e2hi;
                        if (in) {
                            pair_grad<C>(cf[k], dx, dy, cr, cim, wt, a.jk, gr, gim, gw);
                            any_in = true;
                        }
                    }
                    if (any_in) {
                        // three planar arrays: a wavefront's compacted
                        // neighbours are mostly consecutive sorted indices,
                        // so each atomic instruction covers few, fully used
                        // cache lines
                        if (a.det_acc) {
                            // two's-complement fixed point: integer sums do not
                            // depend on the order of the atomics
                            const long long vr = llrint((double)gr * det_scale);
                            const long long vi = llrint((double)gim * det_scale);
                            const long long vw = llrint((double)gw * det_scale);
                            atomicAdd(a.det_acc + gi, (unsigned long long)vr);
                            atomicAdd(a.det_acc + a.n_nb + gi, (unsigned long long)vi);
                            atomicAdd(a.det_acc + 2 * a.n_nb + gi, (unsigned long long)vw);
                        } else {
                            unsafeAtomicAdd(a.nb_gc + gi, gr);
                            unsafeAtomicAdd(a.nb_gc + a.n_nb + gi, gim);
                            unsafeAtomicAdd(a.nb_gw + gi, gw);
                        }
                    }
                },
                wv, kWaves);
        }
    }
}

// Deterministic mode: the chunk's fixed-point sums into the FP64 totals
// (chunk order), clearing them for the next chunk.
__global__ void k_det_fold(unsigned long long *acc, double *tot, int64_t n3, const unsigned *hdr, int n_c, int cs)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n3) return;
    const double inv = ldexp(1.0, -det_exponent(hdr, n_c, cs));
    tot[t] += (double)(long long)acc[t] * inv;
    acc[t] = 0ull;
}

// Deterministic mode: FP64 totals to the FP32 neighbour arrays of k_adj_combine.
__global__ void k_det_out(const double *tot, int64_t n3, float *nb)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n3) nb[t] = (float)tot[t];
}

// cmax = max(1, |Re c| + |Im c|, w) over the sorted catalog (float bits, order-independent max).
__global__ void k_cat_cmax(const float4 *cw, int64_t n, unsigned *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float m = 1.0f;
    if (t < n) {
        const float4 c = cw[t];
        m = fmaxf(m, fmaxf(fabsf(c.x) + fabsf(c.y), fabsf(c.z)));
    }
    for (int d = 32; d > 0; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

__global__ void k_set_u32(unsigned *p, unsigned v) { *p = v; }

__global__ void k_zero_u64(unsigned long long *p, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0ull;
}

__global__ void k_zero_d(double *p, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.0;
}

// cen_gc / cen_gw null: the centre terms are added separately (centre lists).
__global__ void k_adj_combine(const int *perm, int64_t n, const float *nb_gc, const float *nb_gw,
                              const float2 *cen_gc, const float *cen_gw, const float *g1, const float *g2,
                              const float *w, float *out_g1, float *out_g2, float *out_w)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int i = perm[s];
    const float gcr = nb_gc[s] + (cen_gc ? cen_gc[s].x : 0.0f);
    const float gci = nb_gc[n + s] + (cen_gc ? cen_gc[s].y : 0.0f);
    const float gwd = nb_gw[s] + (cen_gw ? cen_gw[s] : 0.0f);
    const float wi = w[i];
    out_g1[i] = wi * gcr;
    out_g2[i] = wi * gci;
    out_w[i] = gwd + g1[i] * gcr + g2[i] * gci;
}

// Centre terms of a centre list: centre k is galaxy idx[k] (c = w gamma chain
// rule as in k_adj_combine, which it follows).  A repeated index adds its
// terms once per occurrence, in an unspecified order.
__global__ void k_adj_centre_add(const int32_t *idx, int64_t n_c, const float2 *cen_gc, const float *cen_gw,
                                 const float *g1, const float *g2, const float *w, float *out_g1, float *out_g2,
                                 float *out_w)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_c) return;
    const int i = idx[k];
    const float gcr = cen_gc[k].x, gci = cen_gc[k].y;
    const float wi = w[i];
    atomicAdd(out_g1 + i, wi * gcr);
    atomicAdd(out_g2 + i, wi * gci);
    atomicAdd(out_w + i, cen_gw[k] + g1[i] * gcr + g2[i] * gci);
}

__global__ void k_zero_f(float *p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// grad Upsilon from grad Gamma (Gamma_{mu,n} = Upsilon_{mu,n} / N_0, mu < 4).
__global__ void k_norm_bwd(const double *ups, const double *ggam, int n_sets, int n_max, int B,
                           double *gups)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t bb = (int64_t)B * B;
    const int64_t per_mu = (int64_t)(n_max + 1) * bb;
    if (t >= (int64_t)n_sets * bb) return;
    const int64_t set = t / bb, e = t % bb;
    const double *u = ups + 2 * (set * 5 * per_mu);
    const double *g = ggam + 2 * (set * 4 * per_mu);
    double *o = gups + 2 * (set * 5 * per_mu);
    const double n0 = u[2 * (4 * per_mu + e)];
    double dn0 = 0.0;
    for (int mu = 0; mu < 4; ++mu)
        for (int n = 0; n <= n_max; ++n) {
            const int64_t k = mu * per_mu + n * bb + e;
            const double gr = g[2 * k], gi = g[2 * k + 1];
            if (n0 != 0.0) {
                const double ur = u[2 * k], ui = u[2 * k + 1];
                o[2 * k] = gr / n0;
                o[2 * k + 1] = gi / n0;
                dn0 -= (gr * ur + gi * ui) / (n0 * n0);
            } else {
                o[2 * k] = 0.0;
                o[2 * k + 1] = 0.0;
            }
        }
    for (int n = 0; n <= n_max; ++n) {
        const int64_t k = 4 * per_mu + n * bb + e;
        o[2 * k] = n == 0 ? dn0 : 0.0;
        o[2 * k + 1] = 0.0;
    }
}

struct ScatterVariant {
    int cap;
    void (*kernel)(ScatterArgs);
};

const ScatterVariant kScatter[] = {
    {4, k_adj_scatter<4>},   {8, k_adj_scatter<8>},   {10, k_adj_scatter<10>}, {12, k_adj_scatter<12>},
    {16, k_adj_scatter<16>}, {20, k_adj_scatter<20>}, {24, k_adj_scatter<24>}, {30, k_adj_scatter<30>},
    {32, k_adj_scatter<32>}, {40, k_adj_scatter<40>}, {48, k_adj_scatter<48>}, {64, k_adj_scatter<64>},
};

}  // namespace

int normalise_backward(t3_plan *plan, const double *ups, const double *ggam, int n_sets, double *gups,
                       hipStream_t s)
{
    const int64_t tot = (int64_t)n_sets * plan->B * plan->B;
    hipLaunchKernelGGL(k_norm_bwd, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, ups, ggam,
                       n_sets, plan->n_max, plan->B, gups);
    T3_HIP_CHECK(hipGetLastError());
    return T3_OK;
}

int backward(t3_plan *plan, const t3_catalog &cat, const int32_t *centres, int64_t n_centres,
             const double *grad_ups, float *gg1, float *gg2, float *gw, hipStream_t s)
{
    T3_TRY(timing_begin_call(plan));
    T3_TRY(plan->flag.reserve(sizeof(int) * 4));
    T3_TRY(plan->counter.reserve(sizeof(unsigned long long) * 4));
    T3_HIP_CHECK(hipMemsetAsync(plan->flag.ptr, 0, sizeof(int) * 4, s));
    SortedCatalog &sc = plan->cats[0];
    const bool all = n_centres < 0;
    // planes kept by the last forward over every galaxy of this very
    // catalog: its sorted catalog, centres and chunk layout are still the plan's
    const t3_catalog &kc = plan->kept_cat;
    const bool kept = all && (plan->flags & T3_FLAG_KEEP_PLANES) && plan->kept_seq == plan->cells_seq &&
                      kc.n == cat.n && kc.x == cat.x && kc.y == cat.y && kc.g1 == cat.g1 && kc.g2 == cat.g2 &&
                      kc.w == cat.w && plan->kept_L.B == plan->B && plan->kept_L.n_max == plan->n_max;
    CentreSet &cen = kept ? plan->csets[0] : plan->centres;
    const int64_t n = cat.n;
    const int64_t n_c = all ? n : n_centres;
    const ScatterVariant *sv = nullptr;
    for (const auto &v : kScatter)
        if (v.cap >= plan->n_max) {
            sv = &v;
            break;
        }
    if (!sv) return fail(T3_ERANGE, "t3_backward: n_max above the compiled variants");
    const int B = plan->B, nm = plan->n_max;
    const size_t lds = sizeof(float2) * ((size_t)B * ((2 * nm + 3) + (nm + 1) + 4) + 2 * kMaxRadialBins);
    if (lds > 160 * 1024)  // a workgroup's LDS limit on gfx950 (B = n_max = 64 needs 101 KiB)
        return fail(T3_ERANGE, "t3_backward: n_bins (3 n_max + 8) above the coefficient kernel's LDS");
    ChunkLayout L;
    L.n_max = plan->n_max;
    L.w_max = plan->w_max;
    L.B = plan->B;
    L.K = choose_chunk(plan, L);
    if (plan->chunk_req <= 0 && (int64_t)L.K > n_c)  // small centre sets, small buffers
        L.K = (int)std::max<int64_t>(256, ((int64_t)n_c + 255) & ~(int64_t)255);
    if (kept) L = plan->kept_L;
    const int CS = coef_size(sv->cap);
    const bool det = (plan->flags & T3_FLAG_DETERMINISTIC) != 0;
    // every buffer is reserved before the first launch that writes an output:
    // a call refused for the workspace limit leaves the gradients untouched
    // scratch: nb_gc [2][n], nb_gw [n], cen_gc [2 n_c], cen_gw [n_c]
    T3_TRY(plan->misc.reserve(sizeof(float) * (3 * (size_t)n + 3 * (size_t)n_c + 4)));
    T3_TRY(plan->misc2.reserve(sizeof(float) * (size_t)L.K * L.B * CS));
    if (!kept) T3_TRY(plan->chunk.reserve(sizeof(float) * L.floats()));
    // deterministic mode: header (max |coef|, cmax), fixed-point sums [3n], FP64 totals [3n]
    if (det) T3_TRY(plan->det.reserve(16 + 16 * 3 * (size_t)n + 64));
    if (!kept) {
        T3_TRY(build_cells(plan, sc, cat, choose_grid(plan, cat.n), s));
        if (all)
            T3_TRY(gather_sorted_centres(plan, sc, plan->centres, s));
        else
            T3_TRY(gather_centres(plan, cat, centres, n_centres, plan->centres, s));
        T3_TRY(check_flag(plan, s, "t3_backward"));
    }
    if (n == 0) return T3_OK;

    float *nb_gc = plan->misc.as<float>();
    float *nb_gw = nb_gc + 2 * n;
    float *cen_base = nb_gw + n;
    // float2 alignment of the centre terms
    float2 *cen_gc = reinterpret_cast<float2 *>(cen_base + ((reinterpret_cast<uintptr_t>(cen_base) & 7) ? 1 : 0));
    float *cen_gw = reinterpret_cast<float *>(cen_gc + n_c);
    hipLaunchKernelGGL(k_zero_f, dim3((unsigned)((3 * n + 3 * n_c + 4 + 255) / 256)), dim3(256), 0, s, nb_gc,
                       (size_t)(3 * n + 3 * n_c + 4));
    T3_HIP_CHECK(hipGetLastError());
    unsigned *det_hdr = nullptr;
    unsigned long long *det_acc = nullptr;
    double *det_tot = nullptr;
    if (det) {
        det_hdr = plan->det.as<unsigned>();
        det_acc = reinterpret_cast<unsigned long long *>(plan->det.as<char>() + 16);
        det_tot = reinterpret_cast<double *>(det_acc + 3 * n);
        hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((3 * n + 255) / 256)), dim3(256), 0, s, det_acc, 3 * n);
        T3_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(k_zero_d, dim3((unsigned)((3 * n + 255) / 256)), dim3(256), 0, s, det_tot, 3 * n);
        T3_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, det_hdr + 1, 0u);
        T3_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(k_cat_cmax, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           (const float4 *)sc.cw.as<float4>(), n, det_hdr + 1);
        T3_HIP_CHECK(hipGetLastError());
    }
    const bool jk = !(plan->flags & T3_FLAG_KEEP_JK);
    if (lds > 64 * 1024)
        T3_HIP_CHECK(hipFuncSetAttribute((const void *)k_adj_coef,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int n_lane = 0;
    if (!kept && n_c > 0) T3_TRY(lane_bins(plan, sc, 0, B, plan->lane_neighbours, s, &n_lane));
    for (int64_t c0 = 0; c0 < n_c; c0 += L.K) {
        const int nc = (int)((n_c - c0) < L.K ? (n_c - c0) : L.K);
        const float *planes = kept ? plan->kept.as<float>() + (size_t)(c0 / L.K) * L.floats() : plan->chunk.as<float>();
        if (!kept) {
            T3_TRY(timing_mark(plan, 1, true, s));
            const SortedCatalog *cl[1] = {&sc};
            T3_TRY(scan_chunk(plan, cl, nullptr, 1, plan->centres, c0, nc, L, plan->chunk.as<float>(), 0, nullptr,
                              plan->scan_mode, s, 0, B, n_lane));
            T3_TRY(timing_mark(plan, 1, false, s));
        }
        T3_TRY(timing_mark(plan, 2, true, s));
        if (det) {
            hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, det_hdr, 0u);
            T3_HIP_CHECK(hipGetLastError());
        }
        CoefArgs ca{};
        ca.planes = planes;
        ca.ccw = cen.cw.as<float4>() + c0;
        ca.gups = grad_ups;
        ca.n_c = nc;
        ca.K = L.K;
        ca.B = B;
        ca.n_max = nm;
        ca.cap = sv->cap;
        ca.jk = jk ? 1 : 0;
        ca.coef = plan->misc2.as<float>();
        ca.cen_gc = cen_gc + c0;
        ca.cen_gw = cen_gw + c0;
        ca.coef_max = det_hdr;
        hipLaunchKernelGGL(k_adj_coef, dim3(nc), dim3(64), lds, s, ca);
        T3_HIP_CHECK(hipGetLastError());
        T3_TRY(timing_mark(plan, 2, false, s));
        T3_TRY(timing_mark(plan, 3, true, s));
        ScatterArgs sa{};
        sa.sw.npos = sc.pos.as<int2>();
        sa.sw.ncw = sc.cw.as<float4>();
        sa.sw.cell_start = sc.cell_start.as<int>();
        sa.sw.g = sc.grid;
        sa.cpos = cen.pos.as<int2>() + c0;
        sa.coef = plan->misc2.as<float>();
        sa.n_c = nc;
        sa.B = B;
        sa.jk = jk ? 1 : 0;
        sa.nb_gc = nb_gc;
        sa.nb_gw = nb_gw;
        sa.det_acc = det_acc;
        sa.det_hdr = det_hdr;
        sa.n_nb = n;
        for (int b = 0; b <= B; ++b) sa.e2[b] = plan->e2[b];
        const int nwg = (nc + kWaves - 1) / kWaves;
        hipLaunchKernelGGL(sv->kernel, dim3((unsigned)nwg), dim3(64 * kWaves), 0, s, sa);
        T3_HIP_CHECK(hipGetLastError());
        if (det) {
            hipLaunchKernelGGL(k_det_fold, dim3((unsigned)((3 * n + 255) / 256)), dim3(256), 0, s, det_acc, det_tot,
                               3 * n, (const unsigned *)det_hdr, nc, CS);
            T3_HIP_CHECK(hipGetLastError());
        }
        T3_TRY(timing_mark(plan, 3, false, s));
    }
    if (det) {
        // nb_gc [2n] and nb_gw [n] are contiguous, as are the three totals
        hipLaunchKernelGGL(k_det_out, dim3((unsigned)((3 * n + 255) / 256)), dim3(256), 0, s,
                           (const double *)det_tot, 3 * n, nb_gc);
        T3_HIP_CHECK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_adj_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       (const int *)sc.perm.as<int>(), n, (const float *)nb_gc, (const float *)nb_gw,
                       all ? (const float2 *)cen_gc : nullptr, all ? (const float *)cen_gw : nullptr, cat.g1, cat.g2,
                       cat.w, gg1, gg2, gw);
    T3_HIP_CHECK(hipGetLastError());
    if (!all && n_c > 0) {
        hipLaunchKernelGGL(k_adj_centre_add, dim3((unsigned)((n_c + 255) / 256)), dim3(256), 0, s, centres, n_c,
                           (const float2 *)cen_gc, (const float *)cen_gw, cat.g1, cat.g2, cat.w, gg1, gg2, gw);
        T3_HIP_CHECK(hipGetLastError());
    }
    T3_HIP_CHECK(hipStreamSynchronize(s));
    T3_TRY(timing_end_call(plan));
    return T3_OK;
}

}  // namespace t3
