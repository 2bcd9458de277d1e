// Stage 1 of the multipole estimator: per-centre harmonic sums
//     G_m(i; b) = sum_j c_j z_ij^m,   W_m(i; b) = sum_j w_j z_ij^m,
// z_ij = e^{i phi_ij}, over the neighbours j of centre i in radial bin b
// (Porth et al. 2023, eq. Gn_disc and the W_n of eq. 3PCF_Normalization),
// plus the single-neighbour sums that remove j = k from the products.
//
// Mapping (one wavefront per centre, one radial bin at a time):
//  * the neighbours of the annulus [e_b, e_{b+1}) come from the shared
//    annulus sweep (sweep.h): row runs of the cell list, coalesced candidate
//    tests, ballot compaction into an LDS ring, 64 in-bin neighbours per
//    batch, each lane taking one through the harmonic recurrence;
//  * per-lane FP32 accumulators hold one bin of one centre; every 64 batches
//    and at the end of the bin a 6-step reduce-scatter (permlane swaps and
//    DPP permutations) leaves each lane a few wave totals, which are added to
//    the wavefront's FP64 partials (in LDS); at the end of the bin those are
//    stored into the chunk planes (layout in t3_internal.h) -- in the
//    single-catalog launch through an LDS stage, from which the last of the
//    workgroup's four wavefronts writes rows of four centres.
//
// Arithmetic per neighbour: dx, dy are exact lattice integers, r^2 is exact
// in FP64 and is compared with the same FP64 squared edges as everywhere
// else, so bin membership is exact.  z is formed in FP64 (rsqrt seed + one
// Newton step), anchors z^{4k} are FP64 and rounded once to FP32 (z^4 by
// squaring, then the three-term relation Z_{k+1} = 2 cos(4 phi) Z_k - Z_{k-1},
// two FMAs per anchor); around an anchor z^a, z^{a+1} takes one FP32 complex
// multiplication and z^{a-1}, z^{a+2} one FMA per component from the
// relation z^{k+1} + z^{k-1} = 2 cos(phi) z^k, so every p_m = z^m is at most
// two FP32 steps from an anchor and its error a few FP32 ulp whatever m
// (with chains of up to 4 steps, small tomographic samples reached the 1e-6
// FP32 bar on single blocks).
// G_m and G_{-m} share p_m:
//     S1 += Re c Re p,  S2 += Im c Im p,  S3 += Re c Im p,  S4 += Im c Re p
//     G_m = (S1 - S2, S3 + S4),   G_{-m} = (S1 + S2, S4 - S3)
// which costs 4 FMAs for two orders.  The conversion is linear, so it is
// applied to the FP64 wave totals when each (S1, S2) and (S3, S4) pair ends
// on one lane of the reduce-scatter, else to the FP32 lane partials first.
// Orders that a pass needs only as G_{-m} (the top three or four of the
// n_max = C pass) take the same 4 FMAs into two registers, Re and Im of
// c conj(p), and skip the conversion.
#include "sweep.h"

namespace t3 {
namespace {

constexpr int kWaves = 4;       // wavefronts (centres) per workgroup
constexpr int kAnchor = 8;      // z^8 steps from the base to the first anchor of a pass above order 8
constexpr int kMaxBins = kMaxRadialBins;
constexpr int kMaxZ = 8;        // neighbour catalogs per launch (tomographic bins)
constexpr int kPartials = 4;    // FP64 partial slots per lane (the P of every plain pass)
constexpr int kFlush = 64;      // batches of 64 neighbours per FP32 run before FP64 promotion

// One launch covers the centres of a chunk against n_z neighbour catalogs
// (n_z = 1 outside tomography).  Task t in [0, n_z n_c) is centre t % n_c
// against catalog order[t / n_c] (catalogs ordered densest first).
struct ScanArgs {
    SweepArgs sw[kMaxZ];    // cell-sorted neighbour catalogs
    float *out[kMaxZ];      // chunk planes per neighbour catalog
    int order[kMaxZ];
    int n_z;
    const int2 *cpos;       // centre positions (chunk-relative)
    int n_c;                // centres in the chunk
    int n_bins;             // bins swept (squared edges e2[0 .. n_bins])
    int B_out;              // bins of the plane layout
    int b_out0;             // swept bin b is stored as bin b_out0 + b
    int n_max;
    int K;                  // chunk capacity (plane layout)
    const short *dest;      // slot -> plane (or -1) for this pass
    unsigned long long *npairs;
    unsigned *queue;        // persistent mode: task counter (zeroed before launch); else null
    int stage;              // single-catalog k_scan: totals staged in LDS, 4-centre rows stored at the end
    int grab;               // persistent mode: tasks taken per counter increment
    double e2[kMaxBins + 1];
};

// First G order of a pass taken only as G_{-m}: a pass whose G orders end
// three above its W capacity C (G_m for m <= n_max - 1 and G_{-m} for
// m <= n_max + 3 with n_max <= C) needs orders C .. C + 3 only as G_{-m}.
constexpr int neg_only_from(int ga, int gb, int wb)
{
    return gb >= ga && gb == wb + 3 ? (wb > ga ? wb : ga) : gb + 1;
}

// Per-pass register footprint.  acc layout: [4 NG S-sums of the +-m order
// pairs][2 NGN (Re, Im) of G_{-m} for the negative-only orders][2 NW W]
// [NX extras].
template <int GA, int GB, int WA, int WB, bool EXTRA>
struct PassShape {
    static constexpr int NEG = neg_only_from(GA, GB, WB);
    static constexpr int NG = NEG - 1 >= GA ? NEG - GA : 0;   // +-m order pairs
    static constexpr int NGN = GB >= NEG ? GB - NEG + 1 : 0;  // negative-only orders
    static constexpr int NW = WB >= WA ? WB - WA + 1 : 0;     // W orders
    static constexpr int NX = EXTRA ? 11 : 0;                  // G0, W0, D terms
    static constexpr int V = 4 * NG + 2 * NGN + 2 * NW + NX;
    static constexpr int P = (V + 63) / 64;                // slots per lane after reduce
    static constexpr int VP = 64 * P;
    static constexpr int M0 = GA > 1 ? ((GA - 1) / kAnchor) * kAnchor : 0;
    static constexpr int MTOP = GB > WB ? GB : WB;
};

// FP64 powers z, z^2, z^4, z^8 of the unit vector z = (dx + i dy) / r.
struct ZPowers {
    double r1, i1, r2, i2, r4, i4, r8, i8;
};

__device__ __forceinline__ ZPowers z_powers(int dx, int dy)
{
    const double xd = (double)dx, yd = (double)dy;
    const double r2 = fma(xd, xd, yd * yd);
    double s = (double)__builtin_amdgcn_rsqf((float)r2);
    s = s * fma(-0.5 * r2 * s, s, 1.5);
    ZPowers z;
    z.r1 = xd * s;
    z.i1 = yd * s;
    z.r2 = fma(z.r1, z.r1, -z.i1 * z.i1);
    z.i2 = 2.0 * z.r1 * z.i1;
    z.r4 = fma(z.r2, z.r2, -z.i2 * z.i2);
    z.i4 = 2.0 * z.r2 * z.i2;
    z.r8 = fma(z.r4, z.r4, -z.i4 * z.i4);
    z.i8 = 2.0 * z.r4 * z.i4;
    return z;
}

// z^E (0 < E < 64) from the binary powers z, z^2, z^4, ... (FP64).
template <int E>
__device__ __forceinline__ void z_power(const ZPowers &z, double &br, double &bi)
{
    static_assert(E > 0 && E < 64, "exponent range");
    double pr = z.r1, pi = z.i1;
    br = 1.0;
    bi = 0.0;
#pragma unroll
    for (int bit = 0; (1 << bit) <= E; ++bit) {
        if (E & (1 << bit)) {
            const double tr = fma(br, pr, -bi * pi);
            bi = fma(br, pi, bi * pr);
            br = tr;
        }
        if ((2 << bit) <= E) {
            const double qr = fma(pr, pr, -pi * pi);
            pi = 2.0 * pr * pi;
            pr = qr;
        }
    }
}

// One neighbour through the recurrence, from its FP64 powers z and the FP64
// base (ar, ai) of the orders: the orders GA .. GB are taken as the powers
// base * z^m (base 1 for the plain passes, z^SEG for the upper order segment;
// UNIT0: the base is 1 at compile time).
// acc layout: [4*NG S-sums][2*NGN G_{-m}][2*NW W][NX extras]
template <int GA, int GB, int WA, int WB, bool EXTRA, int V, bool UNIT0>
__device__ __forceinline__ void accumulate_z(float (&acc)[V], const ZPowers &zp, double ar, double ai, float cr,
                                             float ci, float wt, bool with_extra)
{
    using S = PassShape<GA, GB, WA, WB, EXTRA>;
    static_assert(V == S::V, "accumulator size");
    const double zr = zp.r1, zi = zp.i1, z2r = zp.r2, z2i = zp.i2, z4r = zp.r4, z4i = zp.i4, z8r = zp.r8,
                 z8i = zp.i8;
    const float fzr = (float)zr, fzi = (float)zi;
    // running FP64 anchor a = base z^{M0}
#pragma unroll
    for (int k = 0; k < S::M0 / kAnchor; ++k) {
        const double tr = fma(ar, z8r, -ai * z8i);
        ai = fma(ar, z8i, ai * z8r);
        ar = tr;
    }
    // the sums of one order m with its power (pr, pi)
    auto add = [&](int m, float pr, float pi) {
        if (m >= GA && m < S::NEG) {
            const int k = 4 * (m - GA);
            acc[k + 0] = fmaf(cr, pr, acc[k + 0]);
            acc[k + 1] = fmaf(ci, pi, acc[k + 1]);
            acc[k + 2] = fmaf(cr, pi, acc[k + 2]);
            acc[k + 3] = fmaf(ci, pr, acc[k + 3]);
        } else if (m >= S::NEG && m <= GB) {
            // G_{-m} += c conj(p)
            const int k = 4 * S::NG + 2 * (m - S::NEG);
            acc[k + 0] = fmaf(cr, pr, fmaf(ci, pi, acc[k + 0]));
            acc[k + 1] = fmaf(ci, pr, fmaf(-cr, pi, acc[k + 1]));
        }
        if (m >= WA && m <= WB) {
            const int k = 4 * S::NG + 2 * S::NGN + 2 * (m - WA);
            acc[k + 0] = fmaf(wt, pr, acc[k + 0]);
            acc[k + 1] = fmaf(wt, pi, acc[k + 1]);
        }
    };
    // Powers around an FP32 anchor f = z^a: z^{a+1} = f z by one complex
    // multiplication, z^{a-1} and z^{a+2} from the three-term relation
    // z^{k+1} + z^{k-1} = 2 cos(phi) z^k of a unit z (one FMA per component),
    // each at most two steps from the anchor.  When the anchor is z^0 = 1,
    // z^1 is z itself and z^2 the rounded FP64 square.
    const float tc = 2.0f * fzr;
    auto around = [&](int a, float fr, float fi, bool one) {
        float ur = fzr, ui = fzi;
        if (!one) {
            ur = fmaf(fr, fzr, -fi * fzi);
            ui = fmaf(fr, fzi, fi * fzr);
        }
        add(a - 1, fmaf(tc, fr, -ur), fmaf(tc, fi, -ui));
        add(a, fr, fi);
        add(a + 1, ur, ui);
        if (one)
            add(a + 2, (float)z2r, (float)z2i);
        else
            add(a + 2, fmaf(tc, ur, -fr), fmaf(tc, ui, -fi));
    };
    // FP64 anchors Z_j = a z^{M0 + 4j} (a the base) at every fourth order,
    // each covering orders M0 + 4j - 1 .. M0 + 4j + 2: Z_1 = Z_0 z^4, then
    // the three-term relation Z_{j+1} = 2 cos(4 phi) Z_j - Z_{j-1} (two FMAs
    // per anchor; in FP64 it adds at most about j^2 FP64 ulp, far below one
    // FP32 ulp at any order used here).
    constexpr bool kUnit0 = UNIT0 && S::M0 == 0;
    const double t4 = 2.0 * z4r;
    double cr0 = ar, ci0 = ai, pr0 = 0.0, pi0 = 0.0;
#pragma unroll
    for (int j = 0; S::M0 + 4 * j <= S::MTOP + 1; ++j) {
        const int a0 = S::M0 + 4 * j;
        const bool one = kUnit0 && j == 0;
        around(a0, one ? 1.0f : (float)cr0, one ? 0.0f : (float)ci0, one);
        if (a0 + 3 > S::MTOP) break;
        double nr, ni;
        if (j == 0) {
            nr = one ? z4r : fma(cr0, z4r, -ci0 * z4i);
            ni = one ? z4i : fma(cr0, z4i, ci0 * z4r);
        } else {
            nr = fma(t4, cr0, -pr0);
            ni = fma(t4, ci0, -pi0);
        }
        pr0 = cr0;
        pi0 = ci0;
        cr0 = nr;
        ci0 = ni;
    }
    if (EXTRA && with_extra) {
        constexpr int k = 4 * S::NG + 2 * S::NGN + 2 * S::NW;
        // G_0 += c ; W_0 += w (imaginary part stays 0)
        acc[k + 0] += cr;
        acc[k + 1] += ci;
        acc[k + 2] += wt;
        // z^-2, z^-6 (conjugates of FP64 powers rounded once)
        const float p2r = (float)z2r, p2i = (float)z2i;
        const double z6r = fma(z4r, z2r, -z4i * z2i), z6i = fma(z4r, z2i, z4i * z2r);
        const float p6r = (float)z6r, p6i = (float)z6i;
        const float c2r = fmaf(cr, cr, -ci * ci), c2i = 2.0f * cr * ci;
        const float a2 = fmaf(cr, cr, ci * ci);
        // D6 += c^2 conj(z^6)
        acc[k + 4] = fmaf(c2r, p6r, fmaf(c2i, p6i, acc[k + 4]));
        acc[k + 5] = fmaf(c2i, p6r, fmaf(-c2r, p6i, acc[k + 5]));
        // D2 += c^2 conj(z^2)
        acc[k + 6] = fmaf(c2r, p2r, fmaf(c2i, p2i, acc[k + 6]));
        acc[k + 7] = fmaf(c2i, p2r, fmaf(-c2r, p2i, acc[k + 7]));
        // DA += |c|^2 conj(z^2)
        acc[k + 8] = fmaf(a2, p2r, acc[k + 8]);
        acc[k + 9] = fmaf(-a2, p2i, acc[k + 9]);
        // DW += w^2
        acc[k + 10] = fmaf(wt, wt, acc[k + 10]);
    }
}

// One neighbour (dx, dy, c = cr + i ci, weight wt) through the recurrence.
// SEG > 0 (order segments, see k_scan_seg): when upper is set the orders are
// SEG + GA .. SEG + GB (the chain starts from the FP64 power z^SEG), else GA .. GB.
template <int GA, int GB, int WA, int WB, bool EXTRA, int V, int SEG = 0>
__device__ __forceinline__ void accumulate(float (&acc)[V], int dx, int dy, float cr, float ci,
                                           float wt, bool upper = false, bool with_extra = true)
{
    const ZPowers z = z_powers(dx, dy);
    double ar = 1.0, ai = 0.0;
    if constexpr (SEG > 0) {
        static_assert(GA == 1, "segments start at order 1");
        double br, bi;
        z_power<SEG>(z, br, bi);
        ar = upper ? br : 1.0;
        ai = upper ? bi : 0.0;
    }
    accumulate_z<GA, GB, WA, WB, EXTRA, V, SEG == 0>(acc, z, ar, ai, cr, ci, wt, with_extra);
}

// Cross-lane exchange steps of the reduce-scatter.  Each step halves the
// slots a lane holds: the lane keeps one half and receives its partner's copy
// of that half.  Bits 5 and 4 use the gfx950 permlane swaps (the swap already
// leaves each half on the right lanes); bits 3..0 use DPP permutations fused
// into the add: row_ror:8 (partner l ^ 8), row_half_mirror (partner l ^ 7,
// which differs in bit 2 and agrees on the bits already reduced), and two
// quad permutations (l ^ 2, l ^ 1).  Lane l ends with slots [P l, P l + P).
__device__ __forceinline__ float add_swap32(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float add_swap16(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

constexpr int kDppRowRor8 = 0x128;
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppQuadXor2 = 0x4E;  // quad_perm [2, 3, 0, 1]
constexpr int kDppQuadXor1 = 0xB1;  // quad_perm [1, 0, 3, 2]

template <int CTRL, int H, int N>
__device__ __forceinline__ void dpp_step(float (&v)[N], bool hi)
{
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const float keep = hi ? v[k + H] : v[k];
        const float send = hi ? v[k] : v[k + H];
        v[k] = keep + dpp<CTRL>(send);
    }
}

// Output order of the four slots of an order pair m: Re G_m, Re G_-m, Im G_m,
// Im G_-m (from S1 - S2, S1 + S2, S3 + S4, S4 - S3).
__device__ __forceinline__ void s_to_g(float &s1, float &s2, float &s3, float &s4)
{
    const float a = s1, b = s2, c = s3, d = s4;
    s1 = a - b;
    s2 = a + b;
    s3 = c + d;
    s4 = d - c;
}

// With an even slot count per lane, each (S1, S2) and (S3, S4) pair of the
// reduce-scatter ends on one lane and the conversion waits for the totals.
template <int GA, int GB, int WA, int WB, bool EXTRA>
constexpr bool kConvertAfter = PassShape<GA, GB, WA, WB, EXTRA>::P % 2 == 0;

// Wave reduction of the per-lane accumulators: S -> G conversion unless it
// waits for the totals, then the 6-step reduce-scatter above, after which
// lane l holds the wave totals of slots [P l, P l + P).  These are added to
// the lane's FP64 partials and the FP32 accumulators restart from zero.
// accl: the wavefront's FP64 partials in LDS, slot k of lane l at
// accl[64 k + l] (in LDS rather than registers: the FP32 accumulators of
// the larger passes already fill the register file).
template <int GA, int GB, int WA, int WB, bool EXTRA, int V>
__device__ __forceinline__ void flush(float (&acc)[V], double *accl, int lane)
{
    using S = PassShape<GA, GB, WA, WB, EXTRA>;
    constexpr int VP = S::VP;
    float v[VP];
#pragma unroll
    for (int k = 0; k < S::V; ++k) v[k] = acc[k];
    if constexpr (!kConvertAfter<GA, GB, WA, WB, EXTRA>) {
#pragma unroll
        for (int k = 0; k < S::NG; ++k) s_to_g(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
    }
#pragma unroll
    for (int k = S::V; k < VP; ++k) v[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < VP / 2; ++k) v[k] = add_swap32(v[k], v[k + VP / 2]);
#pragma unroll
    for (int k = 0; k < VP / 4; ++k) v[k] = add_swap16(v[k], v[k + VP / 4]);
    dpp_step<kDppRowRor8, VP / 8>(v, (lane & 8) != 0);
    dpp_step<kDppRowHalfMirror, VP / 16>(v, (lane & 4) != 0);
    dpp_step<kDppQuadXor2, VP / 32>(v, (lane & 2) != 0);
    dpp_step<kDppQuadXor1, VP / 64>(v, (lane & 1) != 0);
#pragma unroll
    for (int k = 0; k < S::P; ++k) accl[64 * k + lane] += (double)v[k];
#pragma unroll
    for (int k = 0; k < S::V; ++k) acc[k] = 0.0f;
}

// Harmonic sums of one centre against one neighbour catalog, every bin.
// stg (else null): the wavefront's column of the workgroup's LDS stage,
// element (slot, bin) at stg[4 (slot n_bins + bin)]; the totals go there
// instead of to the planes.
template <int GA, int GB, int WA, int WB, bool EXTRA>
__device__ __forceinline__ unsigned long long scan_task(const ScanArgs &a, int z, int ci, int lane,
                                                        const SweepLDS &lds, double *accl, float *stg = nullptr)
{
    using S = PassShape<GA, GB, WA, WB, EXTRA>;
    const int2 cp = a.cpos[ci];
    float *out = a.out[z];
    unsigned long long pairs = 0;
    for (int b = 0; b < a.n_bins; ++b) {
        float acc[S::V];
#pragma unroll
        for (int k = 0; k < S::V; ++k) acc[k] = 0.0f;
        static_assert(S::P <= kPartials, "FP64 partial slots");
#pragma unroll
        for (int k = 0; k < S::P; ++k) accl[64 * k + lane] = 0.0;
        int batches = 0;  // wave-uniform: batches since the last FP64 promotion

        pairs += (unsigned long long)sweep_annulus(
            a.sw[z], cp, a.e2[b], a.e2[b + 1], lane, lds,
            [&](const int4 &e, float ew, int, bool) {
                accumulate<GA, GB, WA, WB, EXTRA>(acc, e.x, e.y, __int_as_float(e.z),
                                                  __int_as_float(e.w), ew);
                if (++batches == kFlush) {
                    flush<GA, GB, WA, WB, EXTRA>(acc, accl, lane);
                    batches = 0;
                }
            });
        if (batches > 0) flush<GA, GB, WA, WB, EXTRA>(acc, accl, lane);
        double accd[S::P];
#pragma unroll
        for (int k = 0; k < S::P; ++k) accd[k] = accl[64 * k + lane];
        if constexpr (kConvertAfter<GA, GB, WA, WB, EXTRA>) {
            // slot pairs (2j, 2j + 1) of an order pair are (S1, S2) or (S3, S4)
#pragma unroll
            for (int j = 0; j < S::P / 2; ++j) {
                const int slot = S::P * lane + 2 * j;
                if (slot < 4 * S::NG) {
                    const double x = accd[2 * j], y = accd[2 * j + 1];
                    const bool re = (slot & 2) == 0;
                    accd[2 * j] = re ? x - y : x + y;
                    accd[2 * j + 1] = re ? x + y : y - x;
                }
            }
        }
        // lane holds slots [P*lane, P*lane + P)
#pragma unroll
        for (int k = 0; k < S::P; ++k) {
            const int slot = S::P * lane + k;
            if (stg) {
                if (slot < S::V) stg[4 * (slot * a.n_bins + b)] = (float)accd[k];
            } else {
                const int pl = a.dest[slot];
                if (pl >= 0) out[chunk_offset(pl, ci, a.b_out0 + b, a.K, a.B_out)] = (float)accd[k];
            }
        }
    }
    return pairs;
}

// Store of a workgroup's staged totals: the last of its wavefronts to finish
// writes, per plane, the row of 4 consecutive centres x n_bins bins, which is
// contiguous in the plane layout, as 16-byte vectors (full rows instead of
// 4-byte stores from four wavefronts at different times).  done: the
// workgroup's LDS counter of finished wavefronts, zeroed before any finishes.
template <int V>
__device__ __forceinline__ void store_stage(const ScanArgs &a, int quad, int lane, const float4 *stage, int *done)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    int prev = 0;
    if (lane == 0) prev = atomicAdd(done, 1);
    prev = __shfl(prev, 0, 64);
    const int rem = a.n_c - kWaves * quad;
    const int nq = rem < kWaves ? rem : kWaves;  // centres of this workgroup
    if (prev != nq - 1) return;                  // wave-uniform
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const int nb = a.n_bins;
    const int per = 64 / nb;  // slots per step
    const int ds = lane / nb, b = lane - ds * nb;
    if (ds >= per) return;
    float *out = a.out[0];
    for (int s = ds; s < V; s += per) {
        const int pl = a.dest[s];
        if (pl < 0) continue;
        const float4 v = stage[s * nb + b];
        float *o = out + chunk_offset(pl, kWaves * quad, a.b_out0 + b, a.K, a.B_out);
        if (nq == kWaves) {
            *reinterpret_cast<float4 *>(o) = v;
        } else {
            o[0] = v.x;
            if (nq > 1) o[1] = v.y;
            if (nq > 2) o[2] = v.z;
        }
    }
}

// Two workgroups per CU (2 wavefronts per SIMD): measured faster than one
// wavefront per SIMD without spills, although the largest variants then
// spill some registers.
// GENERAL = false: one catalog, one wavefront per centre (catalog 0 is a
// compile-time choice, which keeps register pressure down; tomography issues
// one such launch per catalog).  GENERAL = true: n_z catalogs in one
// persistent launch with a work counter.
// Workgroup order of the single-catalog kernels.  The hardware deals
// workgroups out round-robin over the 8 XCDs; this map hands each XCD runs
// of kXcdRun consecutive workgroups (4 kXcdRun centres of the cell-sorted
// order), the XCDs' runs side by side.  Each XCD's L2 then holds the
// neighbours of one compact run, while the XCDs stay on the same stretch
// of the chunk and finish together.  It is a bijection on [0, 8 kXcdRun q)
// for whole q, so grids are rounded up to multiples of 8 kXcdRun.
// Measured on the 1M field, stage 1 per step, runs of 32 / 64 / 128 / 256
// workgroups: 775 / 780 / 785 / 798 ms (one box); in plain launch order,
// which misses L2 6.5x as often, 4 ms more than runs of 64, and with each
// XCD on a contiguous eighth of the chunk, whose XCDs finish apart, 16 ms
// more.
constexpr int kXcdRun = 32;
__device__ __forceinline__ int xcd_run_order(int b)
{
    const int x = b & 7, k = b >> 3;
    return ((k / kXcdRun) * 8 + x) * kXcdRun + k % kXcdRun;
}

template <int GA, int GB, int WA, int WB, bool EXTRA, bool GENERAL>
__global__ __launch_bounds__(64 * kWaves, 2) void k_scan(ScanArgs a)
{
    __shared__ int4 q_xyc[kWaves][kRing];
    __shared__ int2 q_wi[kWaves][kRing];
    __shared__ int2 spans[kWaves][2 * kRowsPerBlock + 1];
    __shared__ double partials[kWaves][64 * kPartials];

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: LDS bases stay scalar
    const SweepLDS lds{q_xyc[wv], q_wi[wv], spans[wv]};
    double *accl = partials[wv];
    unsigned long long pairs = 0;
    if constexpr (!GENERAL) {
        // a.stage: [V][n_bins] float4 of dynamic LDS, one float per wavefront
        extern __shared__ float4 stage[];
        __shared__ int done;
        const int wg = xcd_run_order(blockIdx.x);
        const int ci = wg * kWaves + wv;
        if (a.stage) {
            if (threadIdx.x == 0) done = 0;
            __syncthreads();
        }
        if (ci >= a.n_c) return;  // whole wavefront leaves together
        pairs = scan_task<GA, GB, WA, WB, EXTRA>(a, 0, ci, lane, lds, accl,
                                                 a.stage ? reinterpret_cast<float *>(stage) + wv : nullptr);
        if (a.stage) store_stage<PassShape<GA, GB, WA, WB, EXTRA>::V>(a, wg, lane, stage, &done);
        if (lane == 0 && a.npairs) atomicAdd(a.npairs, pairs);
        return;
    }
    const int total = a.n_z * a.n_c;
    int base = 0, end = 0;
    if (!a.queue) {
        // one wavefront per task, tasks in launch order
        base = blockIdx.x * kWaves + wv;
        end = base + 1 < total ? base + 1 : total;
    }
    // persistent mode: take `grab` consecutive tasks per counter increment
    // until the counter passes the task count (every wavefront reaches that exit)
    for (;;) {
        if (a.queue) {
            int b0 = 0;
            if (lane == 0) b0 = (int)atomicAdd(a.queue, (unsigned)a.grab);
            base = __builtin_amdgcn_readfirstlane(b0);
            end = base + a.grab < total ? base + a.grab : total;
        }
        if (base >= total) break;  // wave-uniform
        for (int t = base; t < end; ++t)
            pairs += scan_task<GA, GB, WA, WB, EXTRA>(a, a.order[t / a.n_c], t % a.n_c, lane, lds, accl);
        if (!a.queue) break;
    }
    if (lane == 0 && a.npairs) atomicAdd(a.npairs, pairs);
}

// ---------------------------------------------------------------- order segments
// For n_max above what one pass holds in registers, a wavefront splits its
// orders instead of sweeping every annulus twice: lanes 0-31 accumulate
// orders 1..S of every in-bin neighbour, lanes 32-63 orders S+1..2S.  The code
// is the same for both halves -- the upper one starts its FP64 anchor chain
// at z^S -- and each half takes all 64 neighbours of a batch in two steps
// (first the lower half entries 0-31 and the upper half 32-63, then the other
// way round), so the annulus sweep, the candidate tests and the compaction run
// once per centre and bin.  The j = k sums are accumulated in the first step
// only, so each neighbour's are taken once, by one half or the other, and the
// two halves' totals are added at the end.  The reduce-scatter stays within
// each 32-lane half: permlane16 swaps for lane bit 4, then the same DPP steps
// as the full-wave reduction.
template <int V, int P>
__device__ __forceinline__ void flush_half(float (&acc)[V], double (&accd)[P], int lane, int ng)
{
    constexpr int VP = 32 * P;
    float v[VP];
#pragma unroll
    for (int k = 0; k < V; ++k) v[k] = acc[k];
    // S -> G conversion on the lane partials (P is not even for every shape)
#pragma unroll
    for (int k = 0; k < V / 4; ++k)
        if (k < ng) s_to_g(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
#pragma unroll
    for (int k = V; k < VP; ++k) v[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < VP / 2; ++k) v[k] = add_swap16(v[k], v[k + VP / 2]);
    dpp_step<kDppRowRor8, VP / 4>(v, (lane & 8) != 0);
    dpp_step<kDppRowHalfMirror, VP / 8>(v, (lane & 4) != 0);
    dpp_step<kDppQuadXor2, VP / 16>(v, (lane & 2) != 0);
    dpp_step<kDppQuadXor1, VP / 32>(v, (lane & 1) != 0);
#pragma unroll
    for (int k = 0; k < P; ++k) accd[k] += (double)v[k];
#pragma unroll
    for (int k = 0; k < V; ++k) acc[k] = 0.0f;
}

// zp: the wavefront's LDS table of the batch entries' FP64 powers, [5][64]:
// z, z^2, z^4, z^8 and z^SW of entry j at zp[q][j] (computed once per entry,
// read by the lower-half and the upper-half lane that take it).
template <int SW>
__device__ __forceinline__ unsigned long long scan_task_seg(const ScanArgs &a, int ci, int lane, const SweepLDS &lds,
                                                            double2 (*zp)[64])
{
    using S = PassShape<1, SW, 1, SW, true>;
    constexpr int P = (S::V + 31) / 32;   // slots per lane after the half-wave reduction
    constexpr int VP = 32 * P;
    const int2 cp = a.cpos[ci];
    float *out = a.out[0];
    const bool upper = lane >= 32;
    const int h = lane & 31;
    unsigned long long pairs = 0;
    for (int b = 0; b < a.n_bins; ++b) {
        float acc[S::V];
#pragma unroll
        for (int k = 0; k < S::V; ++k) acc[k] = 0.0f;
        double accd[P];
#pragma unroll
        for (int k = 0; k < P; ++k) accd[k] = 0.0;
        int batches = 0;  // wave-uniform
        pairs += (unsigned long long)sweep_annulus_halves(
            a.sw[0], cp, a.e2[b], a.e2[b + 1], lane, lds,
            [&](const int4 &e, int j) {
                const ZPowers z = z_powers(e.x, e.y);
                double br, bi;
                z_power<SW>(z, br, bi);
                zp[0][j] = make_double2(z.r1, z.i1);
                zp[1][j] = make_double2(z.r2, z.i2);
                zp[2][j] = make_double2(z.r4, z.i4);
                zp[3][j] = make_double2(z.r8, z.i8);
                zp[4][j] = make_double2(br, bi);
            },
            [&](const int4 &e, float ew, int step, int j) {
                const double2 p1 = zp[0][j], p2 = zp[1][j], p4 = zp[2][j], p8 = zp[3][j], pb = zp[4][j];
                const ZPowers z{p1.x, p1.y, p2.x, p2.y, p4.x, p4.y, p8.x, p8.y};
                accumulate_z<1, SW, 1, SW, true, S::V, false>(acc, z, upper ? pb.x : 1.0, upper ? pb.y : 0.0,
                                                              __int_as_float(e.z), __int_as_float(e.w), ew,
                                                              step == 0);
            },
            [&]() {
                // two neighbours per lane per batch: FP32 runs of at most 64 terms
                if (++batches == kFlush / 2) {
                    flush_half<S::V, P>(acc, accd, lane, S::NG);
                    batches = 0;
                }
            });
        if (batches > 0) flush_half<S::V, P>(acc, accd, lane, S::NG);
        // half (lane >> 5) holds slots [P h, P h + P) of its segment; the j = k
        // sums (slots 6 S and up) are split between the halves: add them
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const double other = __shfl_xor(accd[k], 32, 64);
            if (P * h + k >= 6 * SW) accd[k] += other;
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int pl = a.dest[(upper ? VP : 0) + P * h + k];
            if (pl >= 0) out[chunk_offset(pl, ci, a.b_out0 + b, a.K, a.B_out)] = (float)accd[k];
        }
    }
    return pairs;
}

// One wavefront per centre, two order segments per wavefront (one catalog).
template <int SW>
__global__ __launch_bounds__(64 * kWaves, 2) void k_scan_seg(ScanArgs a)
{
    __shared__ int4 q_xyc[kWaves][kRing];
    __shared__ int2 q_wi[kWaves][kRing];
    __shared__ int2 spans[kWaves][2 * kRowsPerBlock + 1];
    __shared__ double2 zpow[kWaves][5][64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: LDS bases stay scalar
    const SweepLDS lds{q_xyc[wv], q_wi[wv], spans[wv]};
    const int ci = xcd_run_order(blockIdx.x) * kWaves + wv;
    if (ci >= a.n_c) return;  // whole wavefront leaves together
    const unsigned long long pairs = scan_task_seg<SW>(a, ci, lane, lds, zpow[wv]);
    if (lane == 0 && a.npairs) atomicAdd(a.npairs, pairs);
}

// Lane per centre, for bins with few neighbours per centre: the wavefront's
// 64 centres are swept independently (each lane walks its own cell rows), so
// the per-(centre, bin) cost follows the neighbour count instead of a full
// 64-lane batch plus a 64-lane reduction.  Each lane first collects up to
// kLaneList in-bin neighbours (indices in LDS), then the wavefront runs the
// same per-pair arithmetic on the lists in lock-step (max count iterations)
// and goes back to collecting until every lane has finished its annulus.
// Sums stay in FP32 per lane (sequential rounding of the ~170 terms of the
// Poisson tail at 128 expected neighbours is below 3e-7 relative).  Two
// wavefronts per SIMD (256 VGPRs, a few spills) measured 10% faster than one.
constexpr int kLaneList = 32;
constexpr int kLaneBlock = 128;

template <int GA, int GB, int WA, int WB, bool EXTRA>
__global__ __launch_bounds__(kLaneBlock, 2) void k_scan_lane(ScanArgs a)
{
    using S = PassShape<GA, GB, WA, WB, EXTRA>;
    __shared__ int list[kLaneList][kLaneBlock];
    const int t = threadIdx.x;
    const int ci = blockIdx.x * kLaneBlock + t;
    const bool active = ci < a.n_c;
    const int2 cp = active ? a.cpos[ci] : make_int2(0, 0);
    const SweepArgs &sw = a.sw[0];
    const CellGrid &g = sw.g;
    float *out = a.out[0];
    unsigned long long pairs = 0;
    {
        const int b = blockIdx.y;  // one bin per grid row: short, evenly spread wavefronts
        const double e2lo = a.e2[b], e2hi = a.e2[b + 1];
        float acc[S::V];
#pragma unroll
        for (int k = 0; k < S::V; ++k) acc[k] = 0.0f;
        // this lane's walk: rows [row, row_hi], current range [gi, gend), second range of the row pending
        const long long R = (long long)sqrt(e2hi) + 1;
        long long row = floor_div((long long)cp.y - R - g.oy, g.cell);
        long long row_hi = floor_div((long long)cp.y + R - g.oy, g.cell);
        row = row < 0 ? 0 : row;
        row_hi = row_hi > g.ncy - 1 ? g.ncy - 1 : row_hi;
        if (!active) row_hi = row - 1;
        int gi = 0, gend = 0;
        int2 second = make_int2(0, 0);
        bool have_second = false;
        for (;;) {
            // collect: up to kLaneList in-bin neighbours or the end of the annulus
            int cnt = 0;
            bool done = false;
            while (cnt < kLaneList) {
                if (gi + 4 <= gend && cnt + 4 <= kLaneList) {
                    // four independent loads in flight (two wavefronts per SIMD hide little latency)
                    int2 p[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) p[u] = sw.npos[gi + u];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int dx = p[u].x - cp.x, dy = p[u].y - cp.y;
                        const double r2 = fma((double)dx, (double)dx, (double)dy * (double)dy);
                        if (r2 >= e2lo && r2 < e2hi) list[cnt++][t] = gi + u;
                    }
                    gi += 4;
                } else if (gi < gend) {
                    const int2 p = sw.npos[gi];
                    const int dx = p.x - cp.x, dy = p.y - cp.y;
                    const double r2 = fma((double)dx, (double)dx, (double)dy * (double)dy);
                    if (r2 >= e2lo && r2 < e2hi) list[cnt++][t] = gi;
                    ++gi;
                } else if (have_second) {
                    gi = second.x;
                    gend = second.y;
                    have_second = false;
                } else if (row <= row_hi) {
                    int2 sa, sb;
                    row_ranges(sw, cp, row, e2lo, e2hi, sa, sb);
                    ++row;
                    gi = sa.x;
                    gend = sa.y;
                    second = sb;
                    have_second = sb.y > sb.x;
                } else {
                    done = true;
                    break;
                }
            }
            pairs += (unsigned long long)cnt;
            // process the lists in lock-step; the next neighbour's loads are
            // issued before the current one's arithmetic
            int most = cnt;
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) most = max(most, __shfl_xor(most, d, 64));
            int2 pc = make_int2(cp.x, cp.y);
            float4 cc = make_float4(0.f, 0.f, 0.f, 0.f);
            if (cnt > 0) {
                const int j = list[0][t];
                pc = sw.npos[j];
                cc = sw.ncw[j];
            }
            for (int k = 0; k < most; ++k) {
                int2 pn = pc;
                float4 cn = cc;
                if (k + 1 < cnt) {
                    const int j = list[k + 1][t];
                    pn = sw.npos[j];
                    cn = sw.ncw[j];
                }
                if (k < cnt) accumulate<GA, GB, WA, WB, EXTRA>(acc, pc.x - cp.x, pc.y - cp.y, cc.x, cc.y, cc.z);
                pc = pn;
                cc = cn;
            }
            if (__all(done)) break;
        }
        if (active) {
            // S -> G conversion (slot order as in the wavefront reduction), then every slot to its plane
#pragma unroll
            for (int k = 0; k < S::NG; ++k) s_to_g(acc[4 * k], acc[4 * k + 1], acc[4 * k + 2], acc[4 * k + 3]);
#pragma unroll
            for (int k = 0; k < S::V; ++k) {
                const int pl = a.dest[k];
                if (pl >= 0) out[chunk_offset(pl, ci, a.b_out0 + b, a.K, a.B_out)] = acc[k];
            }
        }
    }
    // one atomic per wavefront
    unsigned long long tot = pairs;
    for (int d = 32; d > 0; d >>= 1) tot += __shfl_xor(tot, d, 64);
    if ((t & 63) == 0 && a.npairs && tot) atomicAdd(a.npairs, tot);
}

__global__ void k_zero_u32(unsigned *p) { *p = 0u; }

// --------------------------------------------------------------- host side
struct PassDesc {
    int ga, gb, wa, wb;
    bool extra;
    void (*kernel)(ScanArgs);          // single catalog, one wavefront per centre
    void (*kernel_general)(ScanArgs);  // n_z catalogs, either launch mode
    void (*kernel_lane)(ScanArgs);     // single catalog, one lane per centre (small bins)
};

// Accumulator slots of a pass (the V of its PassShape).
inline int pass_slots(const PassDesc &p)
{
    const int NEG = neg_only_from(p.ga, p.gb, p.wb);
    const int NG = NEG - 1 >= p.ga ? NEG - p.ga : 0;
    const int NGN = p.gb >= NEG ? p.gb - NEG + 1 : 0;
    const int NW = p.wb >= p.wa ? p.wb - p.wa + 1 : 0;
    return 4 * NG + 2 * NGN + 2 * NW + (p.extra ? 11 : 0);
}

// Dynamic LDS for staged totals: with the rings and the FP64 partials
// (about 24 KB) a workgroup stays within 64 KB, two workgroups per CU.
constexpr size_t kStageBytes = 38 * 1024;

template <int GA, int GB, int WA, int WB, bool EXTRA>
PassDesc make_pass()
{
    return PassDesc{GA, GB, WA, WB, EXTRA, k_scan<GA, GB, WA, WB, EXTRA, false>,
                    k_scan<GA, GB, WA, WB, EXTRA, true>, k_scan_lane<GA, GB, WA, WB, EXTRA>};
}

// Variant table: a single pass for n_max up to the capacity C (orders
// 1..C+3 for G, 1..C for W); two passes beyond 32.  wext: the W-only pass
// over orders C+1..2C, run when the plan needs N_n up to 2 n_max (mode
// coupling); its power recurrence starts from the FP64 anchor below C+1.
struct Variant {
    int cap;
    int npass;
    PassDesc pass[2];
    PassDesc wext;
    int seg = 0;                        // order-segment width of k_scan_seg (0: none)
    void (*kernel_seg)(ScanArgs) = nullptr;
};

template <int C>
PassDesc make_wext()
{
    return make_pass<C + 1, C, C + 1, 2 * C, false>();
}

// Workgroups of a single-catalog launch over n_c centres, in whole rounds of
// the XCD run order.
int xcd_run_grid(int n_c)
{
    const int round = 8 * kXcdRun;
    return ((n_c + kWaves - 1) / kWaves + round - 1) / round * round;
}

const std::vector<Variant> &variants()
{
    static const std::vector<Variant> v = {
        {2, 1, {make_pass<1, 5, 1, 2, true>()}, make_wext<2>()},
        {4, 1, {make_pass<1, 7, 1, 4, true>()}, make_wext<4>()},
        {8, 1, {make_pass<1, 11, 1, 8, true>()}, make_wext<8>()},
        {10, 1, {make_pass<1, 13, 1, 10, true>()}, make_wext<10>()},
        {12, 1, {make_pass<1, 15, 1, 12, true>()}, make_wext<12>()},
        {16, 1, {make_pass<1, 19, 1, 16, true>()}, make_wext<16>()},
        {20, 1, {make_pass<1, 23, 1, 20, true>()}, make_wext<20>()},
        {24, 1, {make_pass<1, 27, 1, 24, true>()}, make_wext<24>()},
        {30, 1, {make_pass<1, 33, 1, 30, true>()}, make_wext<30>()},
        {32, 1, {make_pass<1, 35, 1, 32, true>()}, make_wext<32>()},
        {40, 2, {make_pass<1, 22, 1, 20, true>(), make_pass<23, 43, 21, 40, false>()}, make_wext<40>(), 22,
         k_scan_seg<22>},
        {48, 2, {make_pass<1, 26, 1, 24, true>(), make_pass<27, 51, 25, 48, false>()}, make_wext<48>(), 26,
         k_scan_seg<26>},
        {64, 2, {make_pass<1, 34, 1, 32, true>(), make_pass<35, 67, 33, 64, false>()}, make_wext<64>()},
    };
    return v;
}

// Destination table of one pass for a given n_max: slot -> plane or -1.
std::vector<short> dest_table(const PassDesc &p, const ChunkLayout &L)
{
    const int NEG = neg_only_from(p.ga, p.gb, p.wb);
    const int NG = NEG - 1 >= p.ga ? NEG - p.ga : 0;
    const int NGN = p.gb >= NEG ? p.gb - NEG + 1 : 0;
    const int NW = p.wb >= p.wa ? p.wb - p.wa + 1 : 0;
    const int V = 4 * NG + 2 * NGN + 2 * NW + (p.extra ? 11 : 0);
    const int VP = 64 * ((V + 63) / 64);
    std::vector<short> d(VP, -1);
    const int nm = L.n_max;
    for (int k = 0; k < NG; ++k) {
        const int m = p.ga + k;
        // slot order Re G_m, Re G_-m, Im G_m, Im G_-m
        if (m <= nm - 1) {
            d[4 * k + 0] = (short)L.plane_G(m, 0);
            d[4 * k + 2] = (short)L.plane_G(m, 1);
        }
        if (m <= nm + 3) {
            d[4 * k + 1] = (short)L.plane_G(-m, 0);
            d[4 * k + 3] = (short)L.plane_G(-m, 1);
        }
    }
    for (int k = 0; k < NGN; ++k) {
        // slot order Re G_-m, Im G_-m
        const int m = NEG + k;
        if (m <= nm + 3) {
            d[4 * NG + 2 * k] = (short)L.plane_G(-m, 0);
            d[4 * NG + 2 * k + 1] = (short)L.plane_G(-m, 1);
        }
    }
    for (int k = 0; k < NW; ++k) {
        const int m = p.wa + k;
        if (m <= L.w_max) {
            d[4 * NG + 2 * NGN + 2 * k] = (short)L.plane_W(m, 0);
            d[4 * NG + 2 * NGN + 2 * k + 1] = (short)L.plane_W(m, 1);
        }
    }
    if (p.extra) {
        const int k = 4 * NG + 2 * NGN + 2 * NW;
        if (nm >= 1) {  // G_0 is needed only for n_max >= 1
            d[k + 0] = (short)L.plane_G(0, 0);
            d[k + 1] = (short)L.plane_G(0, 1);
        }
        d[k + 2] = (short)L.plane_W(0, 0);
        d[k + 3] = (short)L.plane_W(0, 1);  // stays zero
        for (int j = 0; j < 7; ++j) d[k + 4 + j] = (short)L.plane_D(j);
    }
    return d;
}

// Destination table of k_scan_seg: [2 halves][32 P] slots -> plane or -1.
// Half h holds orders h S + 1 .. h S + S (G pairs, then W), then the extra
// sums, of which only the lower half's are kept; W orders above the
// variant's capacity belong to the W-extension pass.
std::vector<short> dest_table_seg(int S, int cap, const ChunkLayout &L)
{
    const int V = 6 * S + 11;
    const int VP = 32 * ((V + 31) / 32);
    std::vector<short> d(2 * VP, -1);
    const int nm = L.n_max;
    for (int h = 0; h < 2; ++h) {
        short *t = d.data() + h * VP;
        for (int k = 0; k < S; ++k) {
            const int m = h * S + 1 + k;
            if (m <= nm - 1) {
                t[4 * k + 0] = (short)L.plane_G(m, 0);
                t[4 * k + 2] = (short)L.plane_G(m, 1);
            }
            if (m <= nm + 3) {
                t[4 * k + 1] = (short)L.plane_G(-m, 0);
                t[4 * k + 3] = (short)L.plane_G(-m, 1);
            }
            if (m <= L.w_max && m <= cap) {
                t[4 * S + 2 * k] = (short)L.plane_W(m, 0);
                t[4 * S + 2 * k + 1] = (short)L.plane_W(m, 1);
            }
        }
        if (h == 0) {
            const int k = 6 * S;
            if (nm >= 1) {
                t[k + 0] = (short)L.plane_G(0, 0);
                t[k + 1] = (short)L.plane_G(0, 1);
            }
            t[k + 2] = (short)L.plane_W(0, 0);
            t[k + 3] = (short)L.plane_W(0, 1);  // stays zero
            for (int j = 0; j < 7; ++j) t[k + 4 + j] = (short)L.plane_D(j);
        }
    }
    return d;
}

}  // namespace

namespace {
// Every destination table of the plan's stage-1 variant, and their offsets.
int dest_tables(const t3_plan *plan, std::vector<short> &all, size_t off[4], int *var_index)
{
    const auto &vars = variants();
    int vi = -1;
    for (size_t i = 0; i < vars.size(); ++i)
        if (vars[i].cap >= plan->n_max) {
            vi = (int)i;
            break;
        }
    if (vi < 0) return fail(T3_ERANGE, "n_max above the largest compiled variant");
    ChunkLayout L;
    L.n_max = plan->n_max;
    L.w_max = plan->w_max;
    L.B = plan->B;
    all.clear();
    for (int p = 0; p < vars[vi].npass; ++p) {
        off[p] = all.size();
        auto d = dest_table(vars[vi].pass[p], L);
        all.insert(all.end(), d.begin(), d.end());
    }
    if (plan->w_max > vars[vi].cap) {
        off[vars[vi].npass] = all.size();
        auto d = dest_table(vars[vi].wext, L);
        all.insert(all.end(), d.begin(), d.end());
    }
    if (vars[vi].seg > 0) {
        off[3] = all.size();
        auto d = dest_table_seg(vars[vi].seg, vars[vi].cap, L);
        all.insert(all.end(), d.begin(), d.end());
    }
    *var_index = vi;
    return T3_OK;
}
}  // namespace

bool scan_uses_segments(const t3_plan *plan)
{
    for (const Variant &v : variants())
        if (v.cap >= plan->n_max) return v.kernel_seg != nullptr;
    return false;
}

size_t scan_dest_entries(const t3_plan *plan)
{
    std::vector<short> all;
    size_t off[4] = {0, 0, 0, 0};
    int vi = -1;
    return dest_tables(plan, all, off, &vi) == T3_OK ? all.size() : 0;
}

int scan_prepare(t3_plan *plan)
{
    std::vector<short> all;
    size_t off[4] = {0, 0, 0, 0};
    int vi = -1;
    T3_TRY(dest_tables(plan, all, off, &vi));
    for (int k = 0; k < 4; ++k) plan->scan_dest_off[k] = off[k];
    T3_TRY(plan->dest.reserve(all.size() * sizeof(short)));
    T3_HIP_CHECK(hipMemcpy(plan->dest.ptr, all.data(), all.size() * sizeof(short), hipMemcpyHostToDevice));
    plan->scan_var = vi;
    return T3_OK;
}

int scan_chunk(t3_plan *plan, const SortedCatalog *const *cats, const int *order, int n_z,
               const CentreSet &cs, int64_t c0, int n_c, const ChunkLayout &L, float *planes,
               size_t zstride, unsigned long long *npairs, int mode, hipStream_t s, int b0, int nb, int n_lane)
{
    if (n_c <= 0) return T3_OK;
    if (nb < 0) nb = L.B;
    if (b0 < 0 || nb < 1 || nb > L.B || b0 + nb > plan->B) return fail(T3_ERANGE, "scan: bad bin range");
    if (n_lane < 0 || n_lane > nb) return fail(T3_ERANGE, "scan: bad lane-bin count");
    if (n_z < 1 || n_z > kMaxZ) return fail(T3_ERANGE, "scan: bad catalog count");
    if (plan->scan_var < 0) T3_TRY(scan_prepare(plan));
    const Variant &var = variants()[plan->scan_var];
    ScanArgs a{};
    for (int z = 0; z < n_z; ++z) {
        const SortedCatalog &sc = *cats[z];
        a.sw[z].npos = sc.pos.as<int2>();
        a.sw[z].ncw = sc.cw.as<float4>();
        a.sw[z].cell_start = sc.cell_start.as<int>();
        a.sw[z].g = sc.grid;
        a.out[z] = planes + (size_t)z * zstride;
        a.order[z] = order ? order[z] : z;
    }
    a.n_z = n_z;
    a.cpos = cs.pos.as<int2>() + c0;
    a.n_c = n_c;
    a.B_out = L.B;
    a.n_max = L.n_max;
    a.K = L.K;
    const int npass = var.npass + (plan->w_max > var.cap ? 1 : 0);
    // bins [b0, b0 + n_lane): one lane per centre, one launch per catalog
    if (n_lane > 0) {
        ScanArgs al = a;
        al.n_bins = n_lane;
        al.b_out0 = 0;
        al.n_z = 1;
        for (int b = 0; b <= n_lane; ++b) al.e2[b] = plan->e2[b0 + b];
        for (int p = 0; p < npass; ++p) {
            const PassDesc &pd = p < var.npass ? var.pass[p] : var.wext;
            al.dest = plan->dest.as<short>() + plan->scan_dest_off[p];
            al.npairs = p == 0 ? npairs : nullptr;
            for (int z = 0; z < n_z; ++z) {
                ScanArgs a1 = al;
                a1.sw[0] = a.sw[z];
                a1.out[0] = a.out[z];
                hipLaunchKernelGGL(pd.kernel_lane,
                                   dim3((unsigned)((n_c + kLaneBlock - 1) / kLaneBlock), (unsigned)n_lane),
                                   dim3(kLaneBlock), 0, s, a1);
                T3_HIP_CHECK(hipGetLastError());
            }
        }
    }
    if (n_lane == nb) return T3_OK;
    // bins [b0 + n_lane, b0 + nb): one wavefront per centre
    a.n_bins = nb - n_lane;
    a.b_out0 = n_lane;
    for (int b = 0; b <= a.n_bins; ++b) a.e2[b] = plan->e2[b0 + n_lane + b];
    const int total = n_z * n_c;
    int nwg;
    if (mode == 1) {
        // persistent grid: two workgroups per CU
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        nwg = 2 * cus;
        T3_TRY(plan->queue.reserve(sizeof(unsigned) * 4));
        a.queue = plan->queue.as<unsigned>();
        a.grab = 4;
    } else {
        nwg = (total + kWaves - 1) / kWaves;
        a.queue = nullptr;
        a.grab = 0;
    }
    const bool seg = var.kernel_seg && !a.queue;
    for (int p = seg ? var.npass - 1 : 0; p < npass; ++p) {
        const PassDesc &pd = p < var.npass ? var.pass[p] : var.wext;
        a.dest = plan->dest.as<short>() + plan->scan_dest_off[p];
        a.npairs = p == 0 ? npairs : nullptr;  // count pairs once
        if (seg && p < var.npass) {
            // every main-pass order in one sweep: k_scan_seg stands for the passes
            a.dest = plan->dest.as<short>() + plan->scan_dest_off[3];
            a.npairs = npairs;
            const int nwg1 = xcd_run_grid(n_c);
            for (int k = 0; k < n_z; ++k) {
                ScanArgs a1 = a;
                const int z = a.order[k];
                a1.sw[0] = a.sw[z];
                a1.out[0] = a.out[z];
                a1.n_z = 1;
                hipLaunchKernelGGL(var.kernel_seg, dim3((unsigned)nwg1), dim3(64 * kWaves), 0, s, a1);
                T3_HIP_CHECK(hipGetLastError());
            }
            continue;
        }
        if (a.queue) {
            // persistent grid over every (centre, catalog) task
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, a.queue);
            T3_HIP_CHECK(hipGetLastError());
            hipLaunchKernelGGL(pd.kernel_general, dim3((unsigned)nwg), dim3(64 * kWaves), 0, s, a);
            T3_HIP_CHECK(hipGetLastError());
        } else {
            // one launch of the single-catalog kernel per catalog, densest first;
            // the totals go through LDS when the workgroup's rows fit
            const int nwg1 = xcd_run_grid(n_c);
            const size_t stage_bytes = sizeof(float4) * (size_t)pass_slots(pd) * (size_t)a.n_bins;
            const bool stage = stage_bytes <= kStageBytes;
            for (int k = 0; k < n_z; ++k) {
                ScanArgs a1 = a;
                const int z = a.order[k];
                a1.sw[0] = a.sw[z];
                a1.out[0] = a.out[z];
                a1.n_z = 1;
                a1.stage = stage ? 1 : 0;
                hipLaunchKernelGGL(pd.kernel, dim3((unsigned)nwg1), dim3(64 * kWaves), stage ? stage_bytes : 0, s,
                                   a1);
                T3_HIP_CHECK(hipGetLastError());
            }
        }
    }
    return T3_OK;
}

}  // namespace t3
