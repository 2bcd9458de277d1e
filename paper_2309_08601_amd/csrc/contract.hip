// Stage 2 of the multipole estimator: the contraction over centres
//     Upsilon_{mu,n}(b1, b2) = sum_i X_{mu,n}(i, b1) Y_{mu,n}(i, b2)
// (Porth et al. 2023, eqs. Upsilon0_Derivation, Upsilon1-3,
// 3PCF_Normalization), one small complex GEMM (B x B, K = centres) per
// (mu, n), run on MFMA.  With c = w (g1 + i g2) of the centre:
//     mu = 0: X = -c  G_{n-3},        Y = G_{-n-3}
//     mu = 1: X = -c* G_{n-1},        Y = G_{-n-1}
//     mu = 2: X = -c  conj G_{-n-1},  Y = G_{-n-3}
//     mu = 3: X = -c  G_{n-3},        Y = conj G_{n-1}
//     mu = 4: X =  w  W_n,            Y = conj W_n       (normaliser N_n)
// A complex product is four real MFMAs: Re += Xr Yr - Xi Yi, Im += Xr Yi + Xi Yr.
//
// Work decomposition (B > 24; blocks of at most 24 bins take the real-
// embedded 16 x 16 kernel k_contract_small below): a workgroup of four
// wavefronts owns one n (the four shear components, one wavefront each) or
// two orders of N, one slice of centres and one 32 x 32 tile of the B x B
// block (grid.y; one tile for B <= 40, four for B = 41..64).  For B = 33..40 only the first tile runs on
// MFMA: the outputs with a bin index of 32 or more (at most 8 rows and
// columns) are summed by k_contract_edge on the vector ALUs (FP32 runs of
// 16 centres promoted to FP64, as the FP32 MFMA runs), rather
// than by three more MFMA tiles holding at most 8 real rows or columns each.
// The operands the four products share (mu = 0
// and 3 have the same X, mu = 0 and 2 the same Y) are formed once per block
// of 16 centres:
// the whole workgroup loads the harmonic planes with coalesced float4 reads,
// multiplies in the centre factor, splits into hi / lo parts where the
// precision asks for it, and stores MFMA-ready rows in LDS; the next block's
// loads are issued before the MFMAs of the current one.  FP32 MFMA runs of
// 16 centres (one block) are promoted into FP64 accumulators, and the slices
// are summed in FP64 in a fixed order (deterministic).  (Runs of 64 centres
// left the FP32 accumulation a third of the worst-block error of small
// samples: 9.2e-7 against 6.4e-7, for 7% more stage-2 time.)  The j = k terms (n-independent,
// diagonal only) are summed separately in FP64 and subtracted in the final
// reduction.
//
// Precision variants of the Upsilon products (N_n is always FP32):
//  * FP32:    v_mfma_f32_32x32x2_f32.
//  * BF16X3:  x = hi + lo, hi = bf16(x), lo = bf16(x - hi) (about 16 bits);
//             hi*hi + hi*lo + lo*hi on v_mfma_f32_32x32x16_bf16 (B > 24;
//             the 16 x 16 kernel of B <= 24 adds lo*lo at no cost).
//  * BF16X6:  x = hi + mid + lo (every FP32 bit); the six products whose
//             part orders sum to at most 2 (dropped terms are below
//             2^-24 |x y|).
//  * FP16X3:  as BF16X3 in fp16 (about 22 bits) after scaling each operand
//             row (array, bin) by a power of two that brings its largest
//             entry into [2^11, 2^12), keeping lo out of the subnormals; the
//             scales are divided out in FP64.
#include <type_traits>

#include "t3_internal.h"

namespace t3 {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

constexpr int kBlk = 16;   // centres staged through LDS per step
constexpr int kRun = 16;   // centres per FP32 accumulation run before FP64 promotion (one block)
constexpr int kSliceStep = 64;  // slice lengths are multiples of this
constexpr int kRows = 32;  // tile rows and columns (bins)
constexpr int kScaleRows = kMaxRadialBins;  // fp16 row scales per operand array
constexpr int kNYArr = 6;  // complex operand arrays of the Upsilon kernel

// One launch covers every ordered pair (Z2, Z3) of neighbour catalogs
// (grid.z = n_z^2; n_z = 1 outside tomography): the X-side harmonics come
// from the planes of Z2, the Y-side ones from those of Z3.
struct ContractArgs {
    const float *planes; // planes of catalog 0; catalog z at planes + z * zstride
    size_t zstride;
    const float4 *ccw;   // centre factors (w g1, w g2, w, 0), chunk-relative
    const float *scale;  // fp16 row scales [pair][n][kNYArr][kScaleRows] or null
    int n_c, K, B, n_max, n_z;
    int w_max;           // largest order of N (n_max, or 2 n_max for mode coupling)
    int slice;           // centres per slice (multiple of kSliceStep)
    int S;               // slices
    int nt;              // MFMA tiles per side of the B x B block (grid.y = nt^2)
    double *partial;     // [pair][S][4 (n_max+1) + w_max + 1][B][B][2]
};

__device__ __forceinline__ void pair_planes(const ContractArgs &a, int pair, const float *&px,
                                            const float *&py)
{
    px = a.planes + (size_t)(pair / a.n_z) * a.zstride;
    py = a.planes + (size_t)(pair % a.n_z) * a.zstride;
}

__device__ __forceinline__ int plane_g(int m, int n_max) { return 2 * (m + n_max + 3); }
__device__ __forceinline__ int plane_w(int m, int n_max) { return 2 * (2 * n_max + 3) + 2 * m; }

// X-side operands of the Upsilon kernel for centre factor c = (cr, ci):
//   o0 = -c G_{n-3},  o1 = -c* G_{n-1},  o2 = -c conj G_{-n-1}.
__device__ __forceinline__ void x_operands(float cr, float ci, float2 g3, float2 g1, float2 gm1,
                                           float2 (&o)[3])
{
    o[0] = make_float2(-fmaf(cr, g3.x, -ci * g3.y), -fmaf(cr, g3.y, ci * g3.x));
    o[1] = make_float2(-fmaf(cr, g1.x, ci * g1.y), -fmaf(cr, g1.y, -ci * g1.x));
    o[2] = make_float2(-fmaf(cr, gm1.x, ci * gm1.y), -fmaf(ci, gm1.x, -cr * gm1.y));
}

// alpha_i of component mu from (w g1, w g2, w): the factor that multiplies
// the j = k sums.
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

// ------------------------------------------------------------ formats
// LDS row of one real operand array and bin: the P parts of kBlk centres side
// by side, plus 16 bytes of padding (one or two parts) so that 16 consecutive
// lanes reading 16 bytes each at rows r..r+15 hit 16 disjoint groups of four
// banks.
template <int PK> struct Fmt;
template <> struct Fmt<T3_PREC_FP32> {
    using T = float;
    static constexpr int parts = 1;
};
template <> struct Fmt<T3_PREC_BF16X3> {
    using T = __bf16;
    using V = bf16x8;
    static constexpr int parts = 2;
};
template <> struct Fmt<T3_PREC_FP16X3> {
    using T = _Float16;
    using V = halfx8;
    static constexpr int parts = 2;
};
template <> struct Fmt<T3_PREC_BF16X6> {
    using T = __bf16;
    using V = bf16x8;
    static constexpr int parts = 3;
};
template <int PK>
constexpr int row_elems()
{
    // (three-part rows stay unpadded: two double-buffered workgroups per CU
    // fit the LDS only that way; the cost is a two-way read conflict)
    using T = typename Fmt<PK>::T;
    return (Fmt<PK>::parts * kBlk * (int)sizeof(T) + (Fmt<PK>::parts == 3 ? 0 : 16)) / (int)sizeof(T);
}

typedef float float2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 halfx2 __attribute__((ext_vector_type(2)));

// Packs the split of two FP32 values: out[p] holds part p of (x0, x1) as
// two 16-bit values, x = part 0 + part 1 [+ part 2].  Each residual
// x - part is exact (a subtraction of a rounding of x from x).
template <int PK>
__device__ __forceinline__ void split2(float x0, float x1, uint32_t (&out)[Fmt<PK>::parts])
{
    using T2 = typename std::conditional<PK == T3_PREC_FP16X3, halfx2, bf16x2>::type;
#pragma unroll
    for (int p = 0; p < Fmt<PK>::parts; ++p) {
        const T2 t = __builtin_convertvector((float2v){x0, x1}, T2);
        out[p] = __builtin_bit_cast(uint32_t, t);
        if (p + 1 < Fmt<PK>::parts) {
            x0 -= (float)t[0];
            x1 -= (float)t[1];
        }
    }
}

// Writes 4 consecutive centres of one real operand row into LDS (row points
// at the row's first element; the parts of the row are kBlk elements apart).
template <int PK>
__device__ __forceinline__ void put4(typename Fmt<PK>::T *row, float v0, float v1, float v2, float v3)
{
    if constexpr (PK == T3_PREC_FP32) {
        *reinterpret_cast<float4 *>(row) = make_float4(v0, v1, v2, v3);
    } else {
        uint32_t lo[Fmt<PK>::parts], hi[Fmt<PK>::parts];
        split2<PK>(v0, v1, lo);
        split2<PK>(v2, v3, hi);
#pragma unroll
        for (int p = 0; p < Fmt<PK>::parts; ++p)
            *reinterpret_cast<uint2 *>(row + p * kBlk) = make_uint2(lo[p], hi[p]);
    }
}

// Accumulator tile (rows r0.., columns c0..) into the B x B block dst.
__device__ __forceinline__ void store_tile(double *dst, int B, int r0, int c0, int lane, const double (&dr)[16],
                                           const double (&di)[16], const float *sx, const float *sy)
{
    const int col = c0 + (lane & 31);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int row = r0 + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
        if (row < B && col < B) {
            const double f = sx ? 1.0 / ((double)sx[row] * (double)sy[col]) : 1.0;
            double2 v;
            v.x = dr[j] * f;
            v.y = di[j] * f;
            *reinterpret_cast<double2 *>(dst + 2 * ((size_t)row * B + col)) = v;
        }
    }
}

// Keeps the first nv of the four centres of a quad (nv in 0..4).  The hot
// loop loads from clamped, always valid addresses without branches, so that
// every load of a block is in flight at once, and masks at first use.
__device__ __forceinline__ float4 keep(float4 v, int nv)
{
    v.x = nv > 0 ? v.x : 0.f;
    v.y = nv > 1 ? v.y : 0.f;
    v.z = nv > 2 ? v.z : 0.f;
    v.w = nv > 3 ? v.w : 0.f;
    return v;
}

__device__ __forceinline__ float comp(const float4 &v, int e)
{
    return e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
}

__device__ __forceinline__ uint4 xor4(uint4 v, uint32_t m)
{
    return make_uint4(v.x ^ m, v.y ^ m, v.z ^ m, v.w ^ m);
}

// The contraction, software-pipelined over blocks of kBlk centres with two
// LDS buffers: while the matrix cores run the products of block b from one
// buffer, the same wavefronts form the operands of block b + 1 (VALU) into
// the other, and the global loads of block b + 2 are in flight; one barrier
// per block.
//  NK = false: four wavefronts = mu 0..3 of one order n.  The staging
//    threads of waves 0-1 form the X operands (-c G_{n-3}, -c* G_{n-1},
//    -c conj G_{-n-1}), those of waves 2-3 the Y operands (G_{-n-3},
//    G_{-n-1}, G_{n-1}), with the same branch-free arithmetic (factor 1 on
//    the Y side).
//  NK = true (FP32 only): N of two orders; wavefront 2k + r computes the
//    real (r = 0) or imaginary (r = 1) part of order 2 grp + k.
template <int PK, bool NK>
__global__ __launch_bounds__(256, 2) void k_contract(ContractArgs a)
{
    using F = Fmt<PK>;
    using T = typename F::T;
    constexpr int P = F::parts, RS = row_elems<PK>();
    constexpr int NC = NK ? 4 : 6;  // complex operand arrays per buffer
    constexpr int NL = NC / 2;      // complex planes per staging thread
    constexpr int BUF = 2 * NC * kRows * RS;
    __shared__ __attribute__((aligned(16))) T lds[2 * BUF];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // Workgroups are dispatched round-robin over the 8 XCDs: XCD x runs the
    // slices x, x + 8, ...; within a slice the catalog pairs vary fastest,
    // then the order group, so that the workgroups reading the same harmonic
    // planes (every pair shares its X catalog with n_z - 1 others and its Y
    // catalog likewise; neighbouring orders share planes) run on one XCD at
    // about the same time and meet in its L2.
    const int ngrp = NK ? (a.w_max + 2) / 2 : a.n_max + 1;
    const int pairs = a.n_z * a.n_z;
    const int xcd = blockIdx.x & 7;
    int jx = blockIdx.x >> 3;
    const int pair = jx % pairs;
    jx /= pairs;
    const int grp = jx % ngrp;
    const int sl = 8 * (jx / ngrp) + xcd;
    if (sl >= a.S) return;
    const int nt = a.nt;  // bin tiles per side
    const int tb1 = (int)blockIdx.y / nt, tb2 = (int)blockIdx.y % nt;
    const float *px, *py;
    pair_planes(a, pair, px, py);
    const int i_begin = sl * a.slice;
    const int i_end = min(i_begin + a.slice, a.n_c);
    const int nm = a.n_max;

    // this wavefront's product X_ia * (conj?) Y_ib
    int n, mu, ia, ib, ri = 0;
    bool cj;
    if constexpr (NK) {
        n = 2 * grp + (wave >> 1);
        mu = 4;
        ia = wave >> 1;
        ib = 2 + (wave >> 1);
        ri = wave & 1;
        cj = true;
    } else {
        n = grp;
        mu = wave;
        ia = mu == 3 ? 0 : mu;
        ib = (mu == 0 || mu == 2) ? 3 : (mu == 1 ? 4 : 5);
        cj = mu == 3;
    }
    const bool active = n <= (NK ? a.w_max : nm);

    // staging role: tile row sb (bin bg), centre quad sq, side sh (0: X from
    // px, bins of tile tb1; 1: Y from py, bins of tile tb2)
    const int sb = tid & 31, sq = (tid >> 5) & 3;
    const int sh = __builtin_amdgcn_readfirstlane(tid >> 7);
    const int bg = (sh ? tb2 : tb1) * kRows + sb;
    int pl[NL];
    if constexpr (NK) {
        pl[0] = plane_w(min(2 * grp, a.w_max), nm);
        pl[1] = plane_w(min(2 * grp + 1, a.w_max), nm);
    } else {
        pl[0] = plane_g(sh ? -grp - 3 : grp - 3, nm);
        pl[1] = plane_g(sh ? -grp - 1 : grp - 1, nm);
        pl[2] = plane_g(sh ? grp - 1 : -grp - 1, nm);
    }
    const float *src = sh ? py : px;
    const int bc = min(bg, a.B - 1);
    unsigned off[NL][2];  // float offset of (plane, centre 0, bin bc)
#pragma unroll
    for (int k = 0; k < NL; ++k)
#pragma unroll
        for (int r = 0; r < 2; ++r) off[k][r] = (unsigned)chunk_offset(pl[k] + r, 0, bc, a.K, a.B);
    const int i_last = i_end - 1;
    const int q_last = i_last >> 2;
    const unsigned qstride = 4u * (unsigned)a.B;  // floats from one centre quad to the next
    // branch-free operand factors: X side (-c), Y side 1
    const float ys = sh ? 1.0f : 0.0f, xs = sh ? 0.0f : 1.0f;
    const float s2 = sh ? 1.0f : -1.0f;  // conj of G_{-n-1} on the X side
    float sc[3] = {1.f, 1.f, 1.f};        // fp16 row scales of this thread's arrays
    const float *scl = nullptr;
    if constexpr (PK == T3_PREC_FP16X3) {
        scl = a.scale + ((size_t)pair * (nm + 1) + n) * kNYArr * kScaleRows;
        const float *srow = a.scale + ((size_t)pair * (nm + 1) + grp) * kNYArr * kScaleRows;
#pragma unroll
        for (int k = 0; k < 3; ++k) sc[k] = srow[(3 * sh + k) * kScaleRows + bg];
    }

    struct Stage {
        float4 ld[NL][2];
        float2 cw[4];  // (Re c, Im c) of the quad's centres, or (w, 0) for N
        int nv;        // valid centres of this thread's quad
    };
    Stage s0, s1;
    // Every thread loads the centre factors (the Y side ignores them) and
    // loads them first: with the same loads on every path, in the same
    // order, the compiler waits only for the stage being used.
    auto load_block = [&](Stage &st, int i0) {
        const int q = (i0 >> 2) + sq;
        const unsigned qo = (unsigned)min(q, q_last) * qstride;
        st.nv = bg < a.B ? max(0, min(4, i_end - 4 * q)) : 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float4 f = a.ccw[min(4 * q + e, i_last)];
            st.cw[e] = NK ? make_float2(f.z, 0.f) : make_float2(f.x, f.y);
        }
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            st.ld[k][0] = *reinterpret_cast<const float4 *>(src + off[k][0] + qo);
            st.ld[k][1] = *reinterpret_cast<const float4 *>(src + off[k][1] + qo);
        }
    };

    auto lrow = [&](int buf, int arr, int part, int row) -> T * {
        return lds + (size_t)buf * BUF + (size_t)(2 * arr + part) * kRows * RS + (size_t)row * RS;
    };

    // operands of one staged block into LDS buffer buf
    auto stage_to_lds = [&](Stage &st, int buf) {
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            st.ld[k][0] = keep(st.ld[k][0], st.nv);
            st.ld[k][1] = keep(st.ld[k][1], st.nv);
        }
        float v[4][NL][2];  // [centre][array][re/im]
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if constexpr (NK) {
                const float w = fmaf(xs, st.cw[e].x, ys);  // w on the X side, 1 on the Y side
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    v[e][k][0] = w * comp(st.ld[k][0], e);
                    v[e][k][1] = w * comp(st.ld[k][1], e);
                }
            } else {
                const float ar = fmaf(-xs, st.cw[e].x, ys), ai = -xs * st.cw[e].y;
                const float g0r = comp(st.ld[0][0], e), g0i = comp(st.ld[0][1], e);
                const float g1r = comp(st.ld[1][0], e), g1i = comp(st.ld[1][1], e);
                const float g2r = comp(st.ld[2][0], e), g2i = s2 * comp(st.ld[2][1], e);
                v[e][0][0] = fmaf(ar, g0r, -ai * g0i) * sc[0];
                v[e][0][1] = fmaf(ar, g0i, ai * g0r) * sc[0];
                v[e][1][0] = fmaf(ar, g1r, ai * g1i) * sc[1];
                v[e][1][1] = fmaf(ar, g1i, -ai * g1r) * sc[1];
                v[e][2][0] = fmaf(ar, g2r, -ai * g2i) * sc[2];
                v[e][2][1] = fmaf(ar, g2i, ai * g2r) * sc[2];
            }
        }
#pragma unroll
        for (int k = 0; k < NL; ++k)
#pragma unroll
            for (int r = 0; r < 2; ++r)
                put4<PK>(lrow(buf, NL * sh + k, r, sb) + 4 * sq, v[0][k][r], v[1][k][r], v[2][k][r], v[3][k][r]);
    };

    floatx16 cr = {}, ci = {};
    double dr[16], di[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) dr[j] = di[j] = 0.0;
    int run = 0;
    auto promote = [&]() {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            dr[j] += (double)cr[j];
            di[j] += (double)ci[j];
            cr[j] = 0.f;
            ci[j] = 0.f;
        }
    };

    // this wavefront's MFMAs over the block in LDS buffer buf.  The FP64
    // promotion of a finished run comes first, so that it reads accumulators
    // whose MFMAs completed while the staging arithmetic ran.
    auto mfma_block = [&](int buf) {
        if (!active) return;
        if (run >= kRun) {
            promote();
            run = 0;
        }
        run += kBlk;
        const int r = lane & 31, kq = lane >> 5;
        if constexpr (PK == T3_PREC_FP32) {
            float4 xr[2], xi[2], yr[2], yi[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                xr[h] = *reinterpret_cast<const float4 *>(lrow(buf, ia, 0, r) + 8 * kq + 4 * h);
                xi[h] = *reinterpret_cast<const float4 *>(lrow(buf, ia, 1, r) + 8 * kq + 4 * h);
                yr[h] = *reinterpret_cast<const float4 *>(lrow(buf, ib, 0, r) + 8 * kq + 4 * h);
                yi[h] = *reinterpret_cast<const float4 *>(lrow(buf, ib, 1, r) + 8 * kq + 4 * h);
            }
            if constexpr (NK) {
                // conj Y: Re = Xr Yr + Xi Yi, Im = -Xr Yi + Xi Yr (one part per wavefront)
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    const float ar = comp(xr[s >> 2], s & 3), ai = comp(xi[s >> 2], s & 3);
                    const float br = comp(yr[s >> 2], s & 3), bi = comp(yi[s >> 2], s & 3);
                    cr = __builtin_amdgcn_mfma_f32_32x32x2f32(ri ? -ar : ar, ri ? bi : br, cr, 0, 0, 0);
                    cr = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, ri ? br : bi, cr, 0, 0, 0);
                }
            } else {
                const uint32_t m1 = cj ? 0u : 0x80000000u;  // Re: X_i * (-Y_i) (or + for conj Y)
                const uint32_t m2 = cj ? 0x80000000u : 0u;  // Im: X_r * Y_i (or - for conj Y)
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    const float ar = comp(xr[s >> 2], s & 3), ai = comp(xi[s >> 2], s & 3);
                    const float br = comp(yr[s >> 2], s & 3), bi = comp(yi[s >> 2], s & 3);
                    const float x1 = __uint_as_float(__float_as_uint(ai) ^ m1);
                    const float x2 = __uint_as_float(__float_as_uint(ar) ^ m2);
                    cr = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, cr, 0, 0, 0);
                    cr = __builtin_amdgcn_mfma_f32_32x32x2f32(x1, bi, cr, 0, 0, 0);
                    ci = __builtin_amdgcn_mfma_f32_32x32x2f32(x2, bi, ci, 0, 0, 0);
                    ci = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, br, ci, 0, 0, 0);
                }
            }
        } else {
            using V = typename F::V;
            const uint32_t m1 = cj ? 0u : 0x80008000u;
            const uint32_t m2 = cj ? 0x80008000u : 0u;
            // one X part at a time (its four vectors), Y parts re-read from
            // LDS for every X part: fewer live registers
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const uint4 xr = *reinterpret_cast<const uint4 *>(lrow(buf, ia, 0, r) + p * kBlk + 8 * kq);
                const uint4 xi = *reinterpret_cast<const uint4 *>(lrow(buf, ia, 1, r) + p * kBlk + 8 * kq);
                const V XR = __builtin_bit_cast(V, xr);
                const V XI = __builtin_bit_cast(V, xi);
                const V X1 = __builtin_bit_cast(V, xor4(xi, m1));
                const V X2 = __builtin_bit_cast(V, xor4(xr, m2));
#pragma unroll
                for (int q = 0; q + p < P; ++q) {
                    const V YR = *reinterpret_cast<const V *>(lrow(buf, ib, 0, r) + q * kBlk + 8 * kq);
                    const V YI = *reinterpret_cast<const V *>(lrow(buf, ib, 1, r) + q * kBlk + 8 * kq);
                    if constexpr (PK == T3_PREC_FP16X3) {
                        cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(XR, YR, cr, 0, 0, 0);
                        cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(X1, YI, cr, 0, 0, 0);
                        ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(X2, YI, ci, 0, 0, 0);
                        ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(XI, YR, ci, 0, 0, 0);
                    } else {
                        cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XR, YR, cr, 0, 0, 0);
                        cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(X1, YI, cr, 0, 0, 0);
                        ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(X2, YI, ci, 0, 0, 0);
                        ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(XI, YR, ci, 0, 0, 0);
                    }
                }
            }
        }
    };

    // Pipeline.  i_begin < i_end here (empty slices are never launched);
    // loads past the end read clamped, valid addresses and are masked (nv = 0).
    load_block(s0, i_begin);
    load_block(s1, i_begin + kBlk);
    stage_to_lds(s0, 0);
    load_block(s0, i_begin + 2 * kBlk);
    __syncthreads();
    for (int i0 = i_begin;; i0 += 2 * kBlk) {
        mfma_block(0);  // block i0
        if (i0 + kBlk >= i_end) break;
        stage_to_lds(s1, 1);  // block i0 + kBlk
        load_block(s1, i0 + 3 * kBlk);
        __syncthreads();
        mfma_block(1);
        if (i0 + 2 * kBlk >= i_end) break;
        stage_to_lds(s0, 0);  // block i0 + 2 kBlk
        load_block(s0, i0 + 4 * kBlk);
        __syncthreads();
    }
    if (!active) return;
    promote();
    const int nq = 4 * (nm + 1) + a.w_max + 1;               // B x B blocks per slice
    const int q = mu < 4 ? mu * (nm + 1) + n : 4 * (nm + 1) + n;  // this block
    double *dst = a.partial + (((size_t)pair * a.S + sl) * nq + q) * a.B * a.B * 2;
    if constexpr (NK) {
        // one part per wavefront: real parts in dr of wave r = 0, imaginary in r = 1
        const int col = kRows * tb2 + (lane & 31);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int row = kRows * tb1 + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
            if (row < a.B && col < a.B) dst[2 * ((size_t)row * a.B + col) + ri] = dr[j];
        }
    } else if constexpr (PK == T3_PREC_FP16X3) {
        store_tile(dst, a.B, kRows * tb1, kRows * tb2, lane, dr, di, scl + ia * kScaleRows, scl + ib * kScaleRows);
    } else {
        store_tile(dst, a.B, kRows * tb1, kRows * tb2, lane, dr, di, nullptr, nullptr);
    }
}

// ------------------------------------------------------------ B <= 24
// A block of at most 24 bins fills a 32 x 32 complex tile to at most 56%
// (39% at B = 20).  For such blocks the complex product is embedded in one
// real product of 2B x 2B: operand row 2b + p holds part p (0 real,
// 1 imaginary) of bin b, so that the real product of X (2B x K) with
// Y^T (K x 2B) holds every X_p Y_q, and at each promotion of an FP32 run
//     Re X Y  = Xr Yr - Xi Yi,   Im X Y  = Xr Yi + Xi Yr,
//     Re X Y* = Xr Yr + Xi Yi,   Im X Y* = Xi Yr - Xr Yi.
// The 2B rows take T = ceil(2B / 16) tiles of 16 x 16 per side, T^2 tiles
// per wavefront (69% of the issued products useful at B = 20, 100% at
// B = 16).  With the parts interleaved, the four real products of one
// (b1, b2) sit in two neighbouring lanes: one DPP-fused FMA per lane forms
// its real (even lane) or imaginary (odd lane) part.
//
// A workgroup of eight wavefronts splits the work by role: wavefronts 0-3
// only multiply, wavefronts 4-7 only load and form operands.  Each step of
// STEP centres is formed into one of two LDS buffers while the multiplying
// wavefronts read the other (one barrier per step), so every SIMD holds a
// multiplying and a staging wavefront of each of two workgroups: the FP32
// MFMAs do not co-issue with vector instructions on this hardware, and the
// staging arithmetic then fills the issue slots the matrix core leaves.
//  NK = false: the four products are mu 0..3 of one order n (operand arrays
//    X0..X2 from the Z2 planes, Y3..Y5 from the Z3 planes, as in k_contract).
//  NK = true (FP32): N_n of one order n (X = w W_n, Y = W_n); the four
//    multiplying wavefronts take the four blocks of each step of 4 kBlk
//    centres and add their FP64 sums in a fixed order at the end (the grid
//    then matches the Upsilon kernel's).
// Staging: item (array, centre quad, bin) is one thread's pair of float4
// loads (real and imaginary planes: four centres of one bin, coalesced over
// the bins); a thread keeps the same items for the whole slice.  The centre
// factors of a step reach LDS one step before its operands are formed, in
// the three sign forms the X operands take.
// Products:
//  * FP32: v_mfma_f32_16x16x4_f32; lane group g (lane / 16) takes centre
//    4 g + s of the block in step s.
//  * splits: v_mfma_f32_16x16x32_{bf16,f16}, whose 32-deep K holds the 16
//    centres of a block twice, for two part products at once: lane groups
//    0-1 carry the centres in part p, groups 2-3 in part p'.  Two-part
//    splits (BF16X3, FP16X3): [X0|X1].[Y0|Y0] + [X0|X1].[Y1|Y1], all four
//    part products: lo*lo shares its MFMA with hi*lo, so it costs nothing
//    here (the 32 x 32 kernel drops it).  BF16X6 (the six products with part
//    orders summing to at most 2): [X0|X1].[Y0|Y0] + [X0|X1].[Y1|Y1] +
//    [X0|X2].[Y2|Y0].  FP16X3 rows carry the power-of-two scales of
//    k_fp16_scale, divided out in FP64.
constexpr int kSmallBins = 24;

template <int PK>
constexpr int small_row_elems()  // LDS elements per operand row: the parts of kBlk centres + 16 bytes
{
    return PK == T3_PREC_FP32 ? kBlk + 4 : Fmt<PK>::parts * kBlk + 8;
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

// SAME (N_n of one catalog: Z2 = Z3): the X operand w W_n and the Y operand
// W_n come from the same loads.
// Waves per SIMD: 4 (two workgroups per CU, at most 128 registers) where the
// registers fit without spilling, else 2.
template <int PK, int T, bool NK, int NIS, bool SAME>
__global__ __launch_bounds__(512, ((NK && !SAME) || (!NK && NIS > 1)) ? 2 : 4) void k_contract_small(ContractArgs a)
{
    using E = typename Fmt<PK>::T;            // LDS element
    constexpr int P = Fmt<PK>::parts;
    constexpr int RS = small_row_elems<PK>();
    constexpr int R = 16 * T;                  // real rows per operand array
    constexpr int NA = NK ? 8 : 6;             // complex operand arrays
    constexpr int NH = NA / 2;                 // per side
    constexpr int ARR = R * RS;                // elements per array
    constexpr int BUF = NA * ARR;              // elements per buffer
    constexpr int NB = NK ? 4 : 1;             // blocks of kBlk centres per step
    constexpr int STEP = NB * kBlk;            // centres per step
    constexpr int NV = NK ? 1 : 3;             // factor forms per centre
    static_assert(!NK || PK == T3_PREC_FP32, "N_n is computed in FP32");
    static_assert(NK || !SAME, "shared loads serve N_n only");
    constexpr int NLS = SAME ? 1 : 2;           // sides that load
    // N_n of one catalog is Hermitian in (b1, b2): only the tiles on and
    // above the diagonal are multiplied, the ones below are their conjugate
    // transposes
    constexpr bool HERM = NK && SAME;
    auto tile_on = [](int r, int c) { return !HERM || c >= r; };
    static_assert(!NK || 3 * T * T * 2 * 64 * sizeof(double) <= 2 * BUF * sizeof(E), "N_n sums fit the LDS");
    // two operand buffers, then a dummy row pair that the stores of unused
    // staging slots go to (the staging has no branches: see below)
    __shared__ __attribute__((aligned(16))) E lds[2 * BUF + 2 * RS];
    __shared__ float4 cwl[2][NV][STEP + 16];  // factor forms of a step's centres + dummy slots

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool producer = wave >= 4;
    // slice / order / pair mapping as in k_contract (XCD-major)
    const int ngrp = (NK ? a.w_max : a.n_max) + 1;  // orders
    const int pairs = a.n_z * a.n_z;
    const int xcd = blockIdx.x & 7;
    int jx = blockIdx.x >> 3;
    const int pair = jx % pairs;
    jx /= pairs;
    const int n = jx % ngrp;
    const int sl = 8 * (jx / ngrp) + xcd;
    if (sl >= a.S) return;
    const float *px, *py;
    pair_planes(a, pair, px, py);
    const int i_begin = sl * a.slice;
    const int i_end = min(i_begin + a.slice, a.n_c);
    const int i_last = i_end - 1, q_last = i_last >> 2;
    const int nsteps = (i_end - i_begin + STEP - 1) / STEP;
    const int nm = a.n_max, B = a.B;
    const float *scl = nullptr;  // fp16 row scales of order n: [array][kScaleRows]
    if constexpr (PK == T3_PREC_FP16X3) scl = a.scale + ((size_t)pair * (nm + 1) + n) * kNYArr * kScaleRows;

    // padding rows 2B..R-1 of every array stay zero
    {
        const int per = (R - 2 * B) * RS;
        for (int e = tid; e < 2 * NA * per; e += 512) lds[(e / per) * ARR + 2 * B * RS + e % per] = E(0.0f);
    }

    if (producer) {
        // ---------------------------------------------------------- staging
        // Item (array k, centre quad q, bin b) of a side: k = it / 4B,
        // q = (it mod 4B) / B, b = it mod B; producer thread p takes items
        // p + 256 u of each side.  Items past the last load the last one
        // again and store into the dummy row pair, so that the staging has
        // no branches and the loads of a step are waited for once, when its
        // operands are formed, while the next step's loads stay in flight.
        const int ptid = tid - 256;
        const int nis = NH * 4 * B;  // items per side (NIS = ceil(nis / 256) per thread, set at launch)
        const unsigned KB = (unsigned)a.K * (unsigned)B;  // floats per plane
        const unsigned qstride = 4u * (unsigned)B;        // floats from one centre quad to the next
        unsigned g0[2][NIS];  // float offset of (real plane, quad 0 of the chunk, bin)
        int qq[2][NIS];       // centre quad of the item within a step
        int lo[2][NIS];       // LDS element offset of (array, row 2 bin, centre 4 quad); >= 2 BUF: dummy
        int kx[NIS];          // X side: the factor form of the item's array
        float sc[2][NIS];     // fp16 row scales (1 otherwise)
#pragma unroll
        for (int side = 0; side < 2; ++side)
#pragma unroll
            for (int u = 0; u < NIS; ++u) {
                const int it0 = ptid + 256 * u, it = min(it0, nis - 1);
                const int k = it / (4 * B), qb = it % (4 * B);
                const int q = qb / B, b = qb % B;
                int pl, wb = 0;
                if constexpr (NK) {
                    pl = plane_w(n, nm);
                    wb = k;  // the block of the step whose operands array k holds
                } else {
                    const int m = side == 0 ? (k == 0 ? n - 3 : k == 1 ? n - 1 : -n - 1)
                                            : (k == 0 ? -n - 3 : k == 1 ? -n - 1 : n - 1);
                    pl = plane_g(m, nm);
                }
                qq[side][u] = 4 * wb + q;
                g0[side][u] = (unsigned)chunk_offset(pl, 0, b, a.K, B);
                lo[side][u] = it0 < nis ? (side * NH + k) * ARR + 2 * b * RS + 4 * q : 2 * BUF + 4 * (ptid & 3);
                sc[side][u] = 1.0f;
                if constexpr (PK == T3_PREC_FP16X3) sc[side][u] = scl[(side * NH + k) * kScaleRows + b];
                if (side == 0) kx[u] = NK ? 0 : k;
            }

        struct Stage {
            float4 re[NLS][NIS], im[NLS][NIS];
            float4 cw;  // centre factors of centre ptid mod STEP of the step
        };
        auto load_step = [&](Stage &st, int step) {
            const int i0 = i_begin + step * STEP;
            st.cw = a.ccw[min(i0 + (ptid & (STEP - 1)), i_last)];
            // quads past the slice's last read its last quad (masked when formed)
            const int qrel = q_last - (i0 >> 2);                  // last valid quad relative to the step
            const unsigned sbase = (unsigned)(i0 >> 2) * qstride;  // the step's first quad
            const unsigned slast = (unsigned)q_last * qstride;
#pragma unroll
            for (int side = 0; side < NLS; ++side) {
                const float *sp = side ? py : px;
#pragma unroll
                for (int u = 0; u < NIS; ++u) {
                    const unsigned o =
                        g0[side][u] + (qq[side][u] <= qrel ? sbase + (unsigned)qq[side][u] * qstride : slast);
                    st.re[side][u] = *reinterpret_cast<const float4 *>(sp + o);
                    st.im[side][u] = *reinterpret_cast<const float4 *>(sp + o + KB);
                }
            }
        };
        // The factor forms (p, q, r, t) of a centre, Re = p gr + q gi and
        // Im = r gi + t gr for the X operand of g = gr + i gi:
        //     -c g: (-cr, ci, -cr, -ci),   -c* g: (-cr, -ci, -cr, ci),
        //     -c conj g: (-cr, -ci, cr, -ci);   N_n: w g as (w, 0, w, 0).
        // Written by the first producer wavefront (lanes past STEP write
        // dummy slots).
        auto put_cw = [&](int buf, float4 cw) {
            if (wave != 4) return;
            const int j = ptid < STEP ? ptid : STEP + (ptid & 15);
            if constexpr (NK) {
                cwl[buf][0][j] = make_float4(cw.z, 0.f, cw.z, 0.f);
            } else {
                const float cr = cw.x, ci = cw.y;
                cwl[buf][0][j] = make_float4(-cr, ci, -cr, -ci);
                cwl[buf][1][j] = make_float4(-cr, -ci, -cr, ci);
                cwl[buf][2][j] = make_float4(-cr, -ci, cr, -ci);
            }
        };
        // one real row of four centres: FP32 as is, splits part p at p kBlk
        auto put_row = [&](E *row, float4 v) {
            if constexpr (PK == T3_PREC_FP32) {
                *reinterpret_cast<float4 *>(row) = v;
            } else {
                uint32_t l[P], h[P];
                split2<PK>(v.x, v.y, l);
                split2<PK>(v.z, v.w, h);
#pragma unroll
                for (int p = 0; p < P; ++p) *reinterpret_cast<uint2 *>(row + p * kBlk) = make_uint2(l[p], h[p]);
            }
        };
        // operands of one step into LDS buffer buf; MASK: the slice's last,
        // partial step, whose centres past the end are zero
        auto stage_mask = [&](Stage &st, int buf, int step, auto mask) {
            const int i0 = i_begin + step * STEP;
            const int boff = buf * BUF;
#pragma unroll
            for (int side = 0; side < 2; ++side)
#pragma unroll
                for (int u = 0; u < NIS; ++u) {
                    const int q = qq[side][u];
                    float4 vr = st.re[SAME ? 0 : side][u], vi = st.im[SAME ? 0 : side][u];
                    if constexpr (decltype(mask)::value) {
                        const int nv = max(0, min(4, i_end - (i0 + 4 * q)));
                        vr = keep(vr, nv);
                        vi = keep(vi, nv);
                    }
                    if (side == 0) {
                        float r[4], m[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const float4 f = cwl[buf][kx[u]][4 * q + e];
                            const float gr = comp(vr, e), gi = comp(vi, e);
                            if constexpr (NK) {  // w W_n
                                r[e] = f.x * gr;
                                m[e] = f.x * gi;
                            } else {
                                r[e] = fmaf(f.x, gr, f.y * gi);
                                m[e] = fmaf(f.z, gi, f.w * gr);
                            }
                        }
                        vr = make_float4(r[0], r[1], r[2], r[3]);
                        vi = make_float4(m[0], m[1], m[2], m[3]);
                    }
                    if constexpr (PK == T3_PREC_FP16X3) {
                        const float s = sc[side][u];
                        vr = make_float4(vr.x * s, vr.y * s, vr.z * s, vr.w * s);
                        vi = make_float4(vi.x * s, vi.y * s, vi.z * s, vi.w * s);
                    }
                    const int o = lo[side][u] + (lo[side][u] < 2 * BUF ? boff : 0);
                    put_row(lds + o, vr);
                    put_row(lds + o + RS, vi);
                }
        };
        auto stage = [&](Stage &st, int buf, int step) {  // one wave-uniform branch
            if (i_begin + (step + 1) * STEP <= i_end)
                stage_mask(st, buf, step, std::false_type{});
            else
                stage_mask(st, buf, step, std::true_type{});
        };

        // Step k goes to buffer k mod 2 before barrier k, its factor forms
        // to cwl[k mod 2] before barrier k - 1; step k + 1 is formed while
        // the multiplying wavefronts read step k.  The loads run NS steps
        // ahead (NS register stages).
        constexpr int NS = 2;
        Stage st[NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) load_step(st[j], j);
        put_cw(0, st[0].cw);
        __syncthreads();  // factor forms of step 0
        stage(st[0], 0, 0);
        load_step(st[0], NS);
        put_cw(1, st[1].cw);
        for (int k = 0;; k += NS) {
            bool done = false;
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                if (!done) {
                    __syncthreads();  // barrier k + j
                    if (k + j + 1 >= nsteps) {
                        done = true;
                    } else {
                        stage(st[(j + 1) % NS], (k + j + 1) & 1, k + j + 1);
                        load_step(st[(j + 1) % NS], k + j + 1 + NS);
                        put_cw((k + j) & 1, st[(j + 2) % NS].cw);  // step k + j + 2
                    }
                }
            }
            if (done) break;
        }
        if constexpr (NK) {  // the consumers' two barriers of the N_n reduction
            __syncthreads();
            __syncthreads();
        }
        return;
    }

    // ------------------------------------------------------------ products
    // this wavefront's product X_ia (conj?) Y_ib; arrays 0 .. NH - 1 are the
    // X side (Z2 planes), NH .. NA - 1 the Y side (Z3 planes)
    int ia, ib;
    bool cj;
    if constexpr (NK) {
        ia = wave;       // w W_n of block `wave` of the step
        ib = NH + wave;  // W_n of the same block
        cj = true;
    } else {
        ia = wave == 3 ? 0 : wave;
        ib = NH + ((wave == 0 || wave == 2) ? 0 : (wave == 1 ? 1 : 2));
        cj = wave == 3;
    }
    // D row 16 r + 4 (lane / 16) + j = 2 b1 + (j & 1), column 16 c + lane mod 16
    // = 2 b2 + (lane & 1): lane pair (even, odd) holds the real and the
    // imaginary column of bins b1 = 8 r + 2 (lane / 16) (j = 0, 1) and b1 + 1
    // (j = 2, 3).  Per bin, with u = D[2 b1][.] and v = D[2 b1 + 1][.] of the
    // lane and v' the partner's v (one DPP swap):
    //     X Y:  even  u - v' = Xr Yr - Xi Yi,     odd  u + v' = Xr Yi + Xi Yr;
    //     X Y*: even  u + v' = Xr Yr + Xi Yi,     odd -(u - v') = Xi Yr - Xr Yi:
    // the even lane forms the real part, the odd lane the imaginary part.
    const int g = lane >> 4, odd = lane & 1;
    // t = u + s1 v' in FP32 (one DPP-fused FMA), then += s2 t in FP64:
    // X Y: s1 = -1 / +1 (even / odd), s2 = 1; X Y*: s1 = +1 / -1, s2 = s1
    const float s1 = (odd ? 1.0f : -1.0f) * (cj ? -1.0f : 1.0f);
    const double s2 = cj ? (double)s1 : 1.0;
    floatx4 acc[T][T];
    double dacc[T][T][2];  // FP64 sums of bins b1 and b1 + 1, this lane's part
#pragma unroll
    for (int r = 0; r < T; ++r)
#pragma unroll
        for (int c = 0; c < T; ++c) {
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[r][c][j] = 0.f;
            dacc[r][c][0] = dacc[r][c][1] = 0.0;
        }
    // FP32 runs of one block (kRun = kBlk centres, the error model of the
    // 32 x 32 kernel): at the end of a run the four real products of (b1, b2)
    // are combined into the complex product in FP32 and promoted into FP64.
    // The promotion of a run comes first in the next step, reading
    // accumulators whose products have completed; the step's first products
    // then start from zero.
    auto swap1 = [](float v) {  // lane ^ 1 (DPP quad_perm 1, 0, 3, 2)
        return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xb1, 0xf, 0xf, true));
    };
    auto promote = [&]() {
#pragma unroll
        for (int r = 0; r < T; ++r)
#pragma unroll
            for (int c = 0; c < T; ++c) {
                if (!tile_on(r, c)) continue;
                const floatx4 d = acc[r][c];
                const float t0 = fmaf(swap1(d[1]), s1, d[0]);
                const float t1 = fmaf(swap1(d[3]), s1, d[2]);
                dacc[r][c][0] = fma((double)t0, s2, dacc[r][c][0]);
                dacc[r][c][1] = fma((double)t1, s2, dacc[r][c][1]);
            }
    };
    const floatx4 zero4 = {0.f, 0.f, 0.f, 0.f};
    auto mfma_block = [&](int buf) {
        promote();
        const E *base = lds + buf * BUF + (lane & 15) * RS;
        if constexpr (PK == T3_PREC_FP32) {
            // column tile by column tile (one Y fragment live), the T row
            // tiles' chains interleaved
            float4 xa[T];
#pragma unroll
            for (int t = 0; t < T; ++t) xa[t] = *reinterpret_cast<const float4 *>(base + ia * ARR + 16 * t * RS + 4 * g);
#pragma unroll
            for (int c = 0; c < T; ++c) {
                const float4 yb = *reinterpret_cast<const float4 *>(base + ib * ARR + 16 * c * RS + 4 * g);
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int r = 0; r < T; ++r) {
                        if (!tile_on(r, c)) continue;
                        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(comp(xa[r], s), comp(yb, s),
                                                                         s == 0 ? zero4 : acc[r][c], 0, 0, 0);
                    }
            }
        } else {
            using V = typename Fmt<PK>::V;
            auto mma = [&](const uint4 &x, const uint4 &y, floatx4 &c) {
                if constexpr (PK == T3_PREC_FP16X3)
                    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(V, x), __builtin_bit_cast(V, y), c,
                                                               0, 0, 0);
                else
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(V, x), __builtin_bit_cast(V, y), c,
                                                                0, 0, 0);
            };
            // fragment offsets within a row (elements): [X0|X1] 8 g, [Y0|Y0] 8 (g & 1),
            // [Y1|Y1] 16 + 8 (g & 1), [X0|X2] 8 g + 16 (g >= 2), [Y2|Y0] 32 + 8 g (g < 2) or 8 (g - 2);
            // column tile by column tile (the Y fragments of one column live)
            const int o01 = 8 * g, o00 = 8 * (g & 1), o11 = 16 + 8 * (g & 1);
            const int o02 = 8 * g + (g >= 2 ? 16 : 0), o20 = g < 2 ? 32 + 8 * g : 8 * (g - 2);
            uint4 x01[T], x02[P == 3 ? T : 1];
#pragma unroll
            for (int t = 0; t < T; ++t) {
                x01[t] = *reinterpret_cast<const uint4 *>(base + ia * ARR + 16 * t * RS + o01);
                if constexpr (P == 3) x02[t] = *reinterpret_cast<const uint4 *>(base + ia * ARR + 16 * t * RS + o02);
            }
#pragma unroll
            for (int c = 0; c < T; ++c) {
                const E *yc = base + ib * ARR + 16 * c * RS;
                const uint4 y00 = *reinterpret_cast<const uint4 *>(yc + o00);
                const uint4 y11 = *reinterpret_cast<const uint4 *>(yc + o11);
#pragma unroll
                for (int r = 0; r < T; ++r) {
                    acc[r][c] = zero4;
                    mma(x01[r], y00, acc[r][c]);
                }
#pragma unroll
                for (int r = 0; r < T; ++r) mma(x01[r], y11, acc[r][c]);
                if constexpr (P == 3) {
                    const uint4 y20 = *reinterpret_cast<const uint4 *>(yc + o20);
#pragma unroll
                    for (int r = 0; r < T; ++r) mma(x02[r], y20, acc[r][c]);
                }
            }
        }
    };

    __syncthreads();  // factor forms of step 0
    for (int k = 0; k < nsteps; ++k) {
        __syncthreads();  // barrier k: step k in buffer k mod 2
        mfma_block(k & 1);
    }
    promote();
    if constexpr (NK) {
        // the four blocks' sums, added in wavefront order
        constexpr int ND = T * T * 2;
        __syncthreads();  // every wavefront is done with the operands
        double *red = reinterpret_cast<double *>(lds);
        if (wave > 0) {
#pragma unroll
            for (int r = 0; r < T; ++r)
#pragma unroll
                for (int c = 0; c < T; ++c)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        if (tile_on(r, c)) red[((wave - 1) * ND + 2 * (r * T + c) + h) * 64 + lane] = dacc[r][c][h];
        }
        __syncthreads();
        if (wave > 0) return;
#pragma unroll
        for (int w = 0; w < 3; ++w)
#pragma unroll
            for (int r = 0; r < T; ++r)
#pragma unroll
                for (int c = 0; c < T; ++c)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        if (tile_on(r, c)) dacc[r][c][h] += red[(w * ND + 2 * (r * T + c) + h) * 64 + lane];
    }
    const int nq = 4 * (nm + 1) + a.w_max + 1;
    const int qb = NK ? 4 * (nm + 1) + n : wave * (nm + 1) + n;
    double *dst = a.partial + (((size_t)pair * a.S + sl) * nq + qb) * B * B * 2;
#pragma unroll
    for (int r = 0; r < T; ++r)
#pragma unroll
        for (int c = 0; c < T; ++c)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (!tile_on(r, c)) continue;
                const int b1 = 8 * r + 2 * g + h, b2 = 8 * c + ((lane & 15) >> 1);
                if (b1 < B && b2 < B) {
                    double f = 1.0;
                    if constexpr (PK == T3_PREC_FP16X3)
                        f = 1.0 / ((double)scl[ia * kScaleRows + b1] * (double)scl[ib * kScaleRows + b2]);
                    const double v = dacc[r][c][h] * f;
                    dst[2 * ((size_t)b1 * B + b2) + odd] = v;  // even lane Re, odd lane Im
                    if (HERM && c > r) dst[2 * ((size_t)b2 * B + b1) + odd] = odd ? -v : v;
                }
            }
}

// Edge bins for B = 33..40: every output (b1, b2) of the B x B blocks with
// b1 >= T or b2 >= T (T = 32, the extent of the one MFMA tile), for the
// slice's centres, written into the slice's partial block like the tiles.
// One workgroup per (slice, catalog pair) x order n: the four Upsilon_mu
// and N_n of order n <= n_max (NK = false), or N_n alone for the orders
// n_max < n <= w_max of the edge correction (NK = true).  Per block of
// kEdgeBlk centres the workgroup forms the operands of every bin in FP32
// with the arithmetic of the MFMA kernel (X = -c G_{n-3}, -c* G_{n-1},
// -c conj G_{-n-1}; Y = G_{-n-3}, G_{-n-1}, G_{n-1}; N: X = w W_n, Y = W_n),
// stores them in LDS, and each thread sums the products of its outputs in
// FP32 over the block and adds that run into FP64 accumulators (the error
// model of the FP32 MFMA runs).  There are E = B^2 - T^2 <= 576 outputs per (mu, n), at most
// kEdgeAcc per thread.
// Staging thread (e, item): centre e = tid mod 16 of the block and the
// (array, bin) items tid / 16 + 16 u; the loads of block b + 1 are issued
// before the products of block b.
constexpr int kEdgeMaxBins = 40;
constexpr int kEdgeT = 32;
constexpr int kEdgeBlk = 16;
constexpr int kEdgeRow = kEdgeBlk + 1;  // LDS row (array, bin) of kEdgeBlk centres, padded
constexpr int kEdgeAcc = (5 * (kEdgeMaxBins * kEdgeMaxBins - kEdgeT * kEdgeT) + 255) / 256;

// output e of one (mu, n) block -> (b1, b2): first the rows T..B-1 (every
// column), then the columns T..B-1 of the rows 0..T-1
__device__ __forceinline__ void edge_output(int e, int B, int &b1, int &b2)
{
    const int r = B - kEdgeT;
    if (e < r * B) {
        b1 = kEdgeT + e / B;
        b2 = e % B;
    } else {
        e -= r * B;
        b1 = e / r;
        b2 = kEdgeT + e % r;
    }
}

template <bool NK>
__global__ __launch_bounds__(256, 2) void k_contract_edge(ContractArgs a)
{
    // complex operand arrays: Upsilon X0..X2 (px), Y0..Y2 (py), then N's X (px)
    // and Y (py); NK: N's X and Y only
    constexpr int NA = NK ? 2 : 8;
    constexpr int NI = (NA * kEdgeMaxBins + 15) / 16;  // staging items per thread
    __shared__ float2 op[NA * kEdgeMaxBins * kEdgeRow];
    const int pairs = a.n_z * a.n_z;
    const int pair = (int)blockIdx.x % pairs, sl = (int)blockIdx.x / pairs;
    const int n = NK ? a.n_max + 1 + (int)blockIdx.y : (int)blockIdx.y;
    const int B = a.B, nm = a.n_max, tid = threadIdx.x;
    const float *px, *py;
    pair_planes(a, pair, px, py);
    const int i_begin = sl * a.slice;
    const int i_end = min(i_begin + a.slice, a.n_c);
    const int E = B * B - kEdgeT * kEdgeT;
    const int nout = (NK ? 1 : 5) * E;
    const unsigned KB = (unsigned)a.K * (unsigned)B;  // floats per plane

    // staging items: (array k, bin b) = kb / B, kb % B with kb = tid / 16 + 16 u
    const int e = tid & 15;
    unsigned off[NI];  // float offset of (plane, centre 0, bin) in its catalog's planes
    int kbp[NI];       // 64 k + b, or -1 past the last item
#pragma unroll
    for (int u = 0; u < NI; ++u) {
        const int kb = (tid >> 4) + 16 * u;
        kbp[u] = -1;
        off[u] = 0;
        if (kb < NA * B) {
            const int k = kb / B, b = kb % B;
            int pl;
            if constexpr (NK)
                pl = plane_w(n, nm);
            else
                pl = k == 0 ? plane_g(n - 3, nm) : k == 1 ? plane_g(n - 1, nm) : k == 2 ? plane_g(-n - 1, nm)
                   : k == 3 ? plane_g(-n - 3, nm) : k == 4 ? plane_g(-n - 1, nm) : k == 5 ? plane_g(n - 1, nm)
                   : plane_w(n, nm);
            kbp[u] = 64 * k + b;
            off[u] = (unsigned)chunk_offset(pl, 0, b, a.K, B);
        }
    }
    // this thread's outputs: LDS rows of X (bits 0-12) and Y (bits 13-25)
    // and the conjugation of Y (bit 26)
    int xyo[kEdgeAcc];
#pragma unroll
    for (int k = 0; k < kEdgeAcc; ++k) {
        const int o = tid + 256 * k;
        xyo[k] = 0;
        if (o < nout) {
            const int mu = NK ? 4 : o / E;
            int b1, b2;
            edge_output(o % E, B, b1, b2);
            const int ia = NK ? 0 : (mu == 4 ? 6 : (mu == 3 ? 0 : mu));
            const int ib = NK ? 1 : (mu == 4 ? 7 : ((mu == 0 || mu == 2) ? 3 : (mu == 1 ? 4 : 5)));
            xyo[k] = (ia * kEdgeMaxBins + b1) * kEdgeRow | (ib * kEdgeMaxBins + b2) * kEdgeRow << 13 |
                     (mu >= 3) << 26;
        }
    }

    float g[NI][2];
    float4 cw;
    auto load = [&](int i0) {
        const int ic = min(i0 + e, i_end - 1);  // clamped: masked when formed
        const unsigned co = (unsigned)(ic >> 2) * 4u * (unsigned)B + (unsigned)(ic & 3);
        cw = a.ccw[ic];
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            const int k = kbp[u] >> 6;
            const bool ysd = NK ? k == 1 : ((k >= 3 && k <= 5) || k == 7);
            const float *sp = ysd ? py : px;
            g[u][0] = sp[off[u] + co];
            g[u][1] = sp[off[u] + co + KB];
        }
    };
    auto stage = [&](int i0) {
        const bool ok = i0 + e < i_end;
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            if (kbp[u] < 0) continue;
            const int k = kbp[u] >> 6, b = kbp[u] & 63;
            float ar, ai;
            if constexpr (NK) {
                ar = k == 0 ? cw.z : 1.0f;
                ai = 0.0f;
            } else {
                ar = k < 3 ? -cw.x : (k == 6 ? cw.z : 1.0f);
                ai = k < 3 ? (k == 1 ? cw.y : -cw.y) : 0.0f;
            }
            const float gr = g[u][0], gi = (!NK && k == 2) ? -g[u][1] : g[u][1];
            float2 v = make_float2(fmaf(ar, gr, -ai * gi), fmaf(ar, gi, ai * gr));
            if (!ok) v = make_float2(0.f, 0.f);
            op[(k * kEdgeMaxBins + b) * kEdgeRow + e] = v;
        }
    };

    double accr[kEdgeAcc], acci[kEdgeAcc];
#pragma unroll
    for (int k = 0; k < kEdgeAcc; ++k) accr[k] = acci[k] = 0.0;
    load(i_begin);
    for (int i0 = i_begin; i0 < i_end; i0 += kEdgeBlk) {
        stage(i0);
        __syncthreads();
        if (i0 + kEdgeBlk < i_end) load(i0 + kEdgeBlk);
#pragma unroll
        for (int k = 0; k < kEdgeAcc; ++k) {
            if (tid + 256 * k < nout) {
                float sr = 0.0f, si = 0.0f;
                const float2 *xp = op + (xyo[k] & 8191), *yp = op + ((xyo[k] >> 13) & 8191);
                const float ys = (xyo[k] >> 26) ? -1.0f : 1.0f;
#pragma unroll 4
                for (int c = 0; c < kEdgeBlk; ++c) {
                    const float2 x = xp[c], y = yp[c];
                    const float yi = ys * y.y;
                    sr = fmaf(x.x, y.x, fmaf(-x.y, yi, sr));
                    si = fmaf(x.x, yi, fmaf(x.y, y.x, si));
                }
                accr[k] += (double)sr;
                acci[k] += (double)si;
            }
        }
        __syncthreads();
    }
    const int nq = 4 * (nm + 1) + a.w_max + 1;
    double *base = a.partial + ((size_t)pair * a.S + sl) * nq * B * B * 2;
#pragma unroll
    for (int k = 0; k < kEdgeAcc; ++k) {
        const int o = tid + 256 * k;
        if (o < nout) {
            const int mu = NK ? 4 : o / E;
            int b1, b2;
            edge_output(o % E, B, b1, b2);
            const int q = mu < 4 ? mu * (nm + 1) + n : 4 * (nm + 1) + n;
            double2 v;
            v.x = accr[k];
            v.y = acci[k];
            *reinterpret_cast<double2 *>(base + ((size_t)q * B * B + (size_t)b1 * B + b2) * 2) = v;
        }
    }
}

// Row scales for FP16X3, in two steps.  k_fp16_max: for every order n,
// operand array (the three X and three Y arrays of the Upsilon kernel) and
// bin, the largest |Re| or |Im| over the chunk's centres, formed with exactly
// the arithmetic of k_contract; grid.z splits the centres and the partial
// maxima meet in an integer atomicMax on the float bits (exact and order
// independent for values >= 0).  k_fp16_scale: the power of two that brings
// that maximum into [2^11, 2^12).
constexpr int kScaleSplit = 16;

__global__ __launch_bounds__(256) void k_fp16_max(ContractArgs a, unsigned *mx_all)
{
    // grid.y = (pair, side, bin tile)
    const int nt = (a.B + 31) >> 5;
    const int n = blockIdx.x, tile = (int)blockIdx.y % nt;
    const int side = ((int)blockIdx.y / nt) & 1, pair = ((int)blockIdx.y / nt) >> 1;
    const float *px, *py;
    pair_planes(a, pair, px, py);
    const int nm = a.n_max;
    const int bl = threadIdx.x & 31, b = 32 * tile + bl, g = threadIdx.x >> 5;
    int pl[3];
    if (side == 0) {
        pl[0] = plane_g(n - 3, nm);
        pl[1] = plane_g(n - 1, nm);
        pl[2] = plane_g(-n - 1, nm);
    } else {
        pl[0] = plane_g(-n - 3, nm);
        pl[1] = plane_g(-n - 1, nm);
        pl[2] = plane_g(n - 1, nm);
    }
    const float *src = side ? py : px;
    const int nq = (a.n_c + 3) >> 2;
    const int per = (nq + kScaleSplit - 1) / kScaleSplit;
    const int q_end = min(nq, ((int)blockIdx.z + 1) * per);
    const int bc = min(b, a.B - 1);
    float m[3] = {0.f, 0.f, 0.f};
    for (int q = (int)blockIdx.z * per + g; q < q_end; q += 8) {
        const int i4 = 4 * q;
        const int nv = b < a.B ? min(4, a.n_c - i4) : 0;
        float4 re[3], im[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            re[k] = keep(*reinterpret_cast<const float4 *>(src + chunk_offset(pl[k], i4, bc, a.K, a.B)), nv);
            im[k] = keep(*reinterpret_cast<const float4 *>(src + chunk_offset(pl[k] + 1, i4, bc, a.K, a.B)), nv);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float2 o[3];
            const float2 g0 = make_float2(comp(re[0], e), comp(im[0], e));
            const float2 g1 = make_float2(comp(re[1], e), comp(im[1], e));
            const float2 g2 = make_float2(comp(re[2], e), comp(im[2], e));
            if (side == 0) {
                const float4 f = a.ccw[min(i4 + e, a.n_c - 1)];
                x_operands(f.x, f.y, g0, g1, g2, o);
            } else {
                o[0] = g0;
                o[1] = g1;
                o[2] = g2;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) m[k] = fmaxf(m[k], fmaxf(fabsf(o[k].x), fabsf(o[k].y)));
        }
    }
    __shared__ float sm[3][8][32];
#pragma unroll
    for (int k = 0; k < 3; ++k) sm[k][g][bl] = m[k];
    __syncthreads();
    if (threadIdx.x < 96) {
        const int k = threadIdx.x >> 5;
        float mx = 0.f;
        for (int j = 0; j < 8; ++j) mx = fmaxf(mx, sm[k][j][bl]);
        atomicMax(mx_all + (((size_t)pair * (nm + 1) + n) * kNYArr + 3 * side + k) * kScaleRows + b,
                  __float_as_uint(mx));
    }
}

__global__ void k_fp16_scale(const unsigned *mx, float *scale, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float m = __uint_as_float(mx[t]);
    scale[t] = (m > 0.0f && isfinite(m)) ? ldexpf(1.0f, 11 - ilogbf(m)) : 1.0f;  // m in [2^e, 2^{e+1})
}

__global__ void k_zero_u32(unsigned *p, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0u;
}

// Diagonal (j = k) sums E_mu(b) = sum_i alpha_i D_mu(i, b) in FP64, for all
// five components.  One workgroup per (bin, catalog, centre range); the
// kDiagSplit partial sums are added in a fixed order by k_reduce.
constexpr int kDiagSplit = 16;

__global__ __launch_bounds__(256) void k_diag(const float *planes0, size_t zstride, const float4 *ccw,
                                              int n_c, int K, int B, int pD, int n_z, double *E0)
{
    const int b = blockIdx.x;
    const float *planes = planes0 + (size_t)blockIdx.y * zstride;
    double *E = E0 + ((size_t)blockIdx.z * n_z + blockIdx.y) * 10 * B;
    double acc[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) acc[j] = 0.0;
    const int nq = (n_c + 3) >> 2;
    const int per = (nq + kDiagSplit - 1) / kDiagSplit;
    const int q_end = min(nq, ((int)blockIdx.z + 1) * per);
    for (int q = (int)blockIdx.z * per + threadIdx.x; q < q_end; q += blockDim.x) {
        const int i4 = 4 * q;
        const int nv = min(4, n_c - i4);
        float4 d[7];
#pragma unroll
        for (int k = 0; k < 7; ++k)
            d[k] = keep(*reinterpret_cast<const float4 *>(planes + chunk_offset(pD + k, i4, b, K, B)), nv);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float4 f = ccw[min(i4 + e, n_c - 1)];
#pragma unroll
            for (int mu = 0; mu < 5; ++mu) {
                float ar, ai;
                alpha_of(mu, f, ar, ai);
                const int k = mu == 0 ? 0 : (mu == 1 ? 2 : (mu == 4 ? 6 : 4));
                const double dr = comp(d[k], e);
                const double di = mu == 4 ? 0.0 : (double)comp(d[k + 1], e);
                acc[2 * mu] += (double)ar * dr - (double)ai * di;
                acc[2 * mu + 1] += (double)ar * di + (double)ai * dr;
            }
        }
    }
    __shared__ double sred[10][256];
#pragma unroll
    for (int j = 0; j < 10; ++j) sred[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
#pragma unroll
            for (int j = 0; j < 10; ++j) sred[j][threadIdx.x] += sred[j][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x < 10) {
        const int mu = threadIdx.x >> 1, part = threadIdx.x & 1;
        E[2 * (mu * B + b) + part] = sred[threadIdx.x][0];
    }
}

// out[pair][block][b1][b2] += sum_s partial[pair][s][...] - [b1 == b2][Z2 == Z3] E_{Z2,mu}(b1),
// blocks mu (n_max+1) + n (Upsilon) and 4 (n_max+1) + n (N, every order)
__global__ void k_reduce(const double *partial, int S, int n_max, int w_max, int B, int n_z,
                         const double *E, int jk, double *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)(4 * (n_max + 1) + w_max + 1) * B * B;
    if (t >= per * n_z * n_z) return;
    const int pair = (int)(t / per);
    const int64_t e = t % per;
    const int b2 = (int)(e % B);
    const int b1 = (int)((e / B) % B);
    const int qb = (int)(e / ((int64_t)B * B));
    const int mu = qb < 4 * (n_max + 1) ? qb / (n_max + 1) : 4;
    const double *p = partial + 2 * ((int64_t)pair * S * per + e);
    double re = 0.0, im = 0.0;
    for (int s = 0; s < S; ++s) {
        re += p[2 * s * per];
        im += p[2 * s * per + 1];
    }
    const int z2 = pair / n_z, z3 = pair % n_z;
    if (jk && z2 == z3 && b1 == b2) {
        double er = 0.0, ei = 0.0;
        for (int sp = 0; sp < kDiagSplit; ++sp) {
            const double *Ez = E + ((size_t)sp * n_z + z2) * 10 * B;
            er += Ez[2 * (mu * B + b1)];
            ei += Ez[2 * (mu * B + b1) + 1];
        }
        re -= er;
        im -= ei;
    }
    out[2 * t] += re;
    out[2 * t + 1] += im;
}

// MFMA tiles per side of a B x B block: B = 33..40 keeps one tile and sums
// the bins past it in k_contract_edge.
int mfma_tiles(int B) { return B <= kEdgeMaxBins ? 1 : (B + kRows - 1) / kRows; }
bool edge_bins(int B) { return B > kEdgeT && B <= kEdgeMaxBins; }

// T = ceil(2B / 16) tiles per side; NIS = staging items per producer thread
// and side (the NA / 2 complex arrays of a side hold 4 B items each).
template <int PK, bool NK, bool SAME>
void launch_small_same(int B, dim3 g, hipStream_t s, const ContractArgs &a)
{
    const int T = (2 * B + 15) / 16;
    const int NIS = ((NK ? 4 : 3) * 4 * B + 255) / 256;
    if (T == 1)
        hipLaunchKernelGGL((k_contract_small<PK, 1, NK, 1, SAME>), g, dim3(512), 0, s, a);
    else if (T == 2 && NIS == 1)
        hipLaunchKernelGGL((k_contract_small<PK, 2, NK, 1, SAME>), g, dim3(512), 0, s, a);
    else if (T == 2)
        hipLaunchKernelGGL((k_contract_small<PK, 2, NK, 2, SAME>), g, dim3(512), 0, s, a);
    else if (NIS == 1)
        hipLaunchKernelGGL((k_contract_small<PK, 3, NK, 1, SAME>), g, dim3(512), 0, s, a);
    else
        hipLaunchKernelGGL((k_contract_small<PK, 3, NK, 2, SAME>), g, dim3(512), 0, s, a);
}

// same: one catalog (Z2 = Z3 for every launched pair), for the N_n kernel
template <int PK, bool NK>
void launch_small(int B, dim3 g, hipStream_t s, const ContractArgs &a, bool same = false)
{
    if (NK && same)
        launch_small_same<PK, NK, NK>(B, g, s, a);
    else
        launch_small_same<PK, NK, false>(B, g, s, a);
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
// every chunk of a call fits the buffers reserved up front.  The Upsilon
// kernel runs (n_max + 1) n_z^2 t^2 workgroups per slice (t bin tiles per
// side); slice s runs on XCD s mod 8, whose 32 compute units hold 64
// workgroups at a time.  The slice length (a multiple of the FP32 run)
// minimises the busiest XCD's rounds x (length + 64), the time of the launch
// with the cost of writing and reducing one partial tile counted as 64
// centres of work, preferring longer slices on ties.  (Counting rounds over
// the whole chip instead left up to one XCD in eight with twice the slices
// of the others: 5-bin tomography stage 2 at 1.24 s instead of 0.9 s.)
int contract_slice(const ChunkLayout &L, int n_z)
{
    const int64_t nt = mfma_tiles(L.B);
    const int64_t per_slice = (int64_t)(L.n_max + 1) * n_z * n_z * nt * nt;
    const int64_t slots_xcd = 2 * 32;
    int best = kSliceStep;
    int64_t best_cost = INT64_MAX;
    for (int slice = kSliceStep; slice <= 4096; slice += kSliceStep) {
        const int64_t S = (L.K + slice - 1) / slice;
        const int64_t busiest = (S + 7) / 8;  // slices of the busiest XCD
        const int64_t rounds = (per_slice * busiest + slots_xcd - 1) / slots_xcd;
        const int64_t cost = rounds * (slice + 64);
        if (cost <= best_cost) {
            best_cost = cost;
            best = slice;
        }
        if (S == 1) break;
    }
    return best;
}

size_t contract_arena_bytes(const t3_plan *plan, const ChunkLayout &L, int n_z)
{
    const int pairs = n_z * n_z;
    const int S = (L.K + contract_slice(L, n_z) - 1) / contract_slice(L, n_z);
    const size_t per = (size_t)L.out_blocks() * L.B * L.B;
    size_t b = arena_bytes(sizeof(double) * 2 * per * (size_t)S * pairs) +
               arena_bytes(sizeof(double) * 2 * 5 * (size_t)L.B * n_z * kDiagSplit);
    if (plan->precision == T3_PREC_FP16X3)
        b += arena_bytes(2 * sizeof(float) * (size_t)kNYArr * kScaleRows * (L.n_max + 1) * pairs);
    return b;
}

int reserve_contract(t3_plan *plan, const ChunkLayout &L, int n_z)
{
    const int pairs = n_z * n_z;
    const int S = (L.K + contract_slice(L, n_z) - 1) / contract_slice(L, n_z);
    const size_t per = (size_t)L.out_blocks() * L.B * L.B;
    T3_TRY(plan->partial.reserve(sizeof(double) * 2 * per * (size_t)S * pairs));
    T3_TRY(plan->diag.reserve(sizeof(double) * 2 * 5 * (size_t)L.B * n_z * kDiagSplit));
    if (plan->precision == T3_PREC_FP16X3)  // maxima (u32) then scales (f32)
        T3_TRY(plan->scales.reserve(2 * sizeof(float) * (size_t)kNYArr * kScaleRows * (L.n_max + 1) * pairs));
    return T3_OK;
}

int contract_chunk(t3_plan *plan, const CentreSet &cs, int64_t c0, int n_c, const ChunkLayout &L,
                   const float *planes, size_t zstride, int n_z, bool jk, double *ups_out, hipStream_t s)
{
    if (n_c <= 0) return T3_OK;
    if (L.B > kMaxRadialBins) return T3_ERANGE;
    if (L.floats() >= ((size_t)1 << 31)) return T3_ERANGE;  // 32-bit plane offsets in k_contract
    const int pairs = n_z * n_z;
    const int slice = contract_slice(L, n_z);
    const int S = (n_c + slice - 1) / slice;
    const size_t per = (size_t)L.out_blocks() * L.B * L.B;
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
    a.w_max = L.w_max;
    a.slice = slice;
    a.S = S;
    a.partial = plan->partial.as<double>();
    a.nt = mfma_tiles(L.B);
    const int S8 = 8 * ((S + 7) / 8);  // slices padded to whole XCD rounds
    const unsigned nt = (unsigned)a.nt;  // bin tiles per side (grid.y: tile pairs)
    const dim3 gy((unsigned)((L.n_max + 1) * S8 * pairs), nt * nt);
    const dim3 gn((unsigned)((L.w_max + 2) / 2 * S8 * pairs), nt * nt);
    const dim3 blk(256);
    // B <= 24: the real-embedded 16 x 16 tiles (unless the plan asks for the
    // complex 32 x 32 ones)
    const bool small = L.B <= kSmallBins && plan->tile_mode == 0;
    const dim3 gs((unsigned)((L.n_max + 1) * S8 * pairs));
    const dim3 gsn((unsigned)((L.w_max + 1) * S8 * pairs));
    switch (plan->precision) {
        case T3_PREC_FP32:
            if (small)
                launch_small<T3_PREC_FP32, false>(L.B, gs, s, a);
            else
                hipLaunchKernelGGL((k_contract<T3_PREC_FP32, false>), gy, blk, 0, s, a);
            break;
        case T3_PREC_BF16X3:
            if (small)
                launch_small<T3_PREC_BF16X3, false>(L.B, gs, s, a);
            else
                hipLaunchKernelGGL((k_contract<T3_PREC_BF16X3, false>), gy, blk, 0, s, a);
            break;
        case T3_PREC_BF16X6:
            if (small)
                launch_small<T3_PREC_BF16X6, false>(L.B, gs, s, a);
            else
                hipLaunchKernelGGL((k_contract<T3_PREC_BF16X6, false>), gy, blk, 0, s, a);
            break;
        default: {
            const int ns = kNYArr * kScaleRows * (L.n_max + 1) * pairs;
            unsigned *mx = plan->scales.as<unsigned>();
            float *sc = plan->scales.as<float>() + ns;
            hipLaunchKernelGGL(k_zero_u32, dim3((ns + 255) / 256), blk, 0, s, mx, ns);
            hipLaunchKernelGGL(k_fp16_max, dim3(L.n_max + 1, 2 * pairs * nt, kScaleSplit), blk, 0, s, a, mx);
            hipLaunchKernelGGL(k_fp16_scale, dim3((ns + 255) / 256), blk, 0, s, (const unsigned *)mx, sc, ns);
            T3_HIP_CHECK(hipGetLastError());
            a.scale = sc;
            if (small)
                launch_small<T3_PREC_FP16X3, false>(L.B, gs, s, a);
            else
                hipLaunchKernelGGL((k_contract<T3_PREC_FP16X3, false>), gy, blk, 0, s, a);
            break;
        }
    }
    T3_HIP_CHECK(hipGetLastError());
    if (small)
        launch_small<T3_PREC_FP32, true>(L.B, gsn, s, a, n_z == 1);
    else
        hipLaunchKernelGGL((k_contract<T3_PREC_FP32, true>), gn, blk, 0, s, a);
    T3_HIP_CHECK(hipGetLastError());
    if (edge_bins(L.B)) {
        hipLaunchKernelGGL(k_contract_edge<false>, dim3((unsigned)(S * pairs), L.n_max + 1), blk, 0, s, a);
        T3_HIP_CHECK(hipGetLastError());
        if (L.w_max > L.n_max) {
            hipLaunchKernelGGL(k_contract_edge<true>, dim3((unsigned)(S * pairs), L.w_max - L.n_max), blk, 0, s, a);
            T3_HIP_CHECK(hipGetLastError());
        }
    }
    if (jk) {
        hipLaunchKernelGGL(k_diag, dim3(L.B, n_z, kDiagSplit), dim3(256), 0, s, planes, zstride, a.ccw, n_c,
                           L.K, L.B, L.plane_D(0), n_z, plan->diag.as<double>());
        T3_HIP_CHECK(hipGetLastError());
    }
    const size_t tot = per * pairs;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       (const double *)plan->partial.as<double>(), S, L.n_max, L.w_max, L.B, n_z,
                       (const double *)plan->diag.as<double>(), jk ? 1 : 0, ups_out);
    T3_HIP_CHECK(hipGetLastError());
    return T3_OK;
}

}  // namespace t3
