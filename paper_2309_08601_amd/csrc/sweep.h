// Annulus sweep over the cell list: the neighbour search shared by the
// forward scan and its adjoint (spatial hashing, Porth et al. 2023, Sect. 3.1).
//
// For one centre and one radial bin [e_b, e_{b+1}) a wavefront
//  1. builds, per cell row, at most two runs of cells that can hold in-bin
//     neighbours (computed in FP64 from the exact lattice position of the
//     centre); each run is one contiguous range of the cell-sorted catalog;
//  2. concatenates the ranges of 64 rows into one virtual candidate list
//     (wave prefix sum of the range lengths, kept in LDS) and walks it 64
//     candidates at a time, every lane one candidate, so loads are coalesced
//     and no lane idles on short ranges;
//  3. prefetches the next candidate's position and factors into registers
//     before handling the current ones, so the L2 / last-level-cache latency
//     overlaps the harmonic work;
//  4. tests exact squared separations against the FP64 squared edges and
//     compacts in-bin neighbours with a ballot into a 128-entry LDS ring;
//     every time 64 are pending the caller's batch routine runs once, each
//     lane taking one neighbour.
#pragma once

#include "t3_internal.h"

namespace t3 {

constexpr int kRing = 128;   // LDS ring entries per wavefront
constexpr int kRowsPerBlock = 64;

struct SweepArgs {
    const int2 *npos;       // cell-sorted neighbour positions
    const float4 *ncw;      // (w g1, w g2, w, 0) in the same order
    const int *cell_start;  // [ncells + 1]
    CellGrid g;
};

// Per-wavefront LDS slices.
struct SweepLDS {
    int4 *q_xyc;  // [kRing] dx, dy, bits(Re c), bits(Im c)
    int2 *q_wi;   // [kRing] bits(w), sorted index of the neighbour
    int2 *span;   // [2 * kRowsPerBlock + 1] (virtual begin, first galaxy)
};

// floor(a / b) for integers |a| < 2^53, b > 0, in FP64 (cheaper than a 64-bit
// integer division): an integral quotient is exact, and any other lies at
// least 1/b from an integer, more than the error |a / b| 2^-53 of one
// correctly rounded division.
__device__ __forceinline__ long long floor_div(long long a, long long b)
{
    return (long long)floor((double)a / (double)b);
}

__device__ __forceinline__ long long ceil_div(long long a, long long b)
{
    return (long long)ceil((double)a / (double)b);
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Galaxy ranges [sa.x, sa.y) and [sb.x, sb.y) of cell row r that can hold
// neighbours of p with e2lo <= r^2 < e2hi (empty ranges have x == y).
__device__ __forceinline__ void row_ranges(const SweepArgs &a, int2 p, long long r, double e2lo,
                                           double e2hi, int2 &sa, int2 &sb)
{
    const CellGrid &g = a.g;
    sa = make_int2(0, 0);
    sb = make_int2(0, 0);
    const long long y0 = (long long)g.oy + r * g.cell;
    const long long y1 = y0 + g.cell - 1;
    const long long py = p.y, px = p.x;
    const long long dyn = py < y0 ? y0 - py : (py > y1 ? py - y1 : 0);
    const long long d0 = y0 - py < 0 ? py - y0 : y0 - py;
    const long long d1 = y1 - py < 0 ? py - y1 : y1 - py;
    const long long dyx = d0 > d1 ? d0 : d1;
    const double dmin2 = (double)dyn * (double)dyn;
    const double dmax2 = (double)dyx * (double)dyx;
    if (!(dmin2 < e2hi)) return;
    const long long xr = (long long)sqrt(e2hi - dmin2) + 1;
    long long c_lo = floor_div(px - xr - g.ox, g.cell);
    long long c_hi = floor_div(px + xr - g.ox, g.cell);
    c_lo = c_lo < 0 ? 0 : c_lo;
    c_hi = c_hi > g.ncx - 1 ? g.ncx - 1 : c_hi;
    if (c_lo > c_hi) return;
    long long a0 = c_lo, a1 = c_hi, b0 = 1, b1 = 0;
    if (e2lo > dmax2) {
        // cells whose every point is closer than e_b are skipped
        const long long xin = (long long)sqrt(e2lo - dmax2) - 1;
        if (xin >= 0) {
            const long long in_lo = ceil_div(px - xin - g.ox, g.cell);
            const long long in_hi = floor_div(px + xin - g.ox + 1, g.cell) - 1;
            if (in_lo <= in_hi) {
                a1 = c_hi < in_lo - 1 ? c_hi : in_lo - 1;
                b0 = c_lo > in_hi + 1 ? c_lo : in_hi + 1;
                b1 = c_hi;
            }
        }
    }
    const int *cs = a.cell_start + r * g.ncx;
    if (a0 <= a1) sa = make_int2(cs[a0], cs[a1 + 1]);
    if (b0 <= b1) sb = make_int2(cs[b0], cs[b1 + 1]);
}

// Virtual index v -> galaxy index, advancing the lane's span cursor t.
__device__ __forceinline__ int locate(const int2 *span, int &t, int v)
{
    while (span[t + 1].x <= v) ++t;
    const int2 s = span[t];
    return s.y + (v - s.x);
}

// Sweep one annulus: the candidate walk and the compaction into the LDS ring
// are shared; consume(head, count) is called (wave-uniformly) whenever 64
// neighbours are pending (count = 64) and once at the end for the remainder
// (0 < count < 64), with the ring index of the first pending entry.
// row_off, row_step: this wavefront sweeps only the cell rows row_lo +
// row_off + k row_step (wavefronts that split one annulus between them).
// Returns the number of in-bin neighbours (wave-uniform).
template <class Consume>
__device__ __forceinline__ int sweep_core(const SweepArgs &a, int2 cp, double e2lo, double e2hi, int lane,
                                          const SweepLDS &L, Consume &&consume, int row_off, int row_step)
{
    const CellGrid &g = a.g;
    const long long R = (long long)sqrt(e2hi) + 1;
    long long row_lo = floor_div((long long)cp.y - R - g.oy, g.cell);
    long long row_hi = floor_div((long long)cp.y + R - g.oy, g.cell);
    row_lo = row_lo < 0 ? 0 : row_lo;
    row_hi = row_hi > g.ncy - 1 ? g.ncy - 1 : row_hi;

    int head = 0, tail = 0;  // wave-uniform ring counters
    for (long long r0 = row_lo + row_off; r0 <= row_hi; r0 += (long long)kRowsPerBlock * row_step) {
        // ---- ranges of this lane's row, then a wave prefix sum of lengths
        int2 sa = make_int2(0, 0), sb = make_int2(0, 0);
        const long long row = r0 + (long long)lane * row_step;
        if (row <= row_hi) row_ranges(a, cp, row, e2lo, e2hi, sa, sb);
        const int la = sa.y - sa.x, lb = sb.y - sb.x;
        int incl = la + lb;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int o = __shfl_up(incl, d, 64);
            if (lane >= d) incl += o;
        }
        const int excl = incl - la - lb;
        const int total = __shfl(incl, 63, 64);
        L.span[2 * lane] = make_int2(excl, sa.x);
        L.span[2 * lane + 1] = make_int2(excl + la, sb.x);
        if (lane == 0) L.span[2 * kRowsPerBlock] = make_int2(0x7fffffff, 0);
        wave_sync_lds();
        if (total == 0) continue;

        // ---- walk the virtual list, prefetching one step ahead (a lane past
        // the end loads the list's last candidate again and is masked off)
        int t = 0;
        int v = lane;
        bool valid = v < total;
        int gi = locate(L.span, t, valid ? v : total - 1);
        int2 p = a.npos[gi];
        float4 c = a.ncw[gi];
        for (int v0 = 0; v0 < total; v0 += 64) {
            const int vn = v0 + 64 + lane;
            const bool valid_n = vn < total;
            const int gn = locate(L.span, t, valid_n ? vn : total - 1);
            const int2 pn = a.npos[gn];
            const float4 cn = a.ncw[gn];
            const int dx = p.x - cp.x, dy = p.y - cp.y;
            const double r2 = fma((double)dx, (double)dx, (double)dy * (double)dy);
            const bool in = valid && r2 >= e2lo && r2 < e2hi;
            const unsigned long long m = __ballot(in);
            if (in) {
                const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                const int slot = (tail + below) & (kRing - 1);
                L.q_xyc[slot] = make_int4(dx, dy, __float_as_int(c.x), __float_as_int(c.y));
                L.q_wi[slot] = make_int2(__float_as_int(c.z), gi);
            }
            tail += __popcll(m);
            if (tail - head >= 64) {
                wave_sync_lds();
                consume(head, 64);
                head += 64;
                __builtin_amdgcn_wave_barrier();
            }
            valid = valid_n;
            gi = gn;
            p = pn;
            c = cn;
        }
        wave_sync_lds();
    }
    if (tail > head) {
        wave_sync_lds();
        consume(head, tail - head);
        __builtin_amdgcn_wave_barrier();
    }
    return tail;
}

// Sweep one annulus, every lane one pending neighbour per batch.
// batch(e, ew, gidx, active) is called with the lane's queue entry (inactive
// lanes of the last batch get dx = 1, dy = 0 and zero factors); it must not
// touch the LDS slices.
template <class Batch>
__device__ __forceinline__ int sweep_annulus(const SweepArgs &a, int2 cp, double e2lo, double e2hi,
                                             int lane, const SweepLDS &L, Batch &&batch, int row_off = 0,
                                             int row_step = 1)
{
    return sweep_core(
        a, cp, e2lo, e2hi, lane, L,
        [&](int head, int count) {
            const bool act = lane < count;
            const int slot = (head + lane) & (kRing - 1);
            int4 e = L.q_xyc[slot];
            int2 ew = L.q_wi[slot];
            if (!act) {
                e = make_int4(1, 0, 0, 0);
                ew = make_int2(0, 0);
            }
            batch(e, __int_as_float(ew.x), ew.y, act);
        },
        row_off, row_step);
}

// Sweep one annulus, every half-wave (lanes 0-31, 32-63) taking all pending
// neighbours of a batch in two steps: in step 0 a lower-half lane gets entry
// (lane & 31) and an upper-half lane entry 32 + (lane & 31), in step 1 the
// other one.  Per batch, prep(e, j) is first called with each lane's own
// entry j = lane (for per-entry values in the caller's wavefront-private
// LDS, visible to every lane afterwards), then item(e, ew, step, j) for each
// step, then done() once.  Inactive entries as in sweep_annulus.
template <class Prep, class Item, class Done>
__device__ __forceinline__ int sweep_annulus_halves(const SweepArgs &a, int2 cp, double e2lo, double e2hi,
                                                    int lane, const SweepLDS &L, Prep &&prep, Item &&item,
                                                    Done &&done)
{
    return sweep_core(
        a, cp, e2lo, e2hi, lane, L,
        [&](int head, int count) {
            int4 e0 = L.q_xyc[(head + lane) & (kRing - 1)];
            if (lane >= count) e0 = make_int4(1, 0, 0, 0);
            prep(e0, lane);
            wave_sync_lds();
#pragma unroll 1
            for (int k = 0; k < 2; ++k) {
                const int j = (((lane >> 5) ^ k) << 5) + (lane & 31);
                const bool act = j < count;
                const int slot = (head + j) & (kRing - 1);
                int4 e = L.q_xyc[slot];
                int2 ew = L.q_wi[slot];
                if (!act) {
                    e = make_int4(1, 0, 0, 0);
                    ew = make_int2(0, 0);
                }
                item(e, __int_as_float(ew.x), k, j);
            }
            done();
        },
        0, 1);
}

}  // namespace t3
