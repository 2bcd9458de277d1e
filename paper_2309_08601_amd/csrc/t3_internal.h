// Internal declarations shared by the t3pcf HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "t3pcf.h"

namespace t3 {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

#define T3_HIP_CHECK(expr)                                                          \
    do {                                                                            \
        hipError_t _e = (expr);                                                     \
        if (_e != hipSuccess)                                                       \
            return ::t3::fail(T3_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

#define T3_TRY(expr)                  \
    do {                              \
        int _rc = (expr);             \
        if (_rc != T3_OK) return _rc; \
    } while (0)

// ---------------------------------------------------------------- device buffers
// Device memory budget of a plan (t3_params.max_workspace_bytes).  Every
// entry point that can allocate installs its plan's budget for the calling
// thread (a plan is never used from two threads at once); DevBuf::reserve
// checks the limit before it calls hipMalloc and keeps the running total.
struct Budget {
    int64_t limit = 0;  // bytes, 0 = unlimited
    int64_t used = 0;   // bytes held by the plan's buffers
    int64_t peak = 0;   // largest value of used
};
Budget *active_budget();
struct BudgetScope {
    Budget *prev;
    explicit BudgetScope(Budget *b);
    ~BudgetScope();
};

// Grow-only device allocation owned by a plan.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int reserve(size_t want);
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Device memory the no-allocation entry point carves its buffers from
// (bump allocation, 256-byte aligned, nothing freed).  While an ArenaScope
// is active on a thread, DevBuf::reserve carves from the arena instead of
// allocating, remembering each buffer's previous state, and the scope's end
// gives every such buffer back its previous (plan-owned) state.
struct Arena {
    char *base = nullptr;
    size_t size = 0, used = 0;
    std::vector<std::pair<DevBuf *, DevBuf>> saved;
};
struct ArenaScope {
    Arena *prev;
    Arena *mine;
    explicit ArenaScope(Arena *a);
    ~ArenaScope();
};
// Bytes one carve of `want` bytes takes from an arena (256-byte granules,
// at least one, as DevBuf::reserve allocates).
inline size_t arena_bytes(size_t want) { return ((want < 256 ? 256 : want) + 255) & ~(size_t)255; }

// ---------------------------------------------------------------- chunk layout
// Stage-1 output for a chunk of K centres (K a multiple of 4): "planes" of
// FP32 values, one plane per (order, real/imag part) or per j = k sum.
// Element (plane p, centre i, bin b) lives at
//     ((p * (K/4) + i/4) * B + b) * 4 + (i & 3)
// so that four consecutive centres of one bin are one 16-byte vector and a
// row of B bins for those four centres is contiguous (stage-2 operand load).
// Plane numbering, with n_g = 2 n_max + 3 G orders m = -n_max-3 .. n_max-1
// and W orders m = 0 .. w_max (w_max = n_max, or 2 n_max when the
// mode-coupling matrix is wanted):
//     G_m   : 2 (m + n_max + 3) + {0 re, 1 im}
//     W_m   : 2 n_g + 2 m + {0, 1},          m = 0 .. w_max
//     D     : 2 n_g + 2 (w_max + 1) + {0..6} = D6 re, D6 im, D2 re, D2 im,
//             DA re, DA im, DW
struct ChunkLayout {
    int n_max = 0, w_max = 0, B = 0, K = 0;
    int n_g() const { return 2 * n_max + 3; }
    int plane_G(int m, int part) const { return 2 * (m + n_max + 3) + part; }
    int plane_W(int m, int part) const { return 2 * n_g() + 2 * m + part; }
    int plane_D(int d) const { return 2 * n_g() + 2 * (w_max + 1) + d; }
    int n_planes() const { return plane_D(0) + 7; }
    size_t plane_stride() const { return (size_t)K * B; }  // floats per plane
    size_t floats() const { return (size_t)n_planes() * plane_stride(); }
    // output blocks of B x B complex per set: Upsilon_{0..3, n <= n_max}, N_{n <= w_max}
    int out_blocks() const { return 4 * (n_max + 1) + w_max + 1; }
};

__host__ __device__ inline size_t chunk_offset(int p, int i, int b, int K, int B)
{
    return (((size_t)p * (K >> 2) + (size_t)(i >> 2)) * B + b) * 4 + (i & 3);
}

// ---------------------------------------------------------------- cell grid
struct CellGrid {
    int cell = 1;        // side, lattice steps
    int ncx = 1, ncy = 1;
    int ox = 0, oy = 0;  // lattice origin of cell (0, 0)
    int64_t ncells() const { return (int64_t)ncx * ncy; }
};

// Cell-sorted copy of one neighbour catalog.
struct SortedCatalog {
    int64_t n = 0;
    CellGrid grid;
    DevBuf pos;         // int2  [n]   (x, y)
    DevBuf cw;          // float4[n]   (w g1, w g2, w, 0)
    DevBuf cell_start;  // int   [ncells + 1]
    DevBuf perm;        // int   [n]   sorted slot -> original index
    DevBuf keys;        // int   [n]   scratch
    DevBuf counts;      // int   [ncells + 1] scratch
    DevBuf scan_tmp;    // int   scratch for the block sums
};

// Centres of one forward call (gathered positions and factors).
struct CentreSet {
    int64_t n = 0;
    DevBuf pos;  // int2  [n]
    DevBuf cw;   // float4[n]
};

// Radial bins of a plan (stage 2 tiles the B x B blocks by 32 x 32).
constexpr int kMaxRadialBins = 64;

// One resolution of the grid-based estimator: its non-empty pixels as a
// catalog and the stage-1 planes of its bins at every pixel.
constexpr int kMaxGridLevels = 8;
struct GridLevel {
    int b_lo = 0, nb = 0;   // bins [b_lo, b_lo + nb) use this level
    int64_t side = 0;       // pixel side, lattice steps
    int64_t n_pix = 0;      // non-empty pixels
    SortedCatalog by_pix;   // galaxies sorted by pixel (cell = pixel)
    DevBuf pix_id;          // int [ncells + 1]: exclusive scan of the non-empty flags
    DevBuf pix_xy;          // int32 x [n_pix], y [n_pix]: pixel corners
    DevBuf pix_sum;         // double [n_pix][3]: sum w g1, sum w g2, sum w
    DevBuf pix_gw;          // float g1 [n_pix], g2 [n_pix], w [n_pix] (catalog view)
    DevBuf gal_pix;         // int [n_gal]: galaxy (input order) -> pixel
    SortedCatalog pix;      // the pixel catalog, cell-sorted for the sweep
    CentreSet pix_centres;  // every pixel, in pix's sorted order
    DevBuf slot_of_pix;     // int [n_pix]: pixel -> sorted slot in pix (pair-sum route)
    DevBuf cen_slot;        // int [n_gal]: galaxy (sorted slot) -> plane slot of its pixel
    DevBuf planes;          // stage-1 planes of every pixel, layout L: by sorted slot
                            // (pair-sum route) or by pixel index (FFT route)
    ChunkLayout L;
    int box[4] = {0, 0, 0, 0};  // occupied corners: x min, y min, x max, y max
    int nx_occ = 0, ny_occ = 0; // occupied extent, pixels
    double w_peak = 0;          // largest pixel weight / mean pixel weight
    int method = 0;             // route taken: T3_GRID_DIRECT or T3_GRID_FFT
    DevBuf fft_misc, fft_buf;   // FFT route: bounding box, grids and tables
    DevBuf fft_spec;            // FFT route: kernel spectra of every (bin, order)
    int64_t spec_key[7] = {-1, -1, -1, -1, -1, -1, -1};  // geometry the spectra belong to
    void release();
};

}  // namespace t3

// ---------------------------------------------------------------- plan
struct t3_plan {
    int B = 0, n_max = 0, precision = 0;
    int w_max = 0;  // n_max, or 2 n_max with T3_FLAG_EDGE_CORRECT
    uint32_t flags = 0;
    double unit = 0;
    std::vector<double> edges_lat;  // [B+1] edges in lattice steps
    std::vector<double> e2;         // [B+1] squared, lattice steps^2
    int32_t box_lo_x = 0, box_lo_y = 0;
    int64_t box_size = 0;
    double cell_arcmin = 0;
    int chunk_req = 0;
    int device = 0;

    t3::SortedCatalog cats[8];
    t3::CentreSet centres;      // centres of t3_harmonics / t3_backward
    t3::CentreSet csets[8];     // centres per tomographic bin of a forward call
    int scan_mode = 0;          // 0: one wavefront per task, 1: persistent work queue
    double lane_neighbours = 128.0;  // stage-1 bins with at most this many expected neighbours: one lane per centre
    int tile_mode = 0;          // stage 2, B <= 24: 0 real-embedded 16 x 16 tiles, 1 complex 32 x 32 tiles
    hipStream_t cap_stream = nullptr;     // graph capture stream (default priority)
    hipGraphExec_t graph_exec = nullptr;  // last captured forward schedule
    std::vector<int64_t> graph_key;       // what that schedule was captured for
    t3::DevBuf graph_out;                 // the schedule's output, copied to the caller's
    int64_t graph_captures = 0;           // schedules captured by this plan
    int64_t graph_replays = 0;            // graph launches (first launch included)
    t3::DevBuf chunk;     // stage-1 planes
    t3::DevBuf partial;   // stage-2 FP64 partial tiles
    t3::DevBuf diag;      // FP64 j = k sums per chunk
    t3::DevBuf flag;      // int error flag (lattice bounds)
    t3::DevBuf dest;      // int16 destination tables of the stage-1 passes
    t3::DevBuf scales;    // fp16 row scales
    t3::DevBuf counter;   // uint64 pair counter
    t3::DevBuf queue;     // persistent-scan work counter
    t3::DevBuf tune_idx;  // autotuner centre sample
    t3::DevBuf tune_out;  // autotuner output
    t3::DevBuf misc;      // adjoint scratch
    t3::DevBuf misc2;
    t3::DevBuf sph_a, sph_b, sph_out;  // sphere patches: projection, compaction, per-patch output
    t3::GridLevel grid[t3::kMaxGridLevels];  // grid-based estimator, level l at grid[l - 1]
    // T3_FLAG_KEEP_PLANES: stage-1 planes of every chunk of the last forward
    // (chunk c at c * kept_L.floats()), valid while cells_seq == kept_seq
    t3::DevBuf kept;
    t3::ChunkLayout kept_L;
    t3_catalog kept_cat{};
    int64_t cells_seq = 0;   // build_cells calls on this plan
    int64_t kept_seq = -1;
    t3::Budget budget;       // device memory held against max_workspace_bytes
    t3::DevBuf det;          // T3_FLAG_DETERMINISTIC adjoint: fixed-point and FP64 accumulators
    int scan_var = -1;          // stage-1 variant index (see scan.hip)
    size_t scan_dest_off[4] = {0, 0, 0, 0};  // main passes, the W extension, the order-segment kernel

    // optional stage timing (T3_FLAG_TIMING)
    std::vector<hipEvent_t> events;  // pool, pairs (start, stop)
    std::vector<int> event_stage;    // stage of each pair
    size_t events_used = 0;          // pairs recorded in the current call
    double stage_ms[4] = {0, 0, 0, 0};
    int64_t stage_launches[4] = {0, 0, 0, 0};
};

namespace t3 {

// Launchers (each returns T3_OK or an error; all asynchronous on `s`).
int build_cells(t3_plan *plan, SortedCatalog &sc, const t3_catalog &cat, const CellGrid &g,
                hipStream_t s);
int gather_centres(t3_plan *plan, const t3_catalog &cat, const int32_t *idx, int64_t n,
                   CentreSet &cs, hipStream_t s);
int gather_sorted_centres(t3_plan *plan, const SortedCatalog &sc, CentreSet &cs, hipStream_t s);
int check_flag(t3_plan *plan, hipStream_t s, const char *what);

int scan_prepare(t3_plan *plan);
// Whether the plan's stage-1 variant sweeps each annulus once for two order
// segments (k_scan_seg: n_max above one pass, up to 48).
bool scan_uses_segments(const t3_plan *plan);
// Stage 1 for centres [c0, c0 + n_c) of cs against n_z neighbour catalogs
// (planes of catalog z at planes + z * zstride).  mode 0: one wavefront per
// centre, one launch per catalog; mode 1: one persistent launch over every
// (centre, catalog) task with a work counter.  Only the plan's bins
// [b0, b0 + nb) are swept (nb < 0: all L.B of them); swept bin k is stored
// as bin k of the layout L (L.B >= nb).  The first n_lane of them (n_z = 1
// only) run one lane per centre: for bins with few neighbours per centre.
int scan_chunk(t3_plan *plan, const SortedCatalog *const *cats, const int *order, int n_z,
               const CentreSet &cs, int64_t c0, int n_c, const ChunkLayout &L, float *planes,
               size_t zstride, unsigned long long *npairs, int mode, hipStream_t s, int b0 = 0,
               int nb = -1, int n_lane = 0);
// Leading bins of [b0, b0 + nb) whose expected neighbours per centre are at
// most `most` (uniform density over the non-empty cells of sc); synchronises s.
// Lane-per-centre sums stay in FP32: a sequential sum of k random-phase
// terms has relative rounding error about 2^-25 sqrt(k / 2), below 3e-7 for
// the ~170 terms of the Poisson tail at 128 expected neighbours.
constexpr double kLaneNeighbours = 128.0;
int lane_bins(t3_plan *plan, const SortedCatalog &sc, int b0, int nb, double most, hipStream_t s, int *n_lane);
int fill_int(int *p, int64_t n, int v, hipStream_t s);
int exclusive_scan(int *data, int64_t n, DevBuf &tmp, hipStream_t s);  // in place, n <= 2^30
int zero_doubles(double *p, size_t n, hipStream_t s);
int reserve_contract(t3_plan *plan, const ChunkLayout &L, int n_z);
int contract_slice(const ChunkLayout &L, int n_z);
// Stage 2 for every ordered pair (Z2, Z3) of the n_z plane sets
// (ups_out[pair] += ..., pair = Z2 n_z + Z3).
int contract_chunk(t3_plan *plan, const CentreSet &cs, int64_t c0, int n_c, const ChunkLayout &L,
                   const float *planes, size_t zstride, int n_z, bool jk, double *ups_out,
                   hipStream_t s);
int normalise_resum(t3_plan *plan, const double *ups, int n_sets, int n_z, int n_phi,
                    double *gamma_n, double *gamma_phi, hipStream_t s);
int x_to_centroid(t3_plan *plan, const double *in, int n_sets, int n_phi, const double *theta, double *out,
                  hipStream_t s);
int aperture_stats(t3_plan *plan, const double *gamma_cent, int n_sets, int n_phi, const double *apertures,
                   int n_ap, double *corr, double *stats, hipStream_t s);
int sphere_patch(t3_plan *plan, const t3_sphere_catalog &cat, const t3_patch &p, double theta_max_arcmin,
                 t3_catalog *view, const int32_t **core, int64_t *n_core, hipStream_t s);
int add_doubles(double *dst, const double *src, size_t n, hipStream_t s);
int forward_grid(t3_plan *plan, const t3_catalog &cat, int64_t delta, const int32_t *levels, int method,
                 double *ups_out, int64_t *n_pairs, hipStream_t s);
int level_bbox(GridLevel &lv, const int32_t *px, const int32_t *py, const double *sum, hipStream_t s);
double fft_cost_ms(const t3_plan *plan, const GridLevel &lv);
int fft_level(t3_plan *plan, GridLevel &lv, hipStream_t s);
// Arena bytes of the buffers a forward pass reserves (no-allocation entry
// point): the cell list of n galaxies on grid g (with its scan scratch), the
// stage-1 destination tables, and the stage-2 partial sums of one chunk.
size_t cells_arena_bytes(int64_t n, const CellGrid &g);
size_t scan_dest_entries(const t3_plan *plan);
size_t contract_arena_bytes(const t3_plan *plan, const ChunkLayout &L, int n_z);
int harmonics_export(t3_plan *plan, const CentreSet &cs, const ChunkLayout &L, const float *planes,
                     int64_t c0, int n_c, float *G, float *W, float *D, hipStream_t s);
int normalise_backward(t3_plan *plan, const double *ups, const double *ggam, int n_sets, double *gups,
                       hipStream_t s);
int backward(t3_plan *plan, const t3_catalog &cat, const int32_t *centres, int64_t n_centres,
             const double *grad_ups, float *gg1, float *gg2, float *gw, hipStream_t s);

// Stage timing helpers (no-ops unless the plan has T3_FLAG_TIMING).
int timing_begin_call(t3_plan *plan);
int timing_mark(t3_plan *plan, int stage, bool start, hipStream_t s);
int timing_end_call(t3_plan *plan);  // after the stream has been synchronised

CellGrid choose_grid(const t3_plan *plan, int64_t n_gal);
int choose_chunk(const t3_plan *plan, const ChunkLayout &L);

}  // namespace t3
