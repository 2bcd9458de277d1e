/*
 * t3pcf -- multipole estimator of the shear three-point correlation
 * function on AMD Instinct MI355X (gfx950).
 *
 * Porth, Heydenreich, Burger, Linke & Schneider (2023), "Efficient
 * estimation of third-order shear correlation functions", Sect. 3.
 *
 * Plain C ABI.  All catalog and output pointers are DEVICE pointers unless
 * stated otherwise; streams are hipStream_t passed as void* (NULL = the
 * null stream).  The caller owns every buffer it passes; the library never
 * frees caller memory.  A plan owns its internal workspace (device memory
 * it allocates on first use and keeps until t3_plan_destroy).  A plan must
 * not be used from two host threads or two streams at the same time.
 *
 * Return codes: 0 on success, a negative T3_E* code on failure.  Argument
 * errors are detected before any launch and leave outputs untouched.
 * t3_last_error_message() returns a thread-local description of the most
 * recent failure on the calling thread.  No C++ exception crosses the ABI.
 *
 * Conventions shared by all entry points
 * --------------------------------------
 * Positions are int32 coordinates on a square lattice of step
 * `lattice_unit` arcmin (default 2^-16); they must lie inside the plan's
 * box [box_lo, box_lo + box_size) on both axes.  Separations are therefore
 * exact integers, and a pair (i, j) falls in radial bin b when
 *     (edges[b] / lattice_unit)^2 <= dx^2 + dy^2 < (edges[b+1] / lattice_unit)^2
 * (half-open bins; squares evaluated in IEEE double).
 * Shears g1 + i g2 and weights w are float32.  c_j = w_j (g1_j + i g2_j).
 * phi_ij is the polar angle of theta_j - theta_i.
 *
 * The multipoles follow eq. (Upsilon0_Derivation), eqs. (Upsilon1-3) and
 * eq. (3PCF_Normalization), summed over pairwise-distinct triplets (the
 * j = k terms that the product of two harmonic sums contains are removed
 * unless T3_FLAG_KEEP_JK is set):
 *   Upsilon_{0,n}(b1,b2) = -sum_i c_i  [G_{n-3}(b1)   G_{-n-3}(b2)]
 *   Upsilon_{1,n}        = -sum_i c_i* [G_{n-1}(b1)   G_{-n-1}(b2)]
 *   Upsilon_{2,n}        = -sum_i c_i  [G_{-n-1}(b1)* G_{-n-3}(b2)]
 *   Upsilon_{3,n}        = -sum_i c_i  [G_{n-3}(b1)   G_{n-1}(b2)*]
 *   N_n                  =  sum_i w_i  [W_n(b1)       W_n(b2)*]
 * with G_m(i;b) = sum_j c_j e^{i m phi_ij}, W_m(i;b) = sum_j w_j e^{i m phi_ij}
 * over neighbours j of centre i in bin b (eq. Gn_disc).
 *
 * Multipole output layout ("ups"): complex128 as interleaved (re, im)
 * doubles, row-major, one set = 4 (n_max+1) + (w_max+1) blocks of [B][B]:
 * Upsilon_{mu,n} for mu = 0..3, n = 0..n_max (block mu (n_max+1) + n), then
 * N_n for n = 0..w_max (block 4 (n_max+1) + n).  w_max = n_max, so a set is
 * [5][n_max+1][B][B], unless the plan has T3_FLAG_EDGE_CORRECT, which makes
 * w_max = 2 n_max (the mode-coupling matrix needs N_{l-n}, |l-n| <= 2 n_max).
 * Negative orders follow from the symmetries of Appendix A:
 * Upsilon_{0,-n}(b1,b2) = Upsilon_{0,n}(b2,b1) (same for 1), Upsilon_{2,-n}
 * (b1,b2) = Upsilon_{3,n}(b2,b1), N_{-n}(b1,b2) = N_n(b1,b2)*.
 * Tomographic output: [n_z][n_z][n_z][set] indexed (Z1 centres, Z2 = b1-side
 * neighbours, Z3 = b2-side neighbours), eq. tomoGn; the symmetries map a set
 * to the one with Z2 and Z3 swapped.
 */
#ifndef T3PCF_H
#define T3PCF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define T3_OK 0
#define T3_EINVAL (-1)   /* bad argument (null pointer, bad size, bad bins) */
#define T3_ERANGE (-2)   /* parameter outside the supported range          */
#define T3_ENOMEM (-3)   /* device allocation failed                       */
#define T3_EHIP (-4)     /* a HIP runtime call failed                      */
#define T3_ELATTICE (-5) /* a position lies outside the plan's box          */

/* Precision of the contraction over centres (stage 2).  With 33 to 40   */
/* radial bins, the outputs involving a bin index of 32 or more are      */
/* summed on the vector ALUs in FP32 runs of 16 centres promoted to FP64 */
/* (the FP32 error model) in every precision.                            */
#define T3_PREC_FP32 0    /* FP32 MFMA products, FP32 runs promoted to FP64 */
#define T3_PREC_BF16X3 1  /* x = hi + lo in bf16; hi*hi + hi*lo + lo*hi for  */
                          /* Upsilon_0..3 (for B <= 24 also lo*lo, which    */
                          /* there shares an MFMA with hi*lo), FP32 for the */
                          /* normaliser N_n                                 */
#define T3_PREC_FP16X3 2  /* same in fp16 with power-of-two row scaling     */
#define T3_PREC_BF16X6 3  /* x = hi + mid + lo in bf16 (all 24 FP32 bits);  */
                          /* the six part products of order <= 2; FP32 N_n  */

#define T3_FLAG_KEEP_JK 1u /* keep the j = k terms (the paper's literal sum) */
#define T3_FLAG_TIMING 2u  /* record HIP events around each stage (t3_stage_times); */
                           /* also runs the schedule eagerly (no graph)           */
#define T3_FLAG_NO_GRAPH 4u /* launch the chunk schedule eagerly instead of as one  */
                            /* captured HIP graph                                  */
#define T3_FLAG_EDGE_CORRECT 8u /* forward: N_n up to 2 n_max (stage 1 sums W_m to  */
                                /* 2 n_max); t3_normalise_resum: edge-corrected    */
                                /* Gamma_n (eq. GammaMultipolesWithEC).  No adjoint. */
#define T3_FLAG_NO_LANE 16u /* stage 1: one wavefront per centre for every bin  */
                            /* (default: bins with at most 128 expected         */
                            /* neighbours per centre run one lane per centre)   */
#define T3_FLAG_KEEP_PLANES 32u /* t3_forward over every galaxy of one catalog   */
                                /* keeps the harmonic planes of every chunk      */
                                /* (n x (4 n_max + 2 w_max + 15) x B floats of   */
                                /* device memory, owned by the plan); the next   */
                                /* t3_backward, if no other call has rebuilt the */
                                /* plan's catalog in between and it is given the */
                                /* same catalog (same pointers and n, contents   */
                                /* unchanged), uses them instead of recomputing  */
                                /* stage 1.                                      */
#define T3_FLAG_DETERMINISTIC 64u /* t3_backward: neighbour gradient terms are   */
                                  /* summed as 64-bit fixed-point integers (one  */
                                  /* power-of-two scale per centre chunk, set    */
                                  /* from a bound on that chunk's terms) and the */
                                  /* chunks in FP64 in a fixed order, so the     */
                                  /* gradients are bitwise reproducible.  The    */
                                  /* forward pass is always reproducible.        */

typedef struct {
    int32_t n_bins;        /* 1 <= B <= 64                                   */
    const double *edges;   /* HOST, n_bins + 1 arcmin, strictly increasing,  */
                           /* edges[0] > 0, edges[n_bins] < 512 arcmin       */
    int32_t n_max;         /* largest multipole, 0 <= n_max <= 64            */
    int32_t precision;     /* T3_PREC_*                                      */
    uint32_t flags;        /* T3_FLAG_*                                      */
    double lattice_unit;   /* arcmin per lattice step; 0 -> 2^-16            */
    int32_t box_lo_x;      /* lattice box holding every position             */
    int32_t box_lo_y;
    int64_t box_size;      /* side in lattice steps, > 0, box_lo + size <= 2^31 */
    double cell_arcmin;    /* spatial-hash cell side; 0 -> automatic          */
    int32_t chunk_centres; /* centres per stage-1/stage-2 chunk; 0 -> auto    */
                           /* (about 1 GiB of planes per catalog, at most     */
                           /* 65,536 centres; 4 GiB and 262,144 for n_max 40  */
                           /* and 48)                                          */
    int32_t scan_mode;     /* stage-1 launch: 0 one wavefront per centre, one */
                           /* launch per neighbour catalog; 1 one persistent  */
                           /* launch over all (centre, catalog) tasks with a  */
                           /* work queue                                      */
    int64_t max_workspace_bytes; /* >= 0; 0 = no limit.  Upper bound on the    */
                           /* device memory the plan holds at any time (the   */
                           /* sum of its internal buffers, checked before     */
                           /* each allocation).  A call that would exceed it  */
                           /* returns T3_ENOMEM without allocating; see       */
                           /* t3_workspace_bytes.                             */
    double lane_neighbours; /* stage-1 bins with at most this many expected   */
                           /* neighbours per centre run one lane per centre;  */
                           /* 0 -> 128 (the bound of the FP32 lane sums);     */
                           /* in (0, 128]; T3_FLAG_NO_LANE turns the lane     */
                           /* kernel off                                      */
    int32_t tile_mode;     /* stage-2 tiles for B <= 24: 0 real-embedded      */
                           /* 16 x 16 (2B x 2B real product), 1 complex       */
                           /* 32 x 32 (as for B > 24)                         */
} t3_params;

typedef struct {
    int64_t n;            /* number of galaxies (>= 0)                       */
    const int32_t *x;     /* DEVICE [n] lattice coordinates                  */
    const int32_t *y;     /* DEVICE [n]                                      */
    const float *g1;      /* DEVICE [n] shear, Cartesian frame               */
    const float *g2;      /* DEVICE [n]                                      */
    const float *w;       /* DEVICE [n] weights                              */
} t3_catalog;

/* A catalog on the sphere (Appendix B). */
typedef struct {
    int64_t n;            /* number of galaxies (>= 0)                       */
    const double *ra;     /* DEVICE [n] right ascension, degrees             */
    const double *dec;    /* DEVICE [n] declination, degrees, |dec| < 89     */
    const float *g1;      /* DEVICE [n] shear in the local (east, north)     */
    const float *g2;      /* DEVICE [n]   frame, angles from east to north   */
    const float *w;       /* DEVICE [n] weights                              */
} t3_sphere_catalog;

/* A patch: the RA/Dec rectangle [ra_lo, ra_hi) x [dec_lo, dec_hi), degrees. */
typedef struct {
    double ra_lo, ra_hi, dec_lo, dec_hi;
} t3_patch;

typedef struct t3_plan t3_plan;

/* Routes of t3_forward_grid for a grid level. */
#define T3_GRID_AUTO 0
#define T3_GRID_DIRECT 1
#define T3_GRID_FFT 2

/* Create a plan: validates parameters, derives squared edges and the
 * cell grid, and picks the stage-1 kernel variant for n_max.  No device
 * memory is allocated here.  *out is set only on success. */
int t3_plan_create(const t3_params *params, t3_plan **out);

/* Release the plan and its workspace (synchronises the device first). */
void t3_plan_destroy(t3_plan *plan);

/* Graph statistics of the plan (HOST outputs, optional): how many times the
 * chunk schedule of t3_forward / t3_forward_tomo was captured into a HIP
 * graph and how many times a captured graph was launched.  A schedule is
 * captured once per key -- the launch shapes and every address and value
 * its kernels take (catalog and centre-set sizes, cell grid, plan buffers,
 * lane-bin split, launch mode, precision, flags, device) -- and replayed
 * while the key is unchanged; the cell lists and centre sets it reads are
 * rebuilt in place before each launch and its output is copied to the
 * caller's, so new data of the same geometry, written anywhere, replays the
 * same graph. */
int t3_graph_stats(const t3_plan *plan, int64_t *captures, int64_t *launches);

/* Device memory the plan currently holds (in_use, HOST, optional) and the
 * largest amount it has held (peak, HOST, optional), in bytes; never more
 * than params.max_workspace_bytes when that is set.  Buffers grow on demand
 * and are kept until t3_plan_destroy, so the peak of a fresh plan after one
 * call is what that call needs: a plan created with that limit runs the
 * same call without T3_ENOMEM.  A call refused for the limit returns
 * T3_ENOMEM before the allocation it would need; t3_forward,
 * t3_forward_tomo and t3_backward then have launched nothing that writes
 * their outputs. */
int t3_workspace_bytes(const t3_plan *plan, int64_t *in_use, int64_t *peak);

/* Non-tomographic forward pass (Sect. 3.1, eq. Upsilon0_Derivation).
 * cat:       the neighbour catalog; centres are drawn from the same catalog.
 * centres:   DEVICE int32 [n_centres] indices into cat.  n_centres < 0 selects
 *            every galaxy of cat (centres must then be NULL); n_centres == 0
 *            selects none (centres may be NULL) and yields zero multipoles.
 * ups_out:   DEVICE double [5][n_max+1][B][B][2]; overwritten.
 * n_pairs:   HOST int64*, optional: number of in-range ordered
 *            (centre, neighbour) pairs visited.
 * The call enqueues its work on `stream` and returns after the last
 * kernel completes (it synchronises the stream once, to check the
 * lattice bounds of the catalog). */
int t3_forward(t3_plan *plan, const t3_catalog *cat, const int32_t *centres,
               int64_t n_centres, double *ups_out, int64_t *n_pairs, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * t3_forward pass -- same arguments, same results -- with every internal
 * buffer (cell list, centre set, stage-1 planes, stage-2 partial sums,
 * counters, destination tables) carved from one static device array of
 * 256 MiB that the library holds on each GPU it runs on until the process
 * ends.  It calls no hipMalloc, hipFree or other allocating routine and
 * never touches the plan's own workspace; it always launches eagerly (no
 * graph, no timing events).  Before any launch it picks the largest chunk of
 * centres (a multiple of 256, at most t3_forward's) whose buffers fit the
 * array, and returns T3_ENOMEM with a message stating the bytes needed if
 * even chunks of 256 centres do not fit (the cell list and centre set take
 * about 57 bytes per galaxy: roughly 4.5 million galaxies, all of them
 * centres, at n_max 30 and 20 bins).
 * Every call on one GPU uses that GPU's array: calls that overlap in time
 * on one GPU (other threads, other streams) race and must be serialised by
 * the caller.  The buffers are cleared by the call itself where it needs
 * zeros, as in t3_forward. */
int t3_forward_noalloc(t3_plan *plan, const t3_catalog *cat, const int32_t *centres,
                       int64_t n_centres, double *ups_out, int64_t *n_pairs, void *stream);

/* Tomographic forward pass over all ordered bin triples (Sect. 3.5,
 * eq. tomoGn).  cats: HOST array of n_z catalogs (device arrays).
 * centres: HOST array of n_z DEVICE pointers, or NULL for every galaxy of
 * every bin; n_centres: HOST array of n_z counts with the t3_forward
 * convention per bin (a count < 0 selects every galaxy of that bin and
 * needs a NULL pointer).  ups_out: DEVICE [n_z][n_z][n_z][5][n_max+1][B][B][2].
 * The normaliser is N_n(Z1,Z2,Z3) = sum_{i in Z1} w_i W^{(Z2)}_n W^{(Z3)*}_n;
 * j = k terms are removed only for Z2 == Z3.  1 <= n_z <= 8. */
int t3_forward_tomo(t3_plan *plan, const t3_catalog *cats, int32_t n_z,
                    const int32_t *const *centres, const int64_t *n_centres,
                    double *ups_out, int64_t *n_pairs, void *stream);

/* Multipoles of a curved-sky catalog from flat patches (Appendix B,
 * eq. PatchGamma): for every patch, the sphere is rotated so that the patch
 * centre lies at (RA, Dec) = (0, 0), shears are rotated by the change of
 * reference direction (gamma' = gamma e^{-2 i psi}, psi the angle from the
 * local north to the image of the original north, towards east), positions
 * are mapped by the sinusoidal projection x = lambda cos(beta), y = beta
 * (arcmin, x east, y north) onto the plan's lattice, and the flat estimator
 * runs with the patch's core galaxies as centres against every galaxy of
 * the patch extended by theta_max (theta_max / cos(Dec) in RA); the results
 * are summed over patches.  Patches whose cores tile the footprint count
 * every centre once.
 * The plan's box must hold every projected extended patch, centred on 0
 * (e.g. box_lo = -box_size / 2); positions outside it give T3_ELATTICE.
 * patches: HOST [n_patches], each side <= 30 degrees; theta_max_arcmin must
 * be >= the plan's largest bin edge.  ups_out: t3_forward layout.  n_pairs:
 * HOST, the ordered pairs summed over patches.  Synchronises the stream
 * (patch sizes are read back to size the flat catalogs). */
int t3_forward_sphere(t3_plan *plan, const t3_sphere_catalog *cat, const t3_patch *patches,
                      int32_t n_patches, double theta_max_arcmin, double *ups_out, int64_t *n_pairs,
                      void *stream);

/* Combined discrete / grid-based multipoles (Sect. 3.2-3.3, eqs.
 * UpsilonmuGrid and CombinedEstimatorRegridding; Appendix A).
 * levels: HOST int32 [B], non-decreasing: 0 = discrete bin (galaxy pairs);
 *   l = 1..8 = grid bin on square pixels of side delta * 2^(l-1) lattice
 *   steps anchored at the plan box corner (nested resolutions).  A grid
 *   pixel carries the sums of w gamma and w of its galaxies (FP64, rounded
 *   once to FP32) at its corner; G_m, W_m of a grid bin are the harmonic
 *   sums over non-empty pixels around each non-empty pixel (the
 *   convolution of the gridded values with the bin kernels).  A block
 *   (b1, b2) is the sum over galaxies of the centre factor times the
 *   harmonics, those of a grid bin taken at the galaxy's pixel: for two
 *   bins of one grid level this is the grid estimator over pixels; across
 *   levels it is the finer side's w gamma G summed into the coarser pixels
 *   and contracted with the coarse harmonics.  Diagonal blocks of a grid
 *   bin remove the degenerate pairs of one neighbour pixel (the discrete
 *   estimator's j = k reading, applied to the pixel catalog) unless
 *   T3_FLAG_KEEP_JK.
 * delta: base pixel side in lattice steps, >= 1; for every level used,
 *   side <= box_size and box_size / side <= 8192.  Every galaxy is a centre.
 * method: how a level's harmonics are computed: T3_GRID_DIRECT (pair sums
 *   over the non-empty pixels), T3_GRID_FFT (FFT convolution on a dense
 *   grid of the occupied pixels, sides products of 2, 3, 5 up to 8192; FP32
 *   transforms, whose rounding scales with the grid's largest values) or
 *   T3_GRID_AUTO (a cost model picks per level; levels whose heaviest
 *   pixel exceeds 100 times the mean pixel weight keep the pair sums).
 * ups_out: t3_forward layout.  n_pairs: HOST, optional: galaxy pairs of the
 *   discrete bins plus pixel pairs of the levels summed pairwise (FFT
 *   levels add none).  Synchronises the stream (pixel counts and extents
 *   are read back to size the pixel catalogs and grids). */
int t3_forward_grid(t3_plan *plan, const t3_catalog *cat, int64_t delta, const int32_t *levels,
                    int32_t method, double *ups_out, int64_t *n_pairs, void *stream);

/* Stage 1 alone, for inspection: the harmonic sums of eq. (Gn_disc) for
 * the given centres against the neighbour catalog.
 * centres: DEVICE int32 [n_centres] indices into cat.
 * G_out:   DEVICE float [n_centres][B][2 n_max + 3][2], orders
 *          m = -n_max-3 .. n_max-1;
 * W_out:   DEVICE float [n_centres][B][n_max + 1][2], orders m = 0..n_max;
 * D_out:   DEVICE float [n_centres][B][4][2]: sum c_j^2 e^{-6i phi},
 *          sum c_j^2 e^{-2i phi}, sum |c_j|^2 e^{-2i phi}, sum w_j^2. */
int t3_harmonics(t3_plan *plan, const t3_catalog *cat, const int32_t *centres,
                 int64_t n_centres, float *G_out, float *W_out, float *D_out,
                 void *stream);

/* Normalisation and resummation in FP64 (Sect. 3.4, eq. Gamma0_binned).
 * ups:       DEVICE double, n_sets sets in the t3_forward output layout
 *            (n_sets = 1, or n_z^3 for tomography).
 * gamma_n:   DEVICE double [n_sets][4][n_max+1][B][B][2]:
 *            Gamma_{mu,n} = Upsilon_{mu,n} / N_0 (0 where N_0 == 0), or, for
 *            a plan with T3_FLAG_EDGE_CORRECT, the edge-corrected multipoles
 *            of eqs. (ModeCoupling), (GammaMultipolesWithEC): for every bin
 *            pair the (2 n_max + 1)-dimensional Hermitian Toeplitz system
 *            sum_{|n|<=n_max} N_{l-n} Gamma_{mu,n} = Upsilon_{mu,l},
 *            |l| <= n_max, solved in FP64 by the Levinson recursion (0 where
 *            N_0 == 0; a numerically singular system yields non-finite
 *            entries for that bin pair only, with no error code).
 * gamma_phi: DEVICE double [n_sets][4][B][B][n_phi][2] or NULL:
 *            sum_{|n|<=n_max} Gamma_{mu,n} s_n(Phi_k), with angular bins
 *            Phi_k = [2 pi k / n_phi, 2 pi (k+1) / n_phi) and
 *            s_n = (e^{i n Phi_up} - e^{i n Phi_lo}) / (i n dPhi), s_0 = 1.
 *            Negative n come from the symmetries (tomographic sets use the
 *            set with Z2 and Z3 swapped).  1 <= n_phi <= 4096. */
int t3_normalise_resum(t3_plan *plan, const double *ups, int32_t n_sets,
                       int32_t n_phi, double *gamma_n, double *gamma_phi,
                       void *stream);

/* x -> centroid projection of the resummed natural components (Sect. 2.3,
 * eqs. X2Centroid0-X2Centroid3 with the rotation factors written in
 * theta_1, theta_2 and phi).  The pointwise conversion is evaluated at one
 * representative triangle per bin: radii theta[b1], theta[b2] and the
 * angular-bin centre phi_k = 2 pi (k + 1/2) / n_phi.
 * gamma_phi_x:    DEVICE double [n_sets][4][B][B][n_phi][2] (t3_normalise_resum);
 * theta:          HOST double [B] arcmin, or NULL for the centres
 *                 (edges[b] + edges[b+1]) / 2 of the plan's bins;
 * gamma_phi_cent: DEVICE double, same layout (may alias gamma_phi_x).
 * Where a conversion factor's denominator is exactly zero (a collinear
 * configuration in which a median direction vanishes) the output is 0. */
int t3_x_to_centroid(t3_plan *plan, const double *gamma_phi_x, int32_t n_sets, int32_t n_phi,
                     const double *theta, double *gamma_phi_cent, void *stream);

/* Third-order aperture statistics from the centroid-projected 3PCF
 * (Sect. 4, Appendix C), FP64: the four complex correlators
 *   <M^3>, <M* M^2>, <M M* M>, <M^2 M*>  (theta_1, theta_2, theta_3)
 * = int d vartheta_1 d vartheta_2 d phi Gamma_mu^cent F_mu (eqs. MFrom3pcfTheory,
 * MFrom3pcfTheoryb; exponential filter, eq. CrittendenQ) by the midpoint rule
 * on the plan's radial bins (centres and widths in arcmin) and the n_phi
 * angular bins, and the eight real statistics of eqs. MapTrafo8_1-8.
 * Filter of component mu: the printed F_1 with its distinguished index at
 * vertex mu (the component conjugated at vertex mu); F_0 as printed.
 * gamma_phi_cent: DEVICE double [n_sets][4][B][B][n_phi][2] (t3_x_to_centroid);
 * apertures:      HOST double [n_ap][3] radii in arcmin (> 0), 1 <= n_ap <= 65535;
 * corr_out:       DEVICE double [n_sets][n_ap][4][2];
 * stats_out:      DEVICE double [n_sets][n_ap][8] or NULL: <Map^3>, <Mx Map^2>,
 *                 <Map Mx Map>, <Map^2 Mx>, <Map Mx^2>, <Mx Map Mx>, <Mx^2 Map>, <Mx^3>. */
int t3_aperture_stats(t3_plan *plan, const double *gamma_phi_cent, int32_t n_sets, int32_t n_phi,
                      const double *apertures, int32_t n_ap, double *corr_out, double *stats_out,
                      void *stream);

/* Reverse of the normalisation Gamma_{mu,n} = Upsilon_{mu,n} / N_0 (mu < 4).
 * ups: DEVICE [n_sets][5][n_max+1][B][B][2] forward multipoles;
 * grad_gamma_n: DEVICE [n_sets][4][n_max+1][B][B][2] holding dL/dRe and
 * dL/dIm of each Gamma entry; grad_ups (DEVICE, layout of ups, overwritten)
 * receives dL/dUpsilon for mu < 4 and dL/dN_0 in the real part of the
 * (mu = 4, n = 0) entries (0 elsewhere).  Bin pairs with N_0 = 0 pass no
 * gradient. */
/* (Not available for plans with T3_FLAG_EDGE_CORRECT: T3_EINVAL.) */
int t3_normalise_backward(t3_plan *plan, const double *ups, int32_t n_sets,
                          const double *grad_gamma_n, double *grad_ups, void *stream);

/* Adjoint of the non-tomographic forward pass (hand-written; the harmonic
 * sums are recomputed, or, with T3_FLAG_KEEP_PLANES and every galaxy as a
 * centre, taken from the planes the last t3_forward over all centres kept
 * when it ran over this same catalog and no call rebuilt the plan's
 * catalog since).  The multilinear structure of eq. (Upsilon0_Derivation):
 * each galaxy enters as a centre factor and, linearly, in the harmonic sums
 * of its neighbours.
 * centres, n_centres: the centre set of the forward pass, with the
 *   t3_forward convention (n_centres < 0: every galaxy, centres NULL;
 *   0: none, the gradients are 0).  Gradients still reach every galaxy
 *   that is a neighbour of a listed centre (a centre shard of the forward
 *   pass has the adjoint of that shard).
 * grad_ups: DEVICE, layout of the t3_forward output, holding dL/dRe and
 * dL/dIm of every Upsilon_{mu,n} and N_n entry (n >= 0).
 * grad_g1, grad_g2, grad_w: DEVICE float [cat->n], overwritten with dL/dg1,
 * dL/dg2, dL/dw of every galaxy.  Neighbour contributions are summed with
 * FP32 atomics, so results can differ between calls at rounding level,
 * unless the plan has T3_FLAG_DETERMINISTIC (then they are bitwise
 * reproducible for a centre list without repeated indices).
 * Synchronises the stream before returning. */
/* (Not available for plans with T3_FLAG_EDGE_CORRECT: T3_EINVAL.  The
 * per-centre coefficient step holds B (3 n_max + 8) complex floats in LDS,
 * at most 101 KiB for B = n_max = 64.) */
int t3_backward(t3_plan *plan, const t3_catalog *cat, const int32_t *centres, int64_t n_centres,
                const double *grad_ups, float *grad_g1, float *grad_g2, float *grad_w, void *stream);

/* Autotuner (Sect. 3.5: the batched tomographic evaluation of eq. tomoGn
 * is tuned once per problem shape and replayed).  Times the forward pass of
 * this plan on a deterministic sample of at most sample_per_bin centres of
 * every catalog (cats: HOST array of n_z catalogs, as for t3_forward_tomo)
 * and keeps the fastest settings in the plan, one coordinate at a time from
 * the best so far: cell size 0.6x / 1x / 1.6x the automatic one with both
 * stage-1 launch modes; the stage-1 lane-kernel threshold (0, 64 or 128
 * expected neighbours per centre; none above 128, the bound of the FP32
 * lane sums; skipped with T3_FLAG_NO_LANE); for B <= 24 the stage-2 tile
 * shape (real-embedded 16 x 16 or complex 32 x 32 MFMA tiles); and, when
 * the plan's chunk capacity is automatic, 1, 1/2 or 1/4 of the automatic
 * capacity (a capacity at or above the sample's centres per catalog runs
 * the sample as one chunk, like the automatic one, and is not tried).
 * Each candidate is timed twice (best kept); ties keep the
 * earlier one.  The choice is cached per process, keyed by (n_bins, n_max,
 * n_z, precision, catalog-size class, box, sample_per_bin, requested chunk
 * capacity); a cached choice is applied without timing.  best_ms (HOST,
 * optional) receives the best sample time (0 for a cached choice).
 * Synchronises the stream. */
int t3_autotune(t3_plan *plan, const t3_catalog *cats, int32_t n_z, int64_t sample_per_bin,
                double *best_ms, void *stream);

/* The plan's current tunable settings (each output HOST and optional):
 * cell side in arcmin, stage-1 launch mode (0 one wavefront per task,
 * 1 persistent work queue), lane-kernel threshold in expected neighbours,
 * stage-2 tile shape for B <= 24 (0 real-embedded 16 x 16, 1 complex
 * 32 x 32) and requested chunk capacity in centres (0: automatic). */
int t3_plan_settings(const t3_plan *plan, double *cell_arcmin, int32_t *scan_mode, double *lane_neighbours,
                     int32_t *tile_mode, int32_t *chunk_centres);

/* Stage timings of the most recent t3_forward / t3_forward_tomo call of a
 * plan created with T3_FLAG_TIMING, from HIP events recorded on the
 * caller's stream around each launch group.  ms[4] (HOST) receives the
 * summed durations in milliseconds of: [0] cell-list build and centre
 * gather, [1] stage 1 (neighbour scan, all chunks), [2] stage 2 (contraction
 * over centres incl. j = k sums and FP64 reduction), [3] unused (0);
 * launches[4] (HOST, optional) the number of stage-1 / stage-2 kernel
 * launches timed.  Returns T3_EINVAL if the plan has no timing flag. */
int t3_stage_times(const t3_plan *plan, double *ms, int64_t *launches);

/* Static description of an error code. */
const char *t3_error_string(int code);

/* Thread-local message describing the last failure on this thread. */
const char *t3_last_error_message(void);

/* Library version string. */
const char *t3_version(void);

#ifdef __cplusplus
}
#endif

#endif /* T3PCF_H */
