/*
 * flowfields.h -- C ABI of the MI355X (gfx950) Flow Fields hot path.
 *
 * Method: Bailer, Taetz, Stricker, "Flow Fields: Dense Correspondence Fields
 * for Highly Accurate Large Displacement Optical Flow Estimation" (journal
 * version).  Two images in, a dense displacement field F(p) = M(p) - p out
 * (Sec. 3, notation), for both directions, plus the forward-backward
 * consistency masks (Sec. 3.7).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Every pointer argument is a DEVICE pointer owned by the caller, unless
 *    its comment says "host".  The library never allocates, frees or
 *    synchronises; each call only enqueues kernels on `stream` (a
 *    hipStream_t passed as void*, NULL = the default stream) and returns.
 *  * Images: uint8 [H][W], row-major, pitch W.
 *  * Descriptors: uint8 [H][W][16], row-major, 16 bytes per pixel.
 *  * Level grid of scale n: ceil(W/n) x ceil(H/n) cells, row-major; cell
 *    (i, j) is the full-resolution pixel (i*n, j*n).  Flows: int16 [cells][2]
 *    = (dx, dy) in full-resolution pixels.  Costs: uint32 [cells]; the value
 *    0xFFFFFFFF marks an UNSET cell, whose flow is (0, 0).
 *  * n_evals: optional (may be NULL) device uint64 counter; every patch-cost
 *    evaluation the call performs adds 1 to it (atomically).
 *  * Argument errors (NULL required pointer, W or H outside [1, 32767],
 *    levels outside [1, 7], iters outside [1, 64], radius outside [0, 7],
 *    n not a power of two in [1, 64], too small a workspace) return
 *    FF_ERR_ARG / FF_ERR_WORKSPACE before anything is enqueued.  A failed
 *    launch returns FF_ERR_LAUNCH.  Faults inside kernels surface at the
 *    caller's next synchronisation of `stream`.
 *  * Calls are re-entrant and keep no mutable global state (launch tables
 *    come with each call, ff_tuning); calls on different streams or threads
 *    may overlap when they write disjoint buffers.  The one exception is
 *    ff_region_filter_noalloc (one static scratch array per GPU).
 */
#ifndef FLOWFIELDS_H
#define FLOWFIELDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FF_OK = 0,
    FF_ERR_ARG = 1,
    FF_ERR_LAUNCH = 2,
    FF_ERR_WORKSPACE = 3,
    FF_ERR_UNSUPPORTED = 4
} ff_status;

#define FF_UNSET_COST 0xFFFFFFFFu

/* Launch tables of the temporally blocked level kernels (speed only: results
 * never depend on them), indexed by scale log2 n = 0..6.  variant: kernel
 * variant of the byte-descriptor path, in [0, ff_level_variant_count()) (the
 * last index selects the step-wise schedule: one launch per step over all
 * cells); passes: most propagation steps per blocked launch, 0 = as many as
 * the variant's halo allows, in [0, 64]; variant_f32 / passes_f32: the same
 * for the learned float features (variant_f32 in
 * [0, ff_level_variant_count_f32())).  Host memory, read during the call
 * only; the library keeps no mutable table, so calls with different tables
 * may run concurrently. */
typedef struct {
    int32_t variant[7];
    int32_t passes[7];
    int32_t variant_f32[7];
    int32_t passes_f32[7];
} ff_tuning;

/* Schedule of one Flow Field computation (Sec. 3.1, 3.2; parameters Sec. 4.1). */
typedef struct {
    int32_t levels;  /* L: scales n = 2^(L-1), ..., 2, 1 (the paper's k = L-1) */
    int32_t iters;   /* T: propagation steps per scale; T-1 random-search steps sit between them */
    int32_t radius;  /* r: patch of (2r+1)^2 positions, subsampled by n (Eq. 3) */
    int32_t R_num;   /* random-search distance R = R_num / R_den; at scale n the */
    int32_t R_den;   /*   integer offset bound is R_n = floor(R_num * n / R_den) */
    float eps;       /* consistency threshold: keep iff |F(p) + F_b(p + F(p))| < eps */
    uint64_t seed;   /* key of the counter-based random-search generator */
    /* Flow Fields+ (Sec. 3.3): plus_iters = P > 0 runs, on every scale, P
     * propagation steps whose random searches use R_n^+ = floor(Rp_num * n /
     * R_den) before the T steps at R_n; random searches sit only between two
     * steps of the same group, and the step index t (direction t mod 4,
     * generator counter) runs on over both groups.  P = 0: the original
     * schedule.  Flow Fields+ Fast (Sec. 3.4): fine_iters > 0 makes the finest
     * scale run only fine_iters steps at R_n.  Limits: P + T <= 64,
     * fine_iters <= 64, Rp_num in [0, 2^20]. */
    int32_t plus_iters;
    int32_t Rp_num;
    int32_t fine_iters;
    /* Subpixel random search (Sec. 3.1: offsets with subpixel accuracy, the
     * target patch's colours by bilinear interpolation): 0 = integer flows;
     * 3 = every flow, random-search offset (uniform on [-R_n, R_n]^2 in
     * steps of 1/8 px) and the consistency threshold in units of 1/8 pixel,
     * image b's descriptors bilinearly interpolated at the target with
     * weights in 1/64, costs 64 times Eq. 3 (exact integers).  Requires
     * W, H <= 4095 (int16 flows); other values FF_ERR_ARG.  Runs on the
     * per-step kernels; ff_flow_fields_batched and ff_flow_fields_f32
     * return FF_ERR_UNSUPPORTED for it. */
    int32_t subpixel;
    /* host, nullable: launch tables of this call (NULL: the built-in table,
     * see ff_default_tuning); an entry out of range is FF_ERR_ARG. */
    const ff_tuning *tuning;
    /* Seed candidates (Sec. 3.1: the l entries of a kd-tree leaf, ranked by
     * matching error, Eq. 1 / Eq. 4; l = 8 in Sec. 4.1): 0 or 1 = the exact
     * nearest neighbour alone; 2..8 = the nn_l nearest pixels by (squared
     * descriptor distance, linear index), of which the one with the lowest
     * E_nc wins (the earlier rank on equal cost); every candidate counts one
     * evaluation.  Other values FF_ERR_ARG. */
    int32_t nn_l;
    /* Propagation order (Sec. 3.1: a cell after its left and upper
     * neighbours): 0 = two checkerboard half-sweeps per step; 1 = the serial
     * order of each step's direction, computed exactly by anti-diagonal
     * wavefronts (ff_propagate_raster; integer costs; a long chain of
     * dependent launches, far slower than the checkerboard).  Other values
     * FF_ERR_ARG.  ff_flow_fields_batched and ff_flow_fields_f32 return
     * FF_ERR_UNSUPPORTED for nn_l > 1 or raster = 1. */
    int32_t raster;
    /* Flow Fields+ Fast x2 (Sec. 3.4): 1 = the finest scale is not run; the
     * scale-2 grid is the last one (its step count is fine_iters when that
     * is > 0), the NN seed searches only the pixels with even x and y (one
     * pixel of every 2x2 region), and ff_flow_fields returns fields, costs
     * and masks on the grid of scale 2 ([ceil(H/2)][ceil(W/2)] cells, cell
     * (i, j) = pixel (2i, 2j), flows in pixels), checked with
     * ff_consistency_filter_grid.  Needs levels >= 2 and subpixel = 0
     * (FF_ERR_ARG otherwise); the batched and learned calls return
     * FF_ERR_UNSUPPORTED. */
    int32_t fast_x2;
    /* Sub-scales (Sec. 3.3, table of scales and sub-scales): 1 = every scale
     * n >= 2 below the coarsest is preceded by a stage on the same grid
     * whose patch spacing, blur and random-search distances follow the
     * sub-scale m = 3n/2 (for L = 4: (8,8) (4,6) (4,4) (2,3) (2,2) (1,1));
     * the step to the next stage on one grid keeps the flows and evaluates
     * the costs at the new patch scale (ff_rescore_level); every stage runs
     * the plus_iters / iters steps (fine_iters on the last one); the
     * generator's level field is log2 n, plus 16 on a sub-scale stage.  Runs
     * on the temporally blocked kernels at radius 3 (the sub-scale stages on
     * descriptor-quad kernels reading both images' maps), else on the
     * per-step kernels.  Not with fast_x2 (FF_ERR_ARG); ff_run_level,
     * the batched and the learned calls return FF_ERR_UNSUPPORTED. */
    int32_t subscales;
} ff_params;

/* The built-in launch tables (host): written to *out. */
void ff_default_tuning(ff_tuning *out);

/* Library version (host). */
int ff_version(void);

/* Human-readable name of a status (host, static string). */
const char *ff_status_str(ff_status s);

/* Scale-space image I^n and per-pixel descriptors of scale n (Sec. 3.2 scale
 * spaces, Sec. 3.6 low-pass and border condition).
 * blurred[y][x] = round-half-up mean of img over the (2h+1)^2 window,
 * h = max(1, n/2), replicate border; desc[y][x][4*gy+gx] =
 * blurred[clamp(y + n*(2gy-3))][clamp(x + n*(2gx-3))], gx, gy in 0..3.
 * img: [H][W]; blurred: [H][W] output; hsum: [H][W] uint16 scratch
 * (required; this single-image path keeps its row sums in LDS and leaves it
 * untouched);
 * desc: the descriptor MAP of scale n (output, ff_descriptor_map_bytes);
 * desc_rowmajor (nullable): the same descriptors as plain [H][W][16] (the
 * input of ff_init_nn's nearest-neighbour search); wform (nullable): the
 * weight-class row map of scale n (output, ff_wform_map_bytes), which the
 * level kernels with weight-class evaluations read.
 * Descriptor map layout (every entry point that takes a "descriptor map"
 * expects it): P = 4n, Wp = W + 2P; Hp = H + 2P rows of Wp 16-byte entries;
 * entry (y + P, col(x + P)) holds desc[clamp(y)][clamp(x)] for x in
 * [-P, W + P), y in [-P, H + P) (replicated border), where inside a row the
 * pixels are grouped by phase, col(c) = (c mod n)*floor(Wp/n) +
 * min(c mod n, Wp mod n) + floor(c/n): the samples x + n*u of a patch row
 * are adjacent and a patch of radius up to 4 around any in-image pixel needs no
 * clamping.  A scale that is not a power of two (a sub-scale, Sec. 3.3)
 * keeps the pixels of a row in image order, col(c) = c.  1 <= n <= 64. */
ff_status ff_descriptors(const uint8_t *img, int32_t W, int32_t H, int32_t n, uint16_t *hsum,
                         uint8_t *blurred, uint8_t *desc, uint8_t *desc_rowmajor, uint8_t *wform, void *stream);

/* Bytes of a descriptor map of scale n (host): (W + 8n) * (H + 8n) * 16;
 * 0 for invalid sizes. */
size_t ff_descriptor_map_bytes(int32_t W, int32_t H, int32_t n);

/* Weight-class row map of scale n (the cost of Eq. 3 written on the
 * blurred image I^n): W * (H + 6n) entries of 16 bytes, entry (y + 3n) * W +
 * x for y in [-3n, H + 3n) holding the 13 samples I^n(clamp(x + n a),
 * clamp(y)), a = -6..6, grouped by how often the subsampled patch of a
 * radius-3 cost counts them: bytes 0-3 a = -6, -5, 5, 6 (once); bytes 4-7
 * a = -4, -3, 3, 4 (twice); bytes 8-11 a = -2, -1, 1, 2 (three times); byte
 * 12 a = 0 (four times); bytes 13-15 zero.  For a pixel and a target both
 * at least 3n inside the image, E_n = sum over b = -6..6 of w(b) times the
 * weighted byte SADs of rows y + n b, w = 1,1,2,2,3,3,4,3,3,2,2,1,1: each
 * descriptor byte is one blurred sample, so the 784 byte differences are
 * 169 samples with multiplicities w(a) w(b).  Bytes (host); 0 for invalid
 * sizes. */
size_t ff_wform_map_bytes(int32_t W, int32_t H, int32_t n);

/* Initial flow of the coarsest scale nc (Sec. 3.1 initialisation, Eq. 1;
 * Sec. 3.2 Eq. 4 with a single candidate): for every cell p of the grid of
 * scale nc, the exact nearest neighbour q over ALL pixels of image b of the
 * level-1 descriptor of p in image a under squared L2 distance (ties: the
 * smallest q.y*W + q.x), computed on int8 matrix cores; then F(p) = q - p and
 * cost(p) = E_nc(p, F(p)) with the scale-nc descriptors.
 * desc_a1, desc_b1: level-1 descriptors, plain [H][W][16] (desc_rowmajor of
 * ff_descriptors); desc_ac, desc_bc: descriptor maps of scale nc;
 * nb_scratch: int32 [ceil(W*H/32)*32] scratch;
 * nn_key: uint64 [cells] output, (squared distance << 32) | q;
 * flow, cost: grid of scale nc, outputs.  W * H must stay below 2^27 (the
 * search addresses the descriptors with 32-bit offsets): FF_ERR_ARG
 * otherwise, as for ff_flow_fields, ff_flow_fields_f32 and the batch calls,
 * whose workspace-size queries return 0 for such sizes. */
ff_status ff_init_nn(const uint8_t *desc_a1, const uint8_t *desc_b1, const uint8_t *desc_ac,
                     const uint8_t *desc_bc, int32_t W, int32_t H, int32_t nc, int32_t radius,
                     int32_t *nb_scratch, uint64_t *nn_key, int16_t *flow, uint32_t *cost,
                     uint64_t *n_evals, void *stream);

/* Scratch bytes of ff_nn_topl and ff_init_nn_l for a grid of scale nc
 * (host; 0 for invalid sizes). */
size_t ff_nn_topl_scratch_bytes(int32_t W, int32_t H, int32_t nc);

/* The l nearest pixels of image b of every cell p of the grid of scale nc
 * (the candidate set of Sec. 3.1, a kd-tree leaf of size l, read as the l
 * nearest neighbours): ranked by (squared L2 distance of the level-1
 * descriptors, q.y*W + q.x).  cand: uint64 [cells][l] output, entry
 * (distance << 32) | q, ~0 where the image has fewer than l pixels.
 * Computed exactly as l passes of ff_init_nn's matrix-core search, pass k
 * leaving out every pixel whose (distance, index) is at most pass k-1's
 * result.  desc_a1, desc_b1: as for ff_init_nn;
 * nb_scratch: as for ff_init_nn; scratch: device, ff_nn_topl_scratch_bytes
 * (FF_ERR_WORKSPACE if smaller); 1 <= l <= 8. */
ff_status ff_nn_topl(const uint8_t *desc_a1, const uint8_t *desc_b1, int32_t W, int32_t H, int32_t nc, int32_t l,
                     int32_t *nb_scratch, void *scratch, size_t scratch_bytes, uint64_t *cand, void *stream);

/* ff_init_nn with nn_l candidates per cell (Eq. 1 / Eq. 4): the seed of
 * cell p is the candidate q of ff_nn_topl with the lowest E_nc(p, q - p),
 * the earlier rank on equal cost; n_evals grows by the number of
 * candidates.  nn_key receives the winner in ff_init_nn's format.  nn_l 0
 * or 1: ff_init_nn (scratch unused); 2..8: scratch of
 * ff_nn_topl_scratch_bytes bytes. */
ff_status ff_init_nn_l(const uint8_t *desc_a1, const uint8_t *desc_b1, const uint8_t *desc_ac,
                       const uint8_t *desc_bc, int32_t W, int32_t H, int32_t nc, int32_t radius, int32_t nn_l,
                       int32_t *nb_scratch, void *scratch, size_t scratch_bytes, uint64_t *nn_key,
                       int16_t *flow, uint32_t *cost, uint64_t *n_evals, void *stream);

/* Coarse-to-fine hand-over from scale 2n to scale n (Sec. 3.2): cells with
 * both grid indices even are the same pixel as a coarse cell and take its
 * flow as a seed, with the cost re-evaluated at scale n; all other cells
 * become UNSET.  desc_a, desc_b: descriptor maps of scale n;
 * coarse_flow/coarse_cost: grid of scale 2n (inputs); flow/cost: grid of
 * scale n (outputs). */
ff_status ff_seed_level(const int16_t *coarse_flow, const uint32_t *coarse_cost, const uint8_t *desc_a,
                        const uint8_t *desc_b, int32_t W, int32_t H, int32_t n, int32_t radius,
                        int16_t *flow, uint32_t *cost, uint64_t *n_evals, void *stream);

/* One propagation step (Sec. 3.1, Eq. 2) at scale n, direction
 * d = pass mod 4 (0: from left and top; 1: from right and bottom; 2: from
 * right and top; 3: from left and bottom).  Run as two checkerboard
 * half-sweeps, cells with (i+j) odd first: each cell keeps the best of its
 * own flow, its horizontal and then its vertical source cell's flow by
 * E_n (strictly lower wins; sources that are UNSET, equal to the held flow or
 * point outside the image are skipped).  desc_a, desc_b: descriptor maps of
 * scale n; flow/cost: grid of scale n, in/out. */
ff_status ff_propagate_level(const uint8_t *desc_a, const uint8_t *desc_b, int32_t W, int32_t H, int32_t n,
                             int32_t radius, int32_t pass, int16_t *flow, uint32_t *cost, uint64_t *n_evals,
                             void *stream);

/* One propagation step (Sec. 3.1, Eq. 2) at scale n in the serial order of
 * direction d = pass mod 4: rows taken from the side of the vertical source
 * cell, the cells of a row from the side of the horizontal source cell
 * (d = 0: raster order), each cell updated as in ff_propagate_level but
 * after its two source cells, whose values of this step it reads.  Same
 * result as that serial scan; the GPU sweeps anti-diagonals of 32 x 32-cell
 * tiles, one launch per tile anti-diagonal (ceil(Wn/32) + ceil(Hn/32) - 1
 * launches).  Arguments as for ff_propagate_level. */
ff_status ff_propagate_raster(const uint8_t *desc_a, const uint8_t *desc_b, int32_t W, int32_t H, int32_t n,
                              int32_t radius, int32_t pass, int16_t *flow, uint32_t *cost, uint64_t *n_evals,
                              void *stream);

/* Patch-scale change on one grid (Sec. 3.3 sub-scales): every set cell
 * (i, j) of the grid of scale n keeps its flow and gets the cost of the
 * patch of scale m, E_m(p, F) with p = (i n, j n) (patch samples p + m(u, v),
 * features of scale m); n_evals grows by the number of set cells.  desc_a,
 * desc_b: descriptor maps of scale m (ff_descriptors with n = m); flow:
 * input; cost: in/out.  n a power of two, 1 <= m <= 64. */
ff_status ff_rescore_level(const uint8_t *desc_a, const uint8_t *desc_b, int32_t W, int32_t H, int32_t n, int32_t m,
                           int32_t radius, const int16_t *flow, uint32_t *cost, uint64_t *n_evals, void *stream);

/* One random-search step (Sec. 3.1) at scale n: every set cell tries
 * F + o with o uniform on [-Rn, Rn]^2 and keeps it if E_n is strictly
 * lower; o = (0, 0) and targets outside the image are skipped.  o is drawn
 * from h = mix(seed ^ mix(ctr)), mix = SplitMix64's output mixer (Steele,
 * Lea, Flood 2014), ctr = stream_id<<56 | level<<48 | pass<<32 | j<<16 | i;
 * ox = (lo32(h) * (2Rn+1)) >> 32) - Rn, oy likewise from hi32(h) (Lemire's
 * multiply-shift).  desc_a, desc_b: descriptor maps of scale n; flow/cost:
 * grid of scale n, in/out. */
ff_status ff_random_search(const uint8_t *desc_a, const uint8_t *desc_b, int32_t W, int32_t H, int32_t n,
                           int32_t radius, int32_t Rn, uint64_t seed, int32_t stream_id, int32_t level,
                           int32_t pass, int16_t *flow, uint32_t *cost, uint64_t *n_evals, void *stream);

/* Forward-backward consistency (Sec. 3.7): keep_a[p] = 1 iff p is set in
 * field a, q = p + F_a(p) is set in field b and |F_a(p) + F_b(q)|^2 < eps^2
 * (exact integer test).  Full-resolution fields [H][W][2] / [H][W].
 * keep_b (nullable) receives the same test with the roles swapped. */
ff_status ff_consistency_filter(const int16_t *flow_a, const uint32_t *cost_a, const int16_t *flow_b,
                                const uint32_t *cost_b, int32_t W, int32_t H, float eps, uint8_t *keep_a,
                                uint8_t *keep_b, void *stream);

/* ff_consistency_filter for flows in units of 1/2^subpixel pixel
 * (subpixel in [0, 3]): q is the pixel nearest to p + F_a(p) (halves
 * rounded up) and the test is |F_a(p) + F_b(q)|^2 < (eps 2^subpixel)^2 in
 * those units; subpixel = 0 is ff_consistency_filter. */
ff_status ff_consistency_filter_sub(const int16_t *flow_a, const uint32_t *cost_a, const int16_t *flow_b,
                                    const uint32_t *cost_b, int32_t W, int32_t H, int32_t subpixel, float eps,
                                    uint8_t *keep_a, uint8_t *keep_b, void *stream);

/* The check of fields on the grid of scale n (one match per n x n region,
 * Flow Fields+ Fast x2, Sec. 3.4): cell (i, j) is pixel p = (i n, j n); its
 * target t = p + F_a is checked against the match of the region holding t,
 * cell (floor(t.x / n), floor(t.y / n)) of field b: kept iff both are set
 * and |F_a + F_b|^2 < eps^2.  Fields, costs and masks: [ceil(H/n)][ceil(W/n)]
 * (W, H: the image size); keep_b nullable (the mask of field b against
 * field a).  n = 1 is ff_consistency_filter. */
ff_status ff_consistency_filter_grid(const int16_t *flow_a, const uint32_t *cost_a, const int16_t *flow_b,
                                     const uint32_t *cost_b, int32_t W, int32_t H, int32_t n, float eps,
                                     uint8_t *keep_a, uint8_t *keep_b, void *stream);

/* Consistency against two backward fields (Sec. 3.7): keep_a[p] = 1 iff p
 * passes the ff_consistency_filter test against field b1 and against field
 * b2 (backward fields made with different generator seeds, and possibly
 * different patch radii: for instance the forward field of a second
 * ff_flow_fields call on the swapped images).  Same layouts and errors as
 * ff_consistency_filter. */
ff_status ff_consistency_filter2(const int16_t *flow_a, const uint32_t *cost_a, const int16_t *flow_b1,
                                 const uint32_t *cost_b1, const int16_t *flow_b2, const uint32_t *cost_b2, int32_t W,
                                 int32_t H, float eps, uint8_t *keep_a, void *stream);

/* Region filter (Sec. 3.7, after the consistency check): the kept pixels
 * (keep_in != 0) form regions, two 4-neighbours belonging to the same region
 * iff their flows differ by less than 3 px (|F(p) - F(q)|^2 < 9, exact); a
 * region of fewer than s pixels is deleted if one of its pixels has a
 * 4-neighbour the check removed (cost not 0xFFFFFFFF, keep_in == 0) whose
 * flow differs from its own by less than 3 px.  keep_out [H][W] (not
 * keep_in) = keep_in minus the deleted regions.  Full-resolution flow
 * [H][W][2], cost [H][W].  scratch: device, at least
 * ff_region_filter_scratch_bytes(W, H) bytes (FF_ERR_WORKSPACE otherwise),
 * 4-byte aligned (FF_ERR_ARG otherwise), contents on return unspecified;
 * s >= 0. */
size_t ff_region_filter_scratch_bytes(int32_t W, int32_t H);
ff_status ff_region_filter(const int16_t *flow, const uint32_t *cost, const uint8_t *keep_in, int32_t W, int32_t H,
                           int32_t s, void *scratch, size_t scratch_bytes, uint8_t *keep_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): the region
 * filter of ff_region_filter with no scratch argument.  Its scratch is a
 * static device array of the library, 24 MiB per GPU the library runs on,
 * held until the process ends; the call itself allocates nothing.  W * H
 * must not exceed ff_region_filter_noalloc_max_pixels() (2,097,152 pixels):
 * larger images return FF_ERR_WORKSPACE before anything is enqueued; other
 * argument errors as ff_region_filter.  Results equal ff_region_filter's.
 * All calls on one GPU share that GPU's array: calls that overlap on one GPU
 * (two streams, two threads) race and must be serialised by the caller. */
size_t ff_region_filter_noalloc_max_pixels(void);
ff_status ff_region_filter_noalloc(const int16_t *flow, const uint32_t *cost, const uint8_t *keep_in, int32_t W,
                                   int32_t H, int32_t s, uint8_t *keep_out, void *stream);

/* Sparsification (Sec. 3.8): for every q x q region of the filtered field
 * a (regions anchored at (0, 0), ragged at the right and bottom; sel is
 * int32 [ceil(H/q)][ceil(W/q)]), sel = y * W + x of the kept sample
 * (keep_a != 0) whose consistency errors |F_a(p) + F_b1(p + F_a(p))| (+ the
 * same against flow_b2, nullable) sum to the least in double precision, ties
 * to the smallest pixel index; -1 if the region holds fewer than e kept
 * samples or none whose target lies in the image.  q in [1, 64], e >= 0
 * (FF_ERR_ARG otherwise). */
ff_status ff_sparsify(const int16_t *flow_a, const uint8_t *keep_a, const int16_t *flow_b1, const int16_t *flow_b2,
                      int32_t W, int32_t H, int32_t q, int32_t e, int32_t *sel, void *stream);

/* All steps of one scale (Sec. 3.2): T propagation steps with T-1
 * random-search steps between them (RS stream `stream_id`, level index
 * `level`, n = 2^level), starting from
 *   mode 0: the state already in flow/cost, which must be consistent:
 *           every set cell's cost equals E_n of its flow (as every state
 *           the library writes is);
 *   mode 1: the coarsest-scale NN seeds (nn_key from ff_init_nn, low 32 bits
 *           = target pixel index; costs evaluated here);
 *   mode 2: seeds from the grid of scale 2n (coarse_flow/coarse_cost), as
 *           ff_seed_level.
 * Equivalent to the corresponding sequence of ff_seed_level,
 * ff_propagate_level and ff_random_search calls (same fields, same
 * evaluation count); radius 3 runs in temporally blocked launches that keep
 * the state on chip and skip evaluations whose value the consistent state
 * already fixes.  desc_a/desc_b: descriptor maps of scale n; wform_a/wform_b
 * (nullable, both or neither): weight-class row maps of scale n, which the
 * weight-class variants of the launch table need (without them those
 * variants run their descriptor-quad twins); params: host
 * (params->tuning selects the launches).  n_work: nullable device uint64
 * [2] counters of the evaluations the kernels actually compute (added to):
 * [0] those of cells the launch owns, [1] all of them, the recomputed halo
 * cells of the blocked launches included; n_evals counts the evaluations of
 * the schedule itself, of which a consistent state makes some unnecessary. */
ff_status ff_run_level(const uint8_t *desc_a, const uint8_t *desc_b, const uint8_t *wform_a, const uint8_t *wform_b,
                       int32_t W, int32_t H, int32_t level,
                       const ff_params *params, int32_t stream_id, int32_t mode, const uint64_t *nn_key,
                       const int16_t *coarse_flow, const uint32_t *coarse_cost, int16_t *flow, uint32_t *cost,
                       void *scratch, size_t scratch_bytes, uint64_t *n_evals, uint64_t *n_work, void *stream);

/* ff_run_level for both directions of a pair in one set of launches, as
 * ff_flow_fields runs a scale (Sec. 3.2: the forward and the backward field
 * are computed together): direction 0 finds image a's cells in image b
 * (desc_a/wform_a on the cell side, random-search stream id 0), direction
 * 1 the reverse (stream id 1).  nn_key, coarse_flow, coarse_cost, flow and
 * cost are host arrays of two device pointers, one per direction, with the
 * meaning of ff_run_level (nn_key only read in mode 1, the coarse grids only
 * in mode 2); n_evals: nullable device uint64 [2], one count per direction
 * (added to); n_work: nullable device uint64 [2], summed over both
 * directions.  scratch: device, at least 2 * ff_run_level_scratch_bytes.
 * Same results as two ff_run_level calls.  The temporally blocked kernels
 * only: FF_ERR_UNSUPPORTED with params->subpixel, raster or subscales, or a
 * radius the blocked kernels do not run at this size; FF_ERR_ARG for
 * invalid arguments, FF_ERR_WORKSPACE for a short scratch. */
ff_status ff_run_level_pair(const uint8_t *desc_a, const uint8_t *desc_b, const uint8_t *wform_a,
                            const uint8_t *wform_b, int32_t W, int32_t H, int32_t level, const ff_params *params,
                            int32_t mode, const uint64_t *const *nn_key, const int16_t *const *coarse_flow,
                            const uint32_t *const *coarse_cost, int16_t *const *flow, uint32_t *const *cost,
                            void *scratch, size_t scratch_bytes, uint64_t *n_evals, uint64_t *n_work, void *stream);

/* Scratch bytes of ff_run_level (host): a second grid of scale 2^level
 * (flow and cost), which the launches of a scale alternate with flow/cost
 * so that no launch reads cells it is writing.  0 for invalid sizes. */
size_t ff_run_level_scratch_bytes(int32_t W, int32_t H, int32_t level);

/* One pair of a batch (host struct; every pointer is a device pointer):
 * images [H][W]; outputs as for ff_flow_fields; keep_bwd and n_evals ([2])
 * may be NULL. */
typedef struct {
    const uint8_t *img1, *img2;
    int32_t W, H;
    int16_t *flow_fwd, *flow_bwd;
    uint32_t *cost_fwd, *cost_bwd;
    uint8_t *keep_fwd, *keep_bwd;
    uint64_t *n_evals;
} ff_pair;

/* Device workspace for a batch (host): the sum of the pairs' shares. */
size_t ff_batch_workspace_bytes(const ff_pair *pairs, int32_t npairs, const ff_params *params);

/* Bytes of the batch table (host). */
size_t ff_batch_table_bytes(int32_t npairs);

/* Writes into table_host (host memory, ff_batch_table_bytes bytes) the
 * device-side record of every pair: its buffers and its share of `ws`
 * (device address of the workspace, not dereferenced here).  The caller
 * copies the table to device memory once; it stays valid as long as the
 * pairs' buffers and `ws` do.  1 <= npairs <= 256. */
ff_status ff_batch_table(const ff_pair *pairs, int32_t npairs, const ff_params *params, void *ws,
                         size_t ws_bytes, void *table_host, size_t table_bytes);

/* Forward and backward Flow Fields plus consistency masks of every pair of a
 * batch (pairs of different sizes), each stage as one persistent launch over
 * all pairs' work items (rows, NN blocks, tiles); per pair the results are
 * those of ff_flow_fields.  pairs: host array (sizes, for the launch
 * geometry); table: device copy of ff_batch_table's output; radius must be 3
 * (FF_ERR_UNSUPPORTED otherwise).  Enqueues kernels only (capturable). */
ff_status ff_flow_fields_batched(const ff_pair *pairs, int32_t npairs, const ff_params *params,
                                 const void *table, void *ws, size_t ws_bytes, void *stream);

/* Float patch cost of learned features (Sec. 3.5 learned data term read as
 * a sum of squared differences over the subsampled patch of Eq. 3, with the
 * replicate border of Sec. 3.6):
 *   cost[e] = sum_{v,u=-r..r} sum_{c<16} (f1(clamp(p+n(u,v)))[c] - f2(clamp(p+f+n(u,v)))[c])^2
 * for entry e = (x, y, fx, fy) = pixel p and flow f (int32 [count][4]).
 * f1, f2: float32 [H][W][16]; cost: float32 [count], accumulated in
 * float32 as four partial sums s_k over the channels 4k .. 4k+3 (one fused
 * multiply-add per term, order v, u, c), returned as (s0 + s1) + (s2 + s3). */
ff_status ff_cost_f32_fwd(const float *f1, const float *f2, int32_t W, int32_t H, int32_t n, int32_t radius,
                          const int32_t *entries, int32_t count, float *cost, void *stream);

/* Gradient of sum_e grad_cost[e] * cost[e] with respect to f1 and f2
 * (d/df1 = +2 g (f1 - f2), d/df2 = -2 g (f1 - f2) at every patch position).
 * Contributions are summed in 64-bit fixed point (2^-32 units) with integer
 * atomics, so the result is deterministic.  A term |2 g (f1 - f2)| of 2^31
 * or more, or a partial sum outside the int64 range, is detected and counted in
 * the last word of acc_scratch; when that count is nonzero every value of
 * grad_f1 and grad_f2 is NaN (never a wrapped sum).  acc_scratch: int64
 * [2 * H * W * 16 + 1] scratch (cleared here); grad_f1, grad_f2: float32
 * [H][W][16] outputs (overwritten). */
ff_status ff_cost_f32_bwd(const float *f1, const float *f2, int32_t W, int32_t H, int32_t n, int32_t radius,
                          const int32_t *entries, int32_t count, const float *grad_cost, int64_t *acc_scratch,
                          float *grad_f1, float *grad_f2, void *stream);

/* Workspace bytes of ff_flow_fields_f32 (host). */
size_t ff_workspace_bytes_f32(int32_t W, int32_t H, const ff_params *params);

/* The multi-scale Flow Fields schedule (Sec. 3.2) on learned features
 * instead of the byte descriptors: feat1[l], feat2[l] (host arrays of
 * `levels` device pointers) are float32 [H][W][16] feature maps of scale
 * 2^l.  The NN seed runs on the level-1 maps of both images quantised to
 * bytes with one shared range (as ff_quantize_pair_u8) on int8 matrix cores; every other matching error is the
 * float32 squared-difference patch cost of ff_cost_f32_fwd.  Costs are
 * returned as the bit patterns of the float32 values (UNSET = 0xFFFFFFFF);
 * the rest as ff_flow_fields. */
ff_status ff_flow_fields_f32(const float *const *feat1, const float *const *feat2, int32_t W, int32_t H,
                             const ff_params *params, void *ws, size_t ws_bytes, int16_t *flow_fwd,
                             int16_t *flow_bwd, uint32_t *cost_fwd, uint32_t *cost_bwd, uint8_t *keep_fwd,
                             uint8_t *keep_bwd, uint64_t *n_evals, void *stream);

/* ---- learned descriptor network (DescNet) ---------------------------------
 * Stands in for the CNN data term the paper reports (Sec. 3.5, results in
 * Sec. 4.7): three 3x3 convolutions 1 -> 32 -> 32 -> 16, ReLU after the
 * first two, "same" zero padding.  Activations are NHWC [B][H][W][C], bf16
 * stored as uint16 bit patterns; weights [cout][9][cin] bf16, tap index
 * 3*(dy+1) + (dx+1); matrix-core products with float32 accumulation.
 * Supported (cin, cout): (1, 32), (32, 32), (32, 16), and (16, 32) for the
 * data gradient of the last layer. */

/* out[p][co] = bias[co] + sum_{tap, ci} w[co][tap][ci] * in[p + d(tap)][ci],
 * then max(0, .) if relu; written as float32 and/or bf16 (either nullable,
 * not both); bias nullable.  in must be 16-byte aligned when cin >= 16
 * (FF_ERR_ARG otherwise). */
ff_status ff_conv3x3_fwd(const uint16_t *in, int32_t B, int32_t H, int32_t W, int32_t cin, int32_t cout,
                         const uint16_t *w, const float *bias, int32_t relu, float *out_f32, uint16_t *out_bf16,
                         void *stream);

/* Gradient with respect to the input of a (cin -> cout) layer: the same
 * convolution of gout ([B][H][W][cout] bf16) with the weights rotated by 180
 * degrees and transposed (written to wflip_scratch, cin*9*cout bf16); gout
 * 16-byte aligned (FF_ERR_ARG otherwise). */
ff_status ff_conv3x3_bwd_data(const uint16_t *gout, int32_t B, int32_t H, int32_t W, int32_t cin, int32_t cout,
                              const uint16_t *w, uint16_t *wflip_scratch, float *gin_f32, uint16_t *gin_bf16,
                              void *stream);

/* Scratch bytes of ff_conv3x3_bwd_weight (host). */
size_t ff_conv3x3_wgrad_scratch_bytes(int32_t B, int32_t H, int32_t cin, int32_t cout);

/* gw[co][tap][ci] = sum_p gout[p][co] * in[p + d(tap)][ci], gbias[co] =
 * sum_p gout[p][co] (gbias nullable), float32: bf16 matrix-core products
 * with float32 accumulation, gout split into two bf16 parts (hi + lo, within
 * 2^-18 |gout| of it), so the error is at most (2^-18 + 3.1 P 2^-24) times
 * the sum of |gout| |in| over the P pixels; per-workgroup partial sums are
 * added in a fixed order (deterministic).  in: bf16, 16-byte aligned when
 * cin > 1; gout: float32, 16-byte aligned; (cin, cout) = (1, 32), (32, 32)
 * or (32, 16); FF_ERR_ARG otherwise. */
ff_status ff_conv3x3_bwd_weight(const uint16_t *in, const float *gout, int32_t B, int32_t H, int32_t W,
                                int32_t cin, int32_t cout, float *scratch, size_t scratch_bytes, float *gw,
                                float *gbias, void *stream);

/* ReLU backward: out = grad where act > 0 (act = the layer's bf16 output;
 * NULL passes grad through), written as float32 and/or bf16. */
ff_status ff_relu_bwd(const uint16_t *act, const float *grad, int64_t count, float *grad_out,
                      uint16_t *grad_out_bf16, void *stream);

/* float32 -> bf16 (round to nearest even). */
ff_status ff_f32_to_bf16(const float *x, int64_t count, uint16_t *y, void *stream);

/* Network input from image bytes: v / 255 - 0.5 as bf16. */
ff_status ff_image_to_bf16(const uint8_t *img, int64_t count, uint16_t *out, void *stream);

/* DescNet inference (Sec. 3.5, the CNN data term; the network of the
 * learned descriptor): the three 3x3 convolutions 1 -> 32 -> 32 -> 16 (ReLU
 * after the first two, "same" zero padding) and, with normalize != 0, unit
 * length per pixel (delta > 0 as in ff_l2norm16_fwd), in one launch whose
 * activations stay on chip.  The features equal those of three
 * ff_conv3x3_fwd calls (bf16 activations between the layers) and
 * ff_l2norm16_fwd bit for bit.  in: bf16 [B][H][W] network input (as
 * ff_image_to_bf16 writes it); w1 [32][9][1], w2 [32][9][32], w3
 * [16][9][32] bf16 (w2, w3 16-byte aligned); b1 [32], b2 [32], b3 [16]
 * float32; out: float32 [B][H][W][16], 16-byte aligned.  All device
 * pointers; FF_ERR_ARG for invalid arguments. */
ff_status ff_descnet_fwd(const uint16_t *in, int32_t B, int32_t H, int32_t W, const uint16_t *w1, const float *b1,
                         const uint16_t *w2, const float *b2, const uint16_t *w3, const float *b3, int32_t normalize,
                         float delta, float *out, void *stream);

/* Unit length per pixel of 16-channel float32 features [pixels][16]
 * (16-byte aligned): out = feat / sqrt(|feat|^2 + delta), delta > 0;
 * inv_norm (nullable, [pixels]) receives 1 / sqrt(|feat|^2 + delta) for the
 * backward pass.  out may alias feat. */
ff_status ff_l2norm16_fwd(const float *feat, int64_t pixels, float delta, float *out, float *inv_norm, void *stream);

/* Backward of ff_l2norm16_fwd: grad_in = inv_norm * (grad - out * <grad, out>)
 * per pixel; grad_in may alias grad. */
ff_status ff_l2norm16_bwd(const float *out, const float *inv_norm, const float *grad, int64_t pixels,
                          float *grad_in, void *stream);

/* Triplet hinge of the descriptor training (learned data term, Sec. 3.5):
 * cost: float32 [2m], the patch costs of m anchors at their positive
 * (cost[0..m)) and negative (cost[m..2m)) matches.
 * loss[0] = weight * sum_k max(0, margin + scale * (cost[k] - cost[m+k]));
 * grad_cost[k] = +weight*scale, grad_cost[m+k] = -weight*scale where the
 * hinge is active, 0 elsewhere (the input of ff_cost_f32_bwd).  The sum is
 * taken in a fixed order (deterministic). */
ff_status ff_triplet_hinge(const float *cost, int32_t m, float margin, float scale, float weight, float *grad_cost,
                           float *loss, void *stream);

/* One Adam step (Kingma and Ba 2015) on float32 parameters with bias
 * correction for step >= 1; param_bf16 (nullable) receives the bf16 copy. */
ff_status ff_adam_step(float *param, const float *grad, float *m, float *v, int32_t count, float lr,
                       float beta1, float beta2, float eps, int32_t step, uint16_t *param_bf16, void *stream);

/* Scratch bytes of ff_quantize_u8 (host). */
size_t ff_quantize_scratch_bytes(void);

/* Learned features to bytes for the matrix-core NN seed: with lo, hi the
 * minimum and maximum over all `count` values, q = clamp(rint((f - lo) *
 * (255 / (hi - lo))), 0, 255) in float32 (q = 0 if hi == lo).
 * scratch: float, ff_quantize_scratch_bytes() bytes. */
ff_status ff_quantize_u8(const float *f, int64_t count, float *scratch, uint8_t *q, void *stream);

/* The same for the two images of a pair with ONE range: lo, hi over the
 * 2 * count values of f1 and f2 together, both quantised with it, so equal
 * feature values become equal bytes in both images and the byte-space
 * nearest neighbour of the seed (Sec. 3.1) compares descriptors on one
 * scale.  q1, q2: [count] outputs. */
ff_status ff_quantize_pair_u8(const float *f1, const float *f2, int64_t count, float *scratch, uint8_t *q1,
                              uint8_t *q2, void *stream);

/* Number of variants in the launch tables (host): byte-descriptor level
 * kernels plus the step-wise schedule (the last index), and float-feature
 * level kernels (0: 16x16 cells with a halo of 2, 1: 8x8 / 2, 2: 8x8 / 4,
 * 3: 8x8 / 6, 4: 16x16 / 4). */
int32_t ff_level_variant_count(void);
int32_t ff_level_variant_count_f32(void);

/* Number of blocked launches the tables give one scale 2^log2n of a
 * schedule with `iters` propagation steps, for the byte descriptors
 * (cost_kind 0) or the float features (1); tuning NULL = the built-in table
 * (host); -1 if out of range. */
int32_t ff_level_launches(const ff_tuning *tuning, int32_t iters, int32_t log2n, int32_t cost_kind);

/* Bytes of device workspace ff_flow_fields needs for a W x H pair (host). */
size_t ff_workspace_bytes(int32_t W, int32_t H, const ff_params *params);

/* The whole hot path for one image pair (Sec. 3.2 multi-scale Flow Fields
 * and Sec. 3.7 consistency): descriptors of both images at every scale, the
 * forward field img1 -> img2 (random-search stream 0) and the backward field
 * img2 -> img1 (stream 1), each from the exact NN seed through L scales of T
 * propagation and T-1 random-search steps, then both consistency masks.
 * params: host pointer.  ws: device workspace of ff_workspace_bytes bytes.
 * flow_fwd/flow_bwd: [H][W][2]; cost_fwd/cost_bwd: [H][W];
 * keep_fwd/keep_bwd: [H][W] (keep_bwd nullable);
 * n_evals: nullable uint64 [2], evaluations per direction (overwritten).
 * Forward field only: flow_bwd, cost_bwd, keep_fwd and keep_bwd all NULL
 * (no backward field, no masks; n_evals[1] = 0); only some of them NULL is
 * FF_ERR_ARG. */
ff_status ff_flow_fields(const uint8_t *img1, const uint8_t *img2, int32_t W, int32_t H,
                         const ff_params *params, void *ws, size_t ws_bytes, int16_t *flow_fwd,
                         int16_t *flow_bwd, uint32_t *cost_fwd, uint32_t *cost_bwd, uint8_t *keep_fwd,
                         uint8_t *keep_bwd, uint64_t *n_evals, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FLOWFIELDS_H */
